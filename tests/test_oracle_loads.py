"""Oracle pins for the loading ramps (Sec. 3, eq. smooth_traction_ramp, eq. kalthoff_velocity_ramp)."""
import math

import numpy as np
import torch

import workloads as w
from oracle.loads import run_loaded, smooth_ramp, velocity_ramp
from oracle.step import Sim, initial_state


def test_smooth_ramp_values_and_smoothness():
    tr = 0.05e-6
    assert smooth_ramp(-1.0, tr) == 0.0 and smooth_ramp(0.0, tr) == 0.0
    assert smooth_ramp(tr, tr) == 1.0 and smooth_ramp(2 * tr, tr) == 1.0
    assert abs(smooth_ramp(0.5 * tr, tr) - 0.5) < 1e-15
    assert abs(smooth_ramp(0.25 * tr, tr) - (1 - math.sqrt(0.5)) / 2) < 1e-15
    h = 1e-6 * tr
    # zero slope at both ends (no load jump, no jerk jump in the load rate)
    assert abs((smooth_ramp(h, tr) - smooth_ramp(0.0, tr)) / h) < 1e-5 / tr
    assert abs((smooth_ramp(tr, tr) - smooth_ramp(tr - h, tr)) / h) < 1e-5 / tr
    ts = np.linspace(0, tr, 101)
    s = np.array([smooth_ramp(t, tr) for t in ts])
    assert np.all(np.diff(s) >= 0)
    # peak slope pi/(2 t_r) at mid-ramp
    assert abs((smooth_ramp(0.5 * tr + h, tr) - smooth_ramp(0.5 * tr - h, tr)) / (2 * h) - math.pi / (2 * tr)) < 1e-6 / tr


def test_velocity_ramp_linear_then_constant():
    tr = 1e-6
    for t, v in ((0.0, 0.0), (0.25 * tr, 0.25), (0.5 * tr, 0.5), (tr, 1.0), (3 * tr, 1.0)):
        assert abs(velocity_ramp(t, tr) - v) < 1e-15


def test_velocity_ramp_displacement_is_exact():
    """With the midpoint velocity, the prescribed DOFs move by v0 (t^2 / (2 t_r)) during the ramp."""
    p = w.small_plate(12, 6, seed=1).with_(steps=10)
    sim = Sim(p)
    tr = 8 * sim.dt
    st = run_loaded(p, 6, t_velocity=tr, sim=sim)
    t = 6 * sim.dt
    fx = np.asarray(p.fixed, dtype=bool)
    expect = np.asarray(p.v0)[fx] * t * t / (2 * tr)
    assert np.max(np.abs(st.u.numpy()[fx] - expect)) < 1e-12 * np.max(np.abs(expect))


def test_traction_ramp_scales_the_load():
    """Undamaged, no split, zero initial state: the response is linear in the load, so a
    traction ramped by S and the same traction scaled by the S values step by step agree."""
    p = w.small_plate(12, 6, seed=1, split="none").with_(steps=6)
    p = p.with_(v0=np.zeros_like(p.v0))
    sim = Sim(p)
    F = np.zeros((p.n_nodes, 2))
    F[np.asarray(p.fixed).any(1) == 0, 0] = 1e-3
    tr = 4 * sim.dt
    a = run_loaded(p, 6, traction=F, t_traction=tr, sim=sim)
    st = initial_state(p)
    for n in range(6):
        st = sim.step(st, f_ext=torch.as_tensor(F) * smooth_ramp((n + 1) * sim.dt, tr))
    assert torch.equal(a.u, st.u)
    # the first step sees S(dt) = (1 - cos(pi/4))/2 of the load
    b = run_loaded(p, 1, traction=F, t_traction=tr, sim=sim)
    a1 = sim.minv[:, None] * torch.as_tensor(F) * smooth_ramp(sim.dt, tr)
    free = ~torch.as_tensor(np.asarray(p.fixed, dtype=bool))
    assert torch.allclose(b.a[free], a1[free], rtol=1e-12, atol=0)

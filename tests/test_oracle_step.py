"""Pins of the oracle's time step, trajectory and gradient (Sec. 2.2-2.3, Sec. 4)."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.step import Sim, State, initial_state, loss_and_grad, run


def free_plate(nx=16, ny=8, split="none", seed=3):
    """Plate without loading or notch, with a smooth initial velocity field."""
    p = w.small_plate(nx, ny, jitter=0.15, seed=seed, split=split, notch=False, pull=0.0)
    p = p.with_(fixed=np.zeros_like(p.fixed))
    xy = p.xy
    Lx, Ly = xy[:, 0].max(), xy[:, 1].max()
    v0 = np.stack([0.3 * np.sin(np.pi * xy[:, 0] / Lx) * np.cos(np.pi * xy[:, 1] / Ly),
                   -0.2 * np.cos(2 * np.pi * xy[:, 0] / Lx) * np.sin(np.pi * xy[:, 1] / Ly)], 1)
    return p.with_(v0=v0)


def test_verlet_modified_energy_is_conserved():
    """P11: linear elasticity, damage frozen: 1/2 v'Mv + 1/2 u'f(u) - dt^2/8 a'Ma is invariant.

    This is the exact discrete invariant of velocity Verlet (eq. vv_u-vv_v)
    for a linear force with lumped mass, so it must hold to rounding over
    10^4 steps.
    """
    p = free_plate()
    d0 = np.random.default_rng(0).uniform(0, 0.6, p.n_nodes)
    p = p.with_(d0=d0)
    sim = Sim(p)
    st = initial_state(p)
    m = sim.mass

    def energy(s):
        _, _, _, sig = sim.stress(s.u, s.d)
        from oracle.fem import internal_force
        f = internal_force(sim.mesh, *sig)
        return float(0.5 * (m[:, None] * s.v * s.v).sum() + 0.5 * (s.u * f).sum()
                     - sim.dt ** 2 / 8 * (m[:, None] * s.a * s.a).sum())
    e0 = energy(st)
    es, plain = [], []
    for k in range(10000):
        u1, v1, a1, H1, _ = sim.explicit(st)
        st = State(u1, v1, a1, st.d, H1)
        if k % 500 == 499:
            es.append(energy(st))
            ek, ee, _ = sim.energies(st)
            plain.append(ek + ee)
    es, plain = np.array(es), np.array(plain)
    assert np.max(np.abs(es - e0)) / e0 < 1e-12
    # the plain kinetic + elastic energy moves by far more: the pin is sharp
    assert np.max(np.abs(plain - e0)) / e0 > 1e-6


@pytest.mark.parametrize("split", ["spectral", "voldev", "starconvex"])
def test_split_energy_has_no_drift(split):
    """With a split and damage frozen, E_kin + E_el stays bounded (no secular drift)."""
    p = free_plate(split=split).with_(gamma_star=1.0)
    sim = Sim(p)
    st = initial_state(p)
    tot = []
    for k in range(3000):
        u1, v1, a1, H1, psi = sim.explicit(st)
        st = State(u1, v1, a1, st.d, H1)
        if k % 100 == 99:
            ek, ee, _ = sim.energies(st)
            tot.append(ek + ee)
    tot = np.array(tot)
    first, last = tot[:10].mean(), tot[-10:].mean()
    assert abs(last - first) / first < 2e-3
    assert (tot.max() - tot.min()) / tot.mean() < 2e-2


def test_bounds_and_irreversibility():
    """P12: 0 <= d <= 1, d_{n+1} >= d_n, H_{n+1} >= H_n and the notch stays at 1."""
    p = w.config0()
    sim = Sim(p)
    st = initial_state(p)
    notch = p.d0 == 1.0
    for _ in range(40):
        new = sim.step(st)
        d0, d1 = st.d.numpy(), new.d.numpy()
        assert np.all(d1 >= d0) and np.all(d1 <= 1.0) and np.all(d1 >= 0.0)
        assert np.all(new.H.numpy() >= st.H.numpy())
        assert np.all(d1[notch] == 1.0)
        st = new
    assert st.d.numpy().max() == 1.0 and float(st.H.max()) > 0


def test_prescribed_dofs_move_with_their_velocity():
    """Prescribed DOFs keep v and zero acceleration; u grows by dt v each step."""
    p = w.small_plate(12, 6)
    st, _, sim = run(p, steps=7)
    fx = p.fixed.astype(bool)
    assert np.all(st.a.numpy()[fx] == 0.0)
    assert np.allclose(st.v.numpy()[fx], p.v0[fx], rtol=0, atol=0)
    assert np.allclose(st.u.numpy()[fx], 7 * sim.dt * p.v0[fx], rtol=1e-14, atol=0)


def test_trajectory_is_deterministic():
    p = w.small_plate(12, 6, model=1, split="voldev")
    a, _, _ = run(p, steps=15)
    b, _, _ = run(p, steps=15)
    for k in ("u", "v", "a", "d", "H"):
        assert np.array_equal(a.numpy()[k], b.numpy()[k])


@pytest.mark.parametrize("model,split", [(2, "spectral"), (1, "voldev")])
def test_forward_gradient_against_central_differences(model, split):
    """P14 (oracle side): forward-mode dL/dGc against central differences of the loss.

    The loss is piecewise smooth in Gc: the history maximum of one element
    of this run switches within a relative change of 1e-5 (Sec. 4, nonsmooth
    operations), so the difference step stays inside one smooth piece.
    """
    p = w.small_plate(20, 10, model=model, split=split, seed=5).with_(steps=40)
    sim = Sim(p)
    st, _, _ = run(p, steps=40, Gc=3.0, sim=sim)
    target = st.d.numpy()
    Gc = 2.4
    L, dL, _ = loss_and_grad(p, target, Gc, sim=sim)
    h = 1e-7 * Gc
    Lp = loss_and_grad(p, target, Gc + h, sim=sim)[0]
    Lm = loss_and_grad(p, target, Gc - h, sim=sim)[0]
    fd = (Lp - Lm) / (2 * h)
    assert L > 0 and abs(dL) > 0
    assert abs(fd - dL) / abs(dL) < 1e-5

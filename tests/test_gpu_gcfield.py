"""Spatially varying toughness Gc_e = Gc phi_e (pf_set_gc_field) against the oracle:
the damage solve, trajectories, energies and the per-element gradient dL/dGc_e."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.damage import DamageQP
from oracle.step import Sim as OSim, loss_and_field_derivative, run as orun
from tests.gpu_common import random_state, rel_err, to_oracle

pytestmark = pytest.mark.gpu


def _field(p, seed, lo=0.4, hi=2.5):
    return np.random.default_rng(seed).uniform(lo, hi, p.n_elems)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", [1, 2])
def test_field_damage_solve_matches_exact_qp(dtype, model):
    from paper_2606_23458_amd import Simulator, State
    from paper_2606_23458_amd.sim import default_tol, CgConfig
    p = w.small_plate(30, 16, jitter=0.15, seed=4, model=model, random_diag=True)
    sim = Simulator(p, dtype=dtype, tile_nodes=64, cg=CgConfig(tol=default_tol(dtype)))
    phi = _field(p, 3)
    sim.set_gc_field([phi])
    r = np.random.default_rng(5)
    H = r.uniform(0, 8000.0, p.n_elems) * (r.random(p.n_elems) < 0.5)
    lb = np.where(r.random(p.n_nodes) < 0.3, r.uniform(0, 0.9, p.n_nodes), 0.0)
    lb[p.d0 == 1.0] = 1.0
    st = {"u": np.zeros((p.n_nodes, 2)), "v": np.zeros((p.n_nodes, 2)), "a": np.zeros((p.n_nodes, 2)),
          "d": lb, "H": H}
    s_in = State.from_user(sim.mesh, [st])
    d_out = torch.zeros_like(s_in.d)
    sim.damage(s_in.H, s_in.d, d_out, sim.active)
    torch.cuda.synchronize()
    got = sim.mesh.nodes_from_internal(d_out.double())[0]
    ref = DamageQP(OSim(p).mesh, p.l0, model).solve(H, p.Gc, lb, phi)[0]
    tol = 1e-10 if dtype == "f64" else 1e-4
    assert np.max(np.abs(got - ref)) < tol, sim.cg_stats()
    # the field changes the answer: the uniform-toughness minimiser differs
    ref1 = DamageQP(OSim(p).mesh, p.l0, model).solve(H, p.Gc, lb)[0]
    assert np.max(np.abs(ref1 - ref)) > 100 * tol


def test_uniform_field_equals_no_field_bitwise():
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(40, 20, seed=5)
    a = Simulator(p, dtype="f64", tile_nodes=128)
    b = Simulator(p, dtype="f64", tile_nodes=128, dt=list(a.dt))
    b.set_gc_field([np.ones(p.n_elems)])
    a.step(15)
    b.step(15)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)
    assert a.energies() == b.energies()
    b.set_gc_field(None)
    assert b.mesh.gc_scale is None


@pytest.mark.parametrize("model,split", [(2, "spectral"), (1, "voldev")])
def test_field_trajectory_matches_oracle(model, split):
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(24, 12, jitter=0.1, seed=5, model=model, split=split)
    phi = _field(p, 8, 0.5, 1.5)
    osim = OSim(p, gc_scale=phi)
    st, _, _ = orun(p, steps=30, sim=osim)
    ref = st.numpy()
    sim = Simulator(p, dtype="f64", tile_nodes=64, dt=[osim.dt])
    sim.set_gc_field([phi])
    sim.step(30)
    torch.cuda.synchronize()
    got = sim.state.to_user()[0]
    for f in ("u", "v", "d", "H"):
        assert rel_err(got[f], ref[f]) < 1e-9, f
    e_got = sim.energies()[0]
    e_ref = osim.energies(st)
    for g, r in zip(e_got, e_ref):
        assert abs(g - r) <= 1e-10 * abs(r), (g, r)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", [1, 2])
def test_field_energies_match_oracle(dtype, model):
    from paper_2606_23458_amd import Simulator, State
    p = w.small_plate(23, 13, jitter=0.2, seed=3, model=model, random_diag=True)
    phi = _field(p, 11)
    osim = OSim(p, gc_scale=phi)
    sim = Simulator(p, dtype=dtype, tile_nodes=64, dt=[osim.dt])
    sim.set_gc_field([phi])
    st = random_state(p, seed=21)
    got = sim.energies(State.from_user(sim.mesh, [st]))[0]
    ref = osim.energies(to_oracle(st))
    tol = 1e-11 if dtype == "f64" else 2e-5
    for g, r in zip(got, ref):
        assert abs(g - r) <= tol * abs(r), (g, r)


@pytest.mark.parametrize("model,split,K", [(2, "spectral", 7), (1, "voldev", 30)])
def test_field_gradient_matches_oracle_directional_derivatives(model, split, K):
    """sum_e (dL/dGc_e) delta_e from the reverse sweep equals the oracle's forward-mode
    derivative along delta, for random directions and for delta = phi (a common scaling)."""
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import field_loss_and_grad
    p = w.small_plate(24, 12, jitter=0.1, seed=5, model=model, split=split)
    osim = OSim(p)
    target = orun(p, steps=30, sim=osim)[0].d.numpy()
    phi = _field(p, 9, 0.6, 1.4)
    sim = Simulator(p, dtype="f64", tile_nodes=64, dt=[osim.dt])
    sim.set_gc_field([phi])
    tgt = torch.tensor(sim.mesh.nodes_to_internal([target]), dtype=torch.float64, device="cuda")
    Lg, g = field_loss_and_grad(sim, tgt, steps=30, checkpoint_every=K)
    g = g[0]
    r = np.random.default_rng(12)
    for direc in (r.normal(size=p.n_elems) * p.Gc, phi * p.Gc):
        L, dL, _ = loss_and_field_derivative(p, target, p.Gc, phi, direc, steps=30, dt=osim.dt)
        assert abs(Lg[0] - L) <= 1e-9 * L
        got = float(g @ direc)
        assert abs(got - dL) <= 1e-8 * abs(dL), (got, dL)


def test_scalar_gradient_with_a_field_is_the_scaling_derivative():
    """With a field, pf_step_backward's per-instance dGc is sum_e phi_e dL/dGc_e."""
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import TrajectoryRunner, instance_mse
    p = w.small_plate(24, 12, seed=6)
    target = orun(p, steps=20)[0].d.numpy()
    phi = _field(p, 4, 0.7, 1.3)
    sim = Simulator(p, dtype="f64", tile_nodes=64)
    sim.set_gc_field([phi])
    run = TrajectoryRunner(sim, 20, 6)
    d = run.forward().d.double().clone().requires_grad_(True)
    tgt = torch.tensor(sim.mesh.nodes_to_internal([target]), dtype=torch.float64, device="cuda")
    instance_mse(sim.mesh, d, tgt).sum().backward()
    ge = torch.zeros(sim.mesh.n_elems, dtype=torch.float64, device="cuda")
    dgc = run.backward(d.grad.contiguous(), field_grad=ge)
    ge_user = sim.mesh.elems_from_internal(ge)[0]
    s = float(ge_user @ phi)
    assert abs(float(dgc[0]) - s) <= 1e-12 * abs(s)


def test_batched_fields_match_single_instances():
    """Two instances with different fields in one handle: each instance's gradient
    field equals its single-instance run's."""
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import field_loss_and_grad
    probs = [w.small_plate(20, 10, seed=s) for s in (1, 2)]
    fields = [_field(pr, 20 + k, 0.6, 1.4) for k, pr in enumerate(probs)]
    targets = [orun(pr, steps=16)[0].d.numpy() for pr in probs]
    both = Simulator(probs, dtype="f64", tile_nodes=64)
    both.set_gc_field(fields)
    tgt = torch.tensor(both.mesh.nodes_to_internal(targets), dtype=torch.float64, device="cuda")
    Lb, gb = field_loss_and_grad(both, tgt, steps=16, checkpoint_every=8)
    for k, pr in enumerate(probs):
        one = Simulator(pr, dtype="f64", tile_nodes=64, dt=[both.dt[k]])
        one.set_gc_field([fields[k]])
        t1 = torch.tensor(one.mesh.nodes_to_internal([targets[k]]), dtype=torch.float64, device="cuda")
        L1, g1 = field_loss_and_grad(one, t1, steps=16, checkpoint_every=8)
        assert abs(Lb[k] - L1[0]) <= 1e-12 * L1[0]
        assert rel_err(gb[k], g1[0]) < 1e-9


def test_bad_field_is_rejected_and_graphs_notice_a_new_field():
    from paper_2606_23458_amd import GraphStepper, Simulator
    from paper_2606_23458_amd._lib import PfError
    p = w.small_plate(20, 10, seed=2)
    sim = Simulator(p, dtype="f64")
    good = np.full(p.n_elems, 1.5)
    sim.set_gc_field([good])
    bad = good.copy()
    bad[7] = -1.0
    with pytest.raises(PfError):
        sim.set_gc_field([bad])
    bad[7] = np.nan
    with pytest.raises(PfError):
        sim.set_gc_field([bad])
    # the previous field stays in place
    assert torch.equal(sim.mesh.gc_scale.cpu(), torch.tensor(sim.mesh.elems_to_internal([good])))
    gs = GraphStepper(sim, rounds=16)
    gs.step(2)
    sim.set_gc_field([np.full(p.n_elems, 0.8)])
    with pytest.raises(RuntimeError):
        gs.step()

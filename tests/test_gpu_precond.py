"""Chebyshev-Jacobi polynomial preconditioner of the damage CG (pf_cg_opts_t.precond):
the solves reach the oracle's exact minimiser, trajectories and gradients match the
oracle, and the round-free stepping modes stay bitwise equal to polled stepping."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.damage import DamageQP
from oracle.step import Sim as OSim, loss_and_grad as oracle_loss_and_grad, run as orun
from tests.gpu_common import rel_err

pytestmark = pytest.mark.gpu


def _cg(dtype, precond, **kw):
    from paper_2606_23458_amd.sim import CgConfig, default_tol
    return CgConfig(tol=default_tol(dtype), precond=precond, **kw)


def _solve(p, dtype, precond, H, lb, monotone=0):
    from paper_2606_23458_amd import Simulator, State
    sim = Simulator(p, dtype=dtype, tile_nodes=64, cg=_cg(dtype, precond, monotone=monotone))
    st = {"u": np.zeros((p.n_nodes, 2)), "v": np.zeros((p.n_nodes, 2)), "a": np.zeros((p.n_nodes, 2)),
          "d": lb, "H": H}
    s_in = State.from_user(sim.mesh, [st])
    d_out = torch.zeros_like(s_in.d)
    sim.damage(s_in.H, s_in.d, d_out, sim.active)
    torch.cuda.synchronize()
    return sim.mesh.nodes_from_internal(d_out.double())[0], sim.cg_stats()[0]


def _problem(model, seed=5):
    p = w.small_plate(30, 16, jitter=0.15, seed=4, model=model, random_diag=True)
    r = np.random.default_rng(seed)
    H = r.uniform(0, 8000.0, p.n_elems) * (r.random(p.n_elems) < 0.5)
    lb = np.where(r.random(p.n_nodes) < 0.3, r.uniform(0, 0.9, p.n_nodes), 0.0)
    lb[p.d0 == 1.0] = 1.0
    return p, H, lb


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("model", [1, 2])
@pytest.mark.parametrize("precond", [2, 3, 4])
def test_chebyshev_solve_matches_exact_qp(dtype, model, precond):
    p, H, lb = _problem(model)
    got, st = _solve(p, dtype, precond, H, lb)
    ref = DamageQP(OSim(p).mesh, p.l0, model).solve(H, p.Gc, lb)[0]
    tol = 1e-10 if dtype == "f64" else 1e-4
    assert st["flags"] == 0, st
    assert np.max(np.abs(got - ref)) < tol, st
    assert np.all(got >= lb - (0 if dtype == "f64" else 1e-7)) and np.all(got <= 1.0)


@pytest.mark.parametrize("monotone", [0, 1])
def test_chebyshev_needs_fewer_rounds(monotone):
    """A damage solve on a larger plate: degree 3 needs fewer rounds (reductions) than Jacobi."""
    p = w.small_plate(96, 48, jitter=0.1, seed=3, model=2)
    r = np.random.default_rng(2)
    H = r.uniform(0, 3000.0, p.n_elems)
    lb = np.where(p.d0 == 1.0, 1.0, 0.0)
    d0, s0 = _solve(p, "f64", 0, H, lb, monotone)
    d3, s3 = _solve(p, "f64", 3, H, lb, monotone)
    assert s0["flags"] == 0 and s3["flags"] == 0
    assert np.max(np.abs(d0 - d3)) < 1e-10
    assert s3["iters"] < s0["iters"], (s0, s3)


def test_chebyshev_trajectory_matches_oracle():
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(24, 12, jitter=0.1, seed=5, model=2, split="spectral")
    osim = OSim(p)
    ref = orun(p, steps=30, sim=osim)[0].numpy()
    sim = Simulator(p, dtype="f64", tile_nodes=64, dt=[osim.dt], cg=_cg("f64", 3))
    sim.step(30)
    torch.cuda.synchronize()
    got = sim.state.to_user()[0]
    for f in ("u", "v", "d", "H"):
        assert rel_err(got[f], ref[f]) < 1e-9, f


def test_chebyshev_adjoint_gradient_matches_oracle():
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import loss_and_grad
    p = w.small_plate(24, 12, jitter=0.1, seed=5, model=1, split="voldev").with_(steps=30)
    osim = OSim(p)
    target = orun(p, steps=30, Gc=3.0, sim=osim)[0].d.numpy()
    L, dL, _ = oracle_loss_and_grad(p, target, 2.4, sim=osim)
    sim = Simulator(p, dtype="f64", tile_nodes=64, dt=[osim.dt], cg=_cg("f64", 2), cg_adj=_cg("f64", 4))
    tgt = torch.tensor(sim.mesh.nodes_to_internal([target]), dtype=torch.float64, device="cuda")
    Lg, g = loss_and_grad(sim, [2.4], tgt, steps=30, checkpoint_every=7)
    assert abs(Lg[0] - L) <= 1e-9 * L
    assert abs(g[0] - dL) <= 1e-8 * abs(dL), (g[0], dL)


def test_chebyshev_windowed_run_and_graphs_equal_step():
    from paper_2606_23458_amd import GraphStepper, Simulator
    p = w.small_plate(40, 20, seed=5)
    a = Simulator(p, dtype="f64", cg=_cg("f64", 3))
    b = Simulator(p, dtype="f64", dt=list(a.dt), cg=_cg("f64", 3))
    c = Simulator(p, dtype="f64", dt=list(a.dt), cg=_cg("f64", 3))
    a.step(12)
    b.run(12, window=5)
    gs = GraphStepper(c, rounds=6, more=2)   # one eager step
    gs.step(11)
    torch.cuda.synchronize()
    for s in (b, c):
        assert torch.equal(a.state.nodes, s.state.nodes) and torch.equal(a.state.H, s.state.H)
        assert torch.equal(a.active, s.active)


def test_chebyshev_batched_equals_plain_bitwise():
    from paper_2606_23458_amd import Simulator
    probs = w.config4(64)[:3]
    both = Simulator(probs, dtype="f32", cg=_cg("f32", 3))
    both.step(15)
    torch.cuda.synchronize()
    got = both.state.to_user()
    for k, pr in enumerate(probs):
        one = Simulator([pr], dtype="f32", cg=_cg("f32", 3), dt=[both.dt[k]])
        one.step(15)
        torch.cuda.synchronize()
        ref = one.state.to_user()[0]
        for f in ("u", "d", "H"):
            assert np.array_equal(got[k][f], ref[f]), (k, f)


def test_precond_out_of_range_is_rejected():
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd._lib import PfError
    p = w.small_plate(16, 8)
    sim = Simulator(p, dtype="f64", cg=_cg("f64", 5))
    with pytest.raises(PfError):
        sim.step()

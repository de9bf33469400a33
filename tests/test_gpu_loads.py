"""Ramped loads (Sec. 3 loading protocols) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.loads import run_loaded
from oracle.step import Sim as OSim
from tests.gpu_common import rel_err

pytestmark = pytest.mark.gpu


def _traction(p, amp=2e-3):
    F = np.zeros((p.n_nodes, 2))
    free = ~np.asarray(p.fixed, dtype=bool).any(1)
    F[free, 1] = amp * np.sin(np.arange(p.n_nodes))[free]
    return F


def test_ramped_loads_match_oracle():
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(32, 16, seed=3)
    osim = OSim(p)
    F = _traction(p)
    tr_f, tr_v = 6 * osim.dt, 9 * osim.dt
    ref = run_loaded(p, 20, traction=F, t_traction=tr_f, t_velocity=tr_v, sim=osim)
    sim = Simulator(p, dtype="f64", dt=[osim.dt])
    sim.set_loading(traction=F, t_traction=tr_f, t_velocity=tr_v)
    sim.step(20)
    torch.cuda.synchronize()
    got = sim.state.to_user()[0]
    for f, o in (("u", ref.u), ("v", ref.v), ("a", ref.a), ("d", ref.d), ("H", ref.H)):
        assert rel_err(got[f], o.numpy()) < 1e-9, f


def test_ramped_loads_windowed_run_and_gradient_checkpoints():
    """run() equals step() under loads, and the gradient does not depend on the checkpoint interval."""
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import loss_and_grad
    p = w.small_plate(24, 12, seed=6).with_(steps=20)
    a = Simulator(p, dtype="f64")
    b = Simulator(p, dtype="f64", dt=list(a.dt))
    F = _traction(p)
    for s in (a, b):
        s.set_loading(traction=F, t_traction=5 * a.dt[0], t_velocity=7 * a.dt[0])
    a.step(13)
    b.run(13, window=4)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)
    tgt = torch.zeros(a.mesh.n_nodes, dtype=torch.float64, device="cuda")
    out = []
    for K in (20, 6):
        s = Simulator(p, dtype="f64", dt=list(a.dt))
        s.set_loading(traction=F, t_traction=5 * a.dt[0], t_velocity=7 * a.dt[0])
        out.append(loss_and_grad(s, [2.5], tgt, steps=20, checkpoint_every=K))
    assert out[0][0][0] == out[1][0][0] and out[0][1][0] == out[1][1][0]


def test_state_time_advances_by_dt_in_fp64():
    """out.t = in.t + dt per instance, in FP64 (the time the ramps are evaluated at)."""
    from paper_2606_23458_amd import Simulator
    probs = w.config4(64)[:3]
    sim = Simulator(probs, dtype="f32")
    sim.step(7)
    torch.cuda.synchronize()
    want = np.zeros(3)
    for _ in range(7):
        want = want + np.asarray(list(sim.dt))
    assert np.array_equal(sim.state.t.cpu().numpy(), want)


def test_graph_replay_under_ramped_loads_equals_eager():
    """The ramps are evaluated on the device from the state time, so a loaded
    step replays from a HIP graph with the eager bits (every replay checked)."""
    from paper_2606_23458_amd import GraphStepper, Simulator
    p = w.small_plate(32, 16, seed=3)
    F = _traction(p)
    eager = Simulator(p, dtype="f64")
    graph = Simulator(p, dtype="f64", dt=list(eager.dt))
    for s in (eager, graph):
        s.set_loading(traction=F, t_traction=6 * eager.dt[0], t_velocity=9 * eager.dt[0])
    gs = GraphStepper(graph, rounds=32, more=8)   # takes one eager step
    eager.step()
    for k in range(14):
        eager.step()
        gs.step()
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for f in ("nodes", "H", "t"):
            assert torch.equal(getattr(eager.state, f), getattr(graph.state, f)), (k, f)


def test_loading_argument_errors():
    """Registered ramps need the state time and exclude a caller's f_ext; the
    loads are copied, so the caller's arrays may be freed."""
    import ctypes as C
    from paper_2606_23458_amd import Simulator, State
    from paper_2606_23458_amd import _lib as L
    p = w.small_plate(16, 8, seed=2)
    sim = Simulator(p, dtype="f64")
    sim.set_loading(traction=_traction(p), t_traction=3 * sim.dt[0])
    a, b = sim.state, State(sim.mesh)
    pa, pb = a.ptrs(), b.ptrs()
    pa.t = None
    st = L.lib().pf_explicit_step(sim.mesh.handle, sim.params, sim.dt, C.byref(pa), C.byref(pb), None, None)
    assert st == L.PF_ERR_ARG and "t are required" in L.lib().pf_last_error().decode()
    fe = torch.zeros(2 * sim.mesh.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PfError, match="f_ext must be NULL"):
        sim.explicit(a, b, fe)
    bad = torch.full((2, sim.mesh.n_nodes), float("nan"), dtype=torch.float64, device="cuda")
    tf = (C.c_double * 1)(1.0)
    st = L.lib().pf_set_loading(sim.mesh.handle, bad.data_ptr(), None, tf, tf, None)
    assert st == L.PF_ERR_ARG and "non-finite" in L.lib().pf_last_error().decode()
    # cleared loads: a caller's f_ext is accepted again
    sim.set_loading()
    sim.explicit(a, b, fe)
    torch.cuda.synchronize()

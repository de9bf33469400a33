"""Steps replayed from HIP graphs equal eager steps bit for bit (every replay checked)."""
import numpy as np
import pytest
import torch

import workloads as w

pytestmark = pytest.mark.gpu


def _pair(probs, dtype, rounds, more, steps, damage_chunks=0):
    from paper_2606_23458_amd import GraphStepper, Mesh, Simulator
    mesh = (lambda: Mesh(probs, dtype, 256, damage_chunks=damage_chunks)) if damage_chunks else (lambda: None)
    eager = Simulator(probs, dtype=dtype, mesh=mesh())
    graph = Simulator(probs, dtype=dtype, dt=list(eager.dt), mesh=mesh())
    gs = GraphStepper(graph, rounds=rounds, more=more)   # takes one eager step
    eager.step()
    for k in range(steps):
        eager.step()
        gs.step()
        # eager work and a synchronisation between replays
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for f in ("nodes", "H", "t"):
            a, b = getattr(eager.state, f), getattr(graph.state, f)
            assert torch.equal(a, b), (k, f)
        assert torch.equal(eager.active, graph.active), k
    return gs


def test_graph_steps_equal_eager_fp64():
    gs = _pair([w.small_plate(40, 20, seed=5)], "f64", rounds=64, more=16, steps=10)
    assert gs.continuations >= 0


def test_graph_continuation_rounds_equal_eager():
    """Tiny first graphs force several resumed continuations per step."""
    gs = _pair([w.small_plate(32, 16, seed=3)], "f64", rounds=3, more=2, steps=8)
    assert gs.continuations > 8


def test_graph_two_element_chunks_equal_eager():
    """Graph-replayed rounds and resumed continuations with the damage passes in two element chunks."""
    gs = _pair([w.small_plate(40, 20, seed=6)], "f64", rounds=5, more=3, steps=6, damage_chunks=2)
    assert gs.sim.mesh.damage_chunks == 2 and gs.continuations > 4


def test_graph_batched_fp32():
    _pair(w.config4(64)[:3], "f32", rounds=24, more=8, steps=6)


@pytest.mark.parametrize("budget", [None, 3])
def test_windowed_run_equals_step(budget):
    """run() (convergence read once per window) gives step()'s states bit for bit;
    a budget of 3 rounds forces the roll-back path."""
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(40, 20, seed=5)
    a = Simulator(p, dtype="f64")
    b = Simulator(p, dtype="f64", dt=list(a.dt))
    a.step(14)
    if budget is not None:
        b._budget = budget
    b.run(14, window=5)
    torch.cuda.synchronize()
    assert b.steps_done == 14
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)
    assert torch.equal(a.active, b.active)
    assert torch.equal(a._next.d, b._next.d)


def test_windowed_run_batched_fp32():
    from paper_2606_23458_amd import Simulator
    probs = w.config4(64)[:4]
    a = Simulator(probs, dtype="f32")
    b = Simulator(probs, dtype="f32", dt=list(a.dt))
    a.step(20)
    b.run(20, window=8)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)


@pytest.mark.parametrize("nx,ny", [(96, 48), (256, 128)])
def test_polled_solve_launches_few_rounds_past_convergence(nx, ny):
    """A polled solve enqueues as many rounds as the previous solve needed plus two, then
    polls every check_every rounds: it launches at most its own rounds + check_every + 2
    passes, also when it needs more rounds than the previous solve (here: a tighter
    tolerance after a looser one).  The 256x128 plate in 64-node tiles has more tiles than
    the pass's last workgroup combines itself, so the separate reduction launch is covered."""
    from paper_2606_23458_amd import CgConfig, Simulator
    p = w.small_plate(nx, ny, seed=3)
    sim = Simulator(p, dtype="f64", tile_nodes=64)
    sim.cg = CgConfig(tol=1e-8, check_every=2)
    sim.step(3)
    first = sim.cg_stats()[0]["iters"]
    sim.cg = CgConfig(tol=1e-13, check_every=2)
    sim.timer(True)
    for f in (1, 4):
        sim.timer_read(f)
    sim.step()
    iters = sim.cg_stats()[0]["iters"]
    _, passes = sim.timer_read(1)
    _, reductions = sim.timer_read(4)
    sim.timer(False)
    assert iters > first + 4, (first, iters)
    assert iters <= passes <= iters + 2 + 2, (first, iters, passes)
    many = sim.mesh.totals.n_tiles > 512   # more tiles than the pass's last workgroup combines
    assert reductions == (passes if many else 0), (reductions, passes, sim.mesh.totals.n_tiles)

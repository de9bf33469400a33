"""Tile-size autotuner: it times every candidate and the tuned plan computes the same step."""
import numpy as np
import pytest
import torch

import workloads as w
from tests.gpu_common import rel_err

pytestmark = pytest.mark.gpu


def test_tuner_reports_every_candidate():
    from paper_2606_23458_amd import tune_tiles
    p = w.small_plate(48, 24)
    rep = tune_tiles([p], "f64", candidates=[64, 128, 256], reps=4)
    assert rep["best"] in (64, 128, 256)
    assert [r["tile_nodes"] for r in rep["candidates"]] == [64, 128, 256]
    for r in rep["candidates"]:
        assert r["status"] == "PF_OK" and r["explicit_us"] > 0 and r["cg_round_us"] > 0, r
    best = min(rep["candidates"], key=lambda r: r["score_us"])
    assert best["tile_nodes"] == rep["best"]


def test_tuned_plan_gives_the_same_trajectory():
    """Tile plans differ only in summation order: FP64 trajectories agree to rounding."""
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(40, 20, seed=5)
    a = Simulator(p, dtype="f64", tile_nodes="auto")
    b = Simulator(p, dtype="f64", tile_nodes=64)
    assert a.dt[0] == b.dt[0]
    a.step(12)
    b.step(12)
    torch.cuda.synchronize()
    ga, gb = a.state.to_user()[0], b.state.to_user()[0]
    for f in ("u", "v", "d", "H"):
        assert rel_err(ga[f], gb[f]) < 1e-10, f


def test_tuner_batched_handle():
    from paper_2606_23458_amd import tune_tiles
    probs = w.config4(64)[:3]
    rep = tune_tiles(probs, "f32", candidates=[256, 512], reps=3)
    assert rep["best"] in (256, 512)
    assert np.all([r["score_us"] > 0 for r in rep["candidates"]])


def test_explicit_workgroup_sizes_agree_bitwise():
    """256- and 512-thread explicit-step workgroups compute the same sums in the same order."""
    from paper_2606_23458_amd import Mesh, Simulator
    p = w.small_plate(48, 24, seed=2)
    a = Simulator(p, dtype="f64", mesh=Mesh([p], "f64", 128, explicit_block=256))
    b = Simulator(p, dtype="f64", mesh=Mesh([p], "f64", 128, explicit_block=512), dt=list(a.dt))
    a.step(6)
    b.step(6)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)


@pytest.mark.parametrize("block", [256, 512])
def test_explicit_element_chunks_agree_bitwise(block):
    """One or two element chunks per workgroup add each node's corner forces in the same order."""
    from paper_2606_23458_amd import Mesh, Simulator
    p = w.small_plate(48, 24, seed=2)
    a = Simulator(p, dtype="f32", mesh=Mesh([p], "f32", 256, explicit_block=block, explicit_chunks=1))
    b = Simulator(p, dtype="f32", mesh=Mesh([p], "f32", 256, explicit_block=block, explicit_chunks=2),
                  dt=list(a.dt))
    a.step(8)
    b.step(8)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)


@pytest.mark.parametrize("dtype,tile,precond,monotone", [("f64", 256, 0, 0), ("f32", 512, 0, 0), ("f64", 512, 0, 1),
                                                         ("f32", 256, 3, 0), ("f64", 256, 3, 0)])
def test_damage_element_chunks_agree_bitwise(dtype, tile, precond, monotone):
    """One or two element chunks per damage pass add each node's corner values in the same order:
    the same bits in every pass type (set-up, restart / check, first / iterate, Chebyshev)."""
    from paper_2606_23458_amd import Mesh, Simulator
    from paper_2606_23458_amd.sim import CgConfig, default_tol
    p = w.small_plate(64, 32, seed=3)
    cg = CgConfig(tol=default_tol(dtype), precond=precond, monotone=monotone)
    ma = Mesh([p], dtype, tile, damage_chunks=1)
    mb = Mesh([p], dtype, tile, damage_chunks=2)
    assert (ma.damage_chunks, mb.damage_chunks) == (1, 2)
    a = Simulator(p, dtype=dtype, mesh=ma, cg=cg)
    b = Simulator(p, dtype=dtype, mesh=mb, dt=list(a.dt), cg=cg)
    for _ in range(10):
        a.step()
        b.step()
        assert a.cg_stats()[0]["iters"] == b.cg_stats()[0]["iters"]
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)


def test_damage_element_chunks_agree_bitwise_batched():
    """A batched handle of two plates of different sizes (fused rounds per instance): one or two
    damage element chunks give the same bits."""
    from paper_2606_23458_amd import Mesh, Simulator
    probs = [w.small_plate(64, 32, seed=3), w.small_plate(30, 14, seed=9, model=1)]
    ma = Mesh(probs, "f32", 256, damage_chunks=1)
    mb = Mesh(probs, "f32", 256, damage_chunks=2)
    a = Simulator(probs, dtype="f32", mesh=ma)
    b = Simulator(probs, dtype="f32", mesh=mb, dt=list(a.dt))
    a.step(10)
    b.step(10)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)

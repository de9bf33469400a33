"""Benchmark of the explicit phase-field hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype f64|f32] [--tile-nodes N|auto]
                    [--no-extras] [--no-cpu] [--cpu-protocol bounded|full] [--sections a,b,...]
                    [--skip-headline] [--copy-calib]

Headline: full staggered steps (explicit step + damage solve) of the
1024x512 plate (1,048,576 triangles, AT2 / vol-dev / plane strain) in FP64,
the arithmetic the paper runs its solver in, reported as element-steps per
second with inputs resident in HBM (--dtype f32 times the FP32 kernels
instead).  The same steps are timed with windowed and with polled stepping
(identical states); the faster sets the headline and both are reported.  Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average launch time (for the damage CG pass: back-to-back
                iterate passes of a solve stopped mid-iteration, with the
                in-solve figure from HIP events around each launch beside it),
                the byte basis, and the measured HBM traffic of that pass from
                the committed counter summary; also its fraction of a plain
                1 GiB device copy timed on the same box (copy_kernel);
  cpu_baseline  the FP64 CPU oracle on one pinned core: the headline plate
                (one warm-up step, two timed), the 64x32 plate in full, the
                perforated plate and four plates of the 64-plate workload
                (--cpu-protocol full: 20-step windows after 5 warm-up steps on
                the large plates);
  damage_cg     the damage CG in element-iterations per second, over the
                whole solve and for the iterate pass alone;
  fp32          the same headline in FP32 kernels (FP64 CG reductions);
  perforated    the 1448x724 perforated plate (AT1 / star-convex / plane
                stress, FP32; the same steps in FP64 under 'f64');
  batched_step  one explicit step and one staggered step of all 64 plates
                (FP32, 6.8M triangles, beyond the Infinity Cache);
  bwd_fwd       backward/forward time of the checkpointed gradient on the
                256x128 FP64 plate (500 steps, checkpoints every 50), with
                and without the checkpoint recompute;
  batched       simulations/s of one batched forward+backward evaluation of
                the 64-plate inverse workload vs the same 64 evaluations one
                plate at a time;
and, unless --no-extras: the explicit step alone, graph-replayed stepping, damage subcycling, the toughness field, the energy kernel, the
preconditioners, and the explicit step and CG pass on a 2048x1024 plate.
Tiles hold 512 owned nodes in FP32 and 448 in FP64 (--tile-nodes changes it;
'auto' lets the autotuner pick the tile size too); the autotuner picks the
explicit step's workgroup shape, the library the damage passes' element chunks.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_TILE = {"f32": 512, "f64": 448}
WIDTH = {"f32": 4, "f64": 8}
# Algorithmic bytes per element and launch (paper layout: precomputed grad phi
# and area, int32 connectivity and corner lists), per arithmetic width w.
#   explicit step: nodes 14w + 4 (u, v, a read and written, m^-1, d, row
#   pointer), elements 24 + 9w (connectivity, 6 grad phi + area, H read and
#   written, 3 corner ids); with N ~ N_e/2 that is 90 B (w = 4), 154 B (w = 8).
#   damage CG iteration pass: nodes 11w + 1 (r, A z, A p, p, x, D^-1 and the
#   held flag read; p, A p, x, r, A z written), elements 4w + 24 (the three
#   off-diagonal entries of the element stiffness, which the pass reads in
#   place of the gradients and the area, the per-solve mass coefficient,
#   connectivity, corner ids): 62.5 B (w = 4), 100.5 B (w = 8).  The restart
#   and check passes move fewer bytes; the family is costed at the iteration
#   pass, which is most of its launches.
BYTES_BASIS = {
    0: "explicit step, paper layout: nodes 14w+4 B (u, v, a read and written, 1/m, d, CSR row pointer) "
       "at N = N_e/2, elements 24+9w B (int32 connectivity, 6 grad phi + area, H read and written, "
       "3 int32 corner ids)",
    1: "damage CG iterate pass, the library's arrays costed with 32-bit indices: nodes 11w+1 B (r, Az, Ap, p, "
       "x, 1/diag and the held flag read; p, Ap, x, r, Az written) at N = N_e/2, elements 4w+24 B "
       "(3 stiffness off-diagonals, the mass coefficient, connectivity, corner ids); intermediates "
       "kept in LDS are not counted",
}


def alg_bytes_per_elem(family: int, w: int) -> float:
    if family == 0:
        return (14 * w + 4) / 2 + 24 + 9 * w
    if family == 1:
        return (11 * w + 1) / 2 + 4 * w + 24
    raise ValueError(family)


FAMILY = {0: "k_explicit", 1: "k_dmg (damage CG pass)", 2: "k_dmg_init / k_dmg_final", 3: "adjoint",
          4: "k_dmg_red (per-instance CG reductions)"}


def gpu_sync():
    import torch
    torch.cuda.synchronize()


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def plate_simulator(p, tile_nodes, dtype: str):
    """A Simulator of plate p (or of a list of plates in one handle): tile_nodes 'auto' lets
    the autotuner pick the whole plan; a number fixes the tile size and the autotuner picks
    only the explicit-step workgroup shape (so repeated runs and profiles use the same tiles)."""
    from paper_2606_23458_amd import Mesh, Simulator, tune_tiles
    probs = list(p) if isinstance(p, (list, tuple)) else [p]
    if tile_nodes == "auto":
        return Simulator(probs, dtype=dtype, tile_nodes="auto")
    rep = tune_tiles(probs, dtype, candidates=[int(tile_nodes)])
    mesh = Mesh(probs, dtype, int(tile_nodes), explicit_block=rep["explicit_block"],
                explicit_chunks=rep["explicit_chunks"])
    return Simulator(probs, dtype=dtype, mesh=mesh)


def timed_run(sim, steps: int) -> float:
    """ms per step of sim.run(steps) (convergence read once per window)."""
    gpu_sync()
    ev0, ev1 = events()
    ev0.record()
    sim.run(steps)
    ev1.record()
    gpu_sync()
    return ev0.elapsed_time(ev1) / steps


def timed_step(sim, steps: int) -> float:
    """ms per step of sim.step(steps) (convergence polled inside every solve)."""
    gpu_sync()
    ev0, ev1 = events()
    ev0.record()
    sim.step(steps)
    ev1.record()
    gpu_sync()
    return ev0.elapsed_time(ev1) / steps


def run_headline(p, dtype: str, steps: int, warmup: int, tile_nodes):
    """The same steps (warmup + 1 .. warmup + steps) timed in both stepping modes, each on a
    fresh simulator: windowed (Simulator.run) and polled (Simulator.step).  Both give the same
    states bit for bit; the faster sets the headline."""
    polled = plate_simulator(p, tile_nodes, dtype)
    polled.step(warmup)
    ms_step = timed_step(polled, steps)
    del polled
    sim = plate_simulator(p, tile_nodes, dtype)
    ne = sim.mesh.n_elems
    sim.run(warmup)
    gpu_sync()
    t0 = time.perf_counter()
    ms_run = timed_run(sim, steps)
    wall = time.perf_counter() - t0
    mode = "windowed" if ms_run <= ms_step else "polled"
    ms = min(ms_run, ms_step) * steps
    # second pass with per-kernel events for the roofline; the solver polls
    # after every round, so every timed damage launch does work
    sim.timer(True)
    for f in range(5):
        sim.timer_read(f)
    iters = []
    cg = sim.cg
    sim.cg = type(cg)(cg.tol, cg.max_iter, 1, cg.start, cg.monotone)
    for _ in range(steps):
        sim.step()
        iters.append(sim.cg_stats()[0]["iters"])
    gpu_sync()
    fam = {f: sim.timer_read(f) for f in (0, 1, 2, 4)}
    sim.timer(False)
    sim.cg = cg
    return {"sim": sim, "ne": ne, "ms": ms, "wall": wall, "fam": fam, "iters": iters, "problem": p,
            "dtype": dtype, "mode": mode, "ms_run": ms_run, "ms_step": ms_step}


def explicit_only(sim, steps: int, w: int) -> dict:
    """The explicit step alone (ping-pong between two states), same plate and tile plan."""
    from paper_2606_23458_amd import State
    a, b = sim.state.clone(), State(sim.mesh)
    b.d.copy_(a.d)
    for _ in range(5):
        sim.explicit(a, b)
        a, b = b, a
    gpu_sync()
    ev0, ev1 = events()
    ev0.record()
    for _ in range(steps):
        sim.explicit(a, b)
        a, b = b, a
    ev1.record()
    gpu_sync()
    ms = ev0.elapsed_time(ev1) / steps
    ne = sim.mesh.n_elems
    gbs = alg_bytes_per_elem(0, w) * ne / (ms / 1e3) / 1e9
    return {"elem_steps_per_s": round(ne / (ms / 1e3), 1), "us_per_step": round(ms * 1e3, 2),
            "alg_GBps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "alg_bytes_per_elem": alg_bytes_per_elem(0, w),
            "note": "explicit step only (predictor, strain, split, force gather, corrector, history), "
                    "back-to-back launches incl. launch gaps"}


def graph_steps(steps: int, tile_nodes, dtype: str) -> dict:
    """The same staggered steps replayed from HIP graphs (GraphStepper)."""
    import workloads as w
    from paper_2606_23458_amd import GraphStepper
    sim = plate_simulator(w.config1().with_(dtype=dtype), tile_nodes, dtype)
    sim.step(20)
    gs = GraphStepper(sim)
    gs.step(5)
    gpu_sync()
    c0 = gs.continuations
    ev0, ev1 = events()
    ev0.record()
    gs.step(steps)
    ev1.record()
    gpu_sync()
    ms = ev0.elapsed_time(ev1) / steps
    return {"elem_steps_per_s": round(sim.mesh.n_elems / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
            "continuations_per_step": round((gs.continuations - c0) / steps, 3),
            "note": f"explicit step + first {gs.rounds} CG rounds in one graph, {gs.more}-round continuation "
                    "graphs as needed"}


def traffic_summary(dtype: str) -> str:
    return os.path.join(ROOT, "profiles", "k_dmg_c1_traffic.md" if dtype == "f32" else "k_dmg_c1_f64_traffic.md")


KERNEL_SOURCES = ["damage.hip", "device_common.hpp", "pf_internal.hpp"]


def measured_traffic(dtype: str):
    """Bytes per damage CG pass from the committed counter summary, if the kernel is unchanged since."""
    import hashlib
    try:
        text = open(traffic_summary(dtype)).read()
    except OSError:
        return None
    fields = dict(l.split(":", 1) for l in text.splitlines() if l.startswith(("traffic_bytes_per_pass:",
                                                                              "sources_sha256:")))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2606_23458_amd", "csrc", f), "rb").read())
    if fields.get("sources_sha256", "").strip() != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_pass"])


def damage_pass_b2b(sim, passes: int = 100, reps: int = 3) -> float | None:
    """Mean time (s) of one damage CG iterate pass, launched back to back.

    The simulator's next solve is stopped after five rounds (set-up, first
    pass, three iterations) and pf_damage_pass_repeat then launches that
    iterate pass `passes` times with no reduction in between; HIP events on
    the library's stream bracket each batch.  Every launch reads and writes
    the bytes of one iterate pass.  This is the last use of that simulator.
    """
    from paper_2606_23458_amd import CgConfig
    from paper_2606_23458_amd import _lib as L
    c = sim.cg
    cg = CgConfig(c.tol, c.max_iter, 0, c.start, c.monotone, 5, 0, 0)
    for _ in range(5):
        sim.explicit(sim.state, sim._next)
        sim.damage(sim._next.H, sim.state.d, sim._next.d, sim._active_next, sim.active, cg=cg)
        arrays = (sim._next.H, sim.state.d, sim._next.d)
        try:
            sim.repeat_damage_pass(10, *arrays)   # warm-up; refused unless the solve stopped in a CG iteration
            break
        except L.PfError:
            sim.step()
    else:
        return None
    gpu_sync()
    ts = []
    for _ in range(reps):
        ev0, ev1 = events()
        ev0.record()
        sim.repeat_damage_pass(passes, *arrays)
        ev1.record()
        gpu_sync()
        ts.append(ev0.elapsed_time(ev1) / passes / 1e3)
    return sum(ts) / len(ts)


def copy_bandwidth(mib: int = 1024, reps: int = 10) -> dict:
    """A plain device-to-device copy (the runtime's copy kernel) of `mib` MiB, beyond the
    Infinity Cache, timed with HIP events over `reps` copies: what a streaming kernel reaches on
    this box, beside the 8 TB/s specification."""
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    ev0, ev1 = events()
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    gpu_sync()
    t = ev0.elapsed_time(ev1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return {"MiB": mib, "bytes_per_copy": 2 * n, "GBps": round(2 * n / t / 1e9, 1), "reps": reps}


def roofline(res) -> dict:
    ne = res["ne"]
    w = WIDTH[res["dtype"]]
    fam = res["fam"]
    dom = max((f for f in fam if f in (0, 1)), key=lambda f: fam[f][0])
    tot_ms, launches = fam[dom]
    # the damage CG passes that did work: the solver's pass counts (launches
    # after a solve has finished exit at once; their time stays in tot_ms)
    work = sum(res["iters"]) if dom == 1 else launches
    ev_s = tot_ms / max(work, 1) / 1e3
    # the launch time: back-to-back iterate passes when measured (events around
    # every launch inside the solve add their own gaps), else the in-solve figure
    b2b = res.get("b2b_s") if dom == 1 else None
    avg_s = b2b if b2b else ev_s
    bytes_per_launch = alg_bytes_per_elem(dom, w) * ne
    achieved = bytes_per_launch / avg_s / 1e9
    traffic = measured_traffic(res["dtype"]) if dom == 1 else None
    out = {"bound": "hbm", "kernel": FAMILY[dom], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "alg_bytes_basis": f"{alg_bytes_per_elem(dom, w)} B per element x {ne} elements per launch; "
                              + BYTES_BASIS[dom],
           "alg_bytes_per_launch": int(bytes_per_launch),
           "measured_GBps": round(traffic / avg_s / 1e9, 1) if traffic else None,
           "avg_launch_us": round(avg_s * 1e6, 2),
           "timed_as": ("100 back-to-back iterate passes of a solve stopped mid-iteration, 3 batches"
                        if b2b else "HIP events around every launch inside the solves"),
           "in_solve_events_us": round(ev_s * 1e6, 2), "launches": launches, "passes_with_work": work}
    out["per_kernel_us"] = {FAMILY[f]: round(fam[f][0] / max(fam[f][1], 1) * 1e3, 2) for f in fam}
    out["share"] = {FAMILY[f]: round(fam[f][0] / sum(v[0] for v in fam.values()), 3) for f in fam}
    return out


def damage_cg_rates(res, hb: dict, explicit_us: float, pass_us: float) -> dict:
    """Damage CG throughput in element-iterations per second (one iteration = one round: a pass
    over the plate and its reduction): over the whole solve (rounds per step over the step time
    less the explicit step alone), and for the iterate pass alone (back to back)."""
    ne = res["ne"]
    rounds = hb["cg_iters_per_solve"]["mean"]
    solve_s = (hb["ms_per_step"] - explicit_us / 1e3) / 1e3
    return {"elem_iterations_per_s": round(ne * rounds / solve_s, 1),
            "pass_elem_iterations_per_s": round(ne / (pass_us / 1e6), 1),
            "rounds_per_solve": rounds, "us_per_round": round(solve_s / rounds * 1e6, 2),
            "basis": "rounds per solve x elements / (step time - explicit step alone); the pass alone: "
                     "elements / back-to-back iterate pass time"}


def headline_block(res, steps: int) -> dict:
    """value, time per step and CG counts of a run_headline result."""
    ne = res["ne"]
    it = res["iters"]
    return {"value": round(ne * steps / (res["ms"] / 1e3), 1), "ms_per_step": round(res["ms"] / steps, 4),
            "cg_iters_per_solve": {"mean": round(sum(it) / len(it), 2), "max": max(it)},
            "stepping": {"timed": res["mode"], "windowed_ms_per_step": round(res["ms_run"], 4),
                         "polled_ms_per_step": round(res["ms_step"], 4)}}


def fp32_companion(steps: int, warmup: int, tile_nodes) -> dict:
    """The headline plate in FP32 kernels (FP64 CG reductions), with its own roofline figures."""
    import workloads as w
    res = run_headline(w.config1(), "f32", steps, warmup, DEFAULT_TILE["f32"] if tile_nodes is None else tile_nodes)
    out = {"unit": "elem-steps/s", "dtype": "f32", **headline_block(res, steps)}
    out["explicit_step"] = explicit_only(res["sim"], steps, 4)
    res["b2b_s"] = damage_pass_b2b(res["sim"])
    rf = roofline(res)
    out["roofline"] = {k: rf[k] for k in ("kernel", "achieved", "frac", "traffic", "measured_GBps",
                                          "avg_launch_us", "alg_bytes_per_launch", "in_solve_events_us")}
    out["damage_cg"] = damage_cg_rates(res, out, out["explicit_step"]["us_per_step"], rf["avg_launch_us"])
    out["tile_nodes"] = res["sim"].mesh.tile_nodes
    return out


def perforated(steps: int = 60, warmup: int = 20) -> dict:
    """The perforated plate (2.09M triangles, random diagonals, six holes; AT1 / star-convex / plane
    stress, FP32 as configured): staggered steps and the explicit step alone; the same steps again
    in FP64 (the paper's arithmetic) under 'f64'."""
    import workloads as w

    def one(dtype: str) -> dict:
        p = w.config2().with_(dtype=dtype)
        sim = plate_simulator(p, DEFAULT_TILE[dtype], dtype)
        ne = sim.mesh.n_elems
        sim.run(warmup)
        ms = timed_run(sim, steps)
        it = []
        for _ in range(10):
            sim.step()
            it.append(sim.cg_stats()[0]["iters"])
        return {"workload": f"1448x724 perforated plate, {ne} triangles, {sim.mesh.n_nodes} nodes, AT1 / "
                            f"star-convex / plane stress, {dtype.upper()}, steps {warmup + 1}-{warmup + steps}",
                "elem_steps_per_s": round(ne / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                "cg_iters_per_solve": round(sum(it) / len(it), 2),
                "explicit_step": explicit_only(sim, 40, WIDTH[dtype]),
                "tile_plan": {"tile_nodes": sim.mesh.tile_nodes, "damage_chunks": sim.mesh.damage_chunks,
                              "n_tiles": int(sim.mesh.totals.n_tiles)}}

    out = one("f32")
    gpu_sync()
    out["f64"] = one("f64")
    return out


def batched_step(steps: int = 30) -> dict:
    """All 64 plates of the inverse workload in one handle (FP32, 6.8M triangles): the explicit
    step alone (612 MB of algorithmic traffic per step, beyond the 256 MB Infinity Cache) and
    full staggered steps."""
    import workloads as w
    probs = w.config4(64)
    sim = plate_simulator(probs, DEFAULT_TILE["f32"], "f32")
    ne = sim.mesh.n_elems
    sim.run(10)
    ms = timed_run(sim, steps)
    ex = explicit_only(sim, steps, 4)
    return {"workload": f"64 plates 128x64..512x256, {ne} triangles, FP32, one handle",
            "tile_plan": {"tile_nodes": sim.mesh.tile_nodes, "explicit_block": sim.mesh.explicit_block,
                          "explicit_chunks": sim.mesh.explicit_chunks, "damage_chunks": sim.mesh.damage_chunks},
            "explicit_step": ex,
            "alg_MB_per_explicit_step": round(alg_bytes_per_elem(0, 4) * ne / 1e6, 1),
            "staggered_ms_per_step": round(ms, 4), "elem_steps_per_s": round(ne / (ms / 1e3), 1)}


def subcycling(steps: int) -> dict:
    """Damage subcycling at N_sub = N_max on the 1024x512 plate (FP32): time per step against every-step solves."""
    import workloads as w
    from paper_2606_23458_amd import Simulator
    p = w.config1()
    a = Simulator(p, dtype="f32")
    nmax = min(a.n_max)
    b = Simulator(p, dtype="f32", n_sub=nmax, dt=list(a.dt))
    out = {"n_sub": nmax, "c_p_over_0.6c_R": round(min(a.subcycle_ratio), 3)}
    for key, sim in (("every_step", a), ("subcycled", b)):
        sim.run(20)
        out[key + "_ms_per_step"] = round(timed_run(sim, steps), 4)
    out["saving"] = round(1.0 - out["subcycled_ms_per_step"] / out["every_step_ms_per_step"], 3)
    return out


def gc_field(steps: int) -> dict:
    """Toughness field Gc_e = Gc phi_e (phi ~ U[0.5, 1.5] per element) on the 1024x512 plate (FP32)
    against a uniform Gc, and the per-element gradient's reverse sweep against the scalar one
    (256x128, FP64)."""
    import numpy as np
    import torch
    import workloads as w
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import TrajectoryRunner
    p = w.config1()
    phi = np.random.default_rng(17).uniform(0.5, 1.5, p.n_elems)
    a = Simulator(p, dtype="f32")
    b = Simulator(p, dtype="f32", dt=list(a.dt))
    b.set_gc_field([phi])
    out = {}
    for key, sim in (("uniform", a), ("field", b)):
        sim.run(20)
        ms = timed_run(sim, steps)
        out[key + "_ms_per_step"] = round(ms, 4)
        out[key + "_elem_steps_per_s"] = round(p.n_elems / (ms / 1e3), 1)
    p3 = w.config3().with_(steps=100)
    phi3 = np.random.default_rng(18).uniform(0.5, 1.5, p3.n_elems)
    sim = Simulator(p3, dtype="f64")
    sim.set_gc_field([phi3])
    run = TrajectoryRunner(sim, steps=100, checkpoint_every=25)
    run.forward()
    dbar = (sim.state.d * (2.0 / sim.mesh.n_nodes)).contiguous()
    ge = torch.zeros(sim.mesh.n_elems, dtype=torch.float64, device="cuda")
    times = {}
    for key, fg in (("scalar", None), ("per_element", ge)):
        gpu_sync()
        t0 = time.perf_counter()
        run.backward(dbar, field_grad=fg)
        gpu_sync()
        times[key] = time.perf_counter() - t0
    out["bwd_workload"] = "256x128 plate, FP64, 100 steps, checkpoint every 25"
    out["bwd_scalar_s"] = round(times["scalar"], 3)
    out["bwd_per_element_s"] = round(times["per_element"], 3)
    return out


def preconditioners(steps: int) -> dict:
    """Jacobi against the Chebyshev-Jacobi polynomials of degree 2-4 on the 1024x512 plate (FP32):
    time per step and CG rounds (one reduction each) per solve."""
    import workloads as w
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.sim import CgConfig, default_tol
    p = w.config1()
    out = {}
    dt = None
    for deg in (0, 2, 3, 4):
        sim = Simulator(p, dtype="f32", dt=dt, cg=CgConfig(tol=default_tol("f32"), precond=deg))
        dt = list(sim.dt)
        sim.run(20)
        gpu_sync()
        ev0, ev1 = events()
        rounds = []
        ev0.record()
        for _ in range(steps):
            sim.step()
            rounds.append(sim.cg_stats()[0]["iters"])
        ev1.record()
        gpu_sync()
        mean = sum(rounds) / len(rounds)
        out["jacobi" if deg == 0 else f"chebyshev{deg}"] = {
            "ms_per_step": round(ev0.elapsed_time(ev1) / steps, 4), "rounds_per_solve": round(mean, 2)}
    out["note"] = ("polled steps (Simulator.step); a round is one reduction and, with a degree-k "
                   "polynomial, k passes (restart and check rounds make one)")
    return out


def beyond_cache(steps: int = 40) -> dict:
    """The explicit step and the damage CG passes on a 2048x1024 plate (4.2M triangles, FP32,
    the 1024x512 plate's physics): 378 MB per explicit step and ~262 MB per CG pass exceed the
    256 MB Infinity Cache, so these rates are HBM rates."""
    import workloads as w
    from paper_2606_23458_amd import Simulator
    p = w.plate_problem("c1x4", 2048, 1024, 0.10, 1, model=2, split="voldev", plane="strain", dtype="f32")
    sim = Simulator(p, dtype="f32", tile_nodes="auto")
    ne = sim.mesh.n_elems
    sim.run(20)
    ex = explicit_only(sim, steps, 4)
    # full steps with per-pass events
    sim.timer(True)
    for f in range(5):
        sim.timer_read(f)
    cg = sim.cg
    sim.cg = type(cg)(cg.tol, cg.max_iter, 1, cg.start, cg.monotone)
    passes = 0
    ev0, ev1 = events()
    ev0.record()
    for _ in range(steps):
        sim.step()
        passes += sim.cg_stats()[0]["iters"]
    ev1.record()
    gpu_sync()
    ms1, _ = sim.timer_read(1)
    sim.timer(False)
    sim.cg = cg
    pass_us = ms1 / max(passes, 1) * 1e3
    gb_cg = alg_bytes_per_elem(1, 4) * ne / (pass_us * 1e-6) / 1e9
    return {"workload": f"2048x1024 plate, {ne} triangles, FP32", "tile_nodes": sim.mesh.tile_nodes,
            "explicit_us": ex["us_per_step"], "explicit_alg_GBps": ex["alg_GBps"],
            "explicit_frac_hbm_peak": ex["frac_hbm_peak"],
            "cg_pass_us": round(pass_us, 2), "cg_pass_alg_GBps": round(gb_cg, 1),
            "cg_pass_frac_hbm_peak": round(gb_cg / HBM_PEAK_GBS, 4),
            "ms_per_step_polled": round(ev0.elapsed_time(ev1) / steps, 4)}


def energies_cost(reps: int = 50) -> dict:
    """pf_energies on the 1024x512 plate (FP32): time per call."""
    import workloads as w
    from paper_2606_23458_amd import Simulator
    sim = Simulator(w.config1(), dtype="f32")
    sim.run(50)
    gpu_sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        sim.energies()
    gpu_sync()
    return {"us_per_call_incl_readback": round((time.perf_counter() - t0) / reps * 1e6, 1)}


def bwd_fwd_ratio() -> dict:
    import torch
    import workloads as w
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import TrajectoryRunner

    p = w.config3()
    sim = Simulator(p, dtype="f64")
    runner = TrajectoryRunner(sim, steps=p.steps, checkpoint_every=50)
    runner.forward()
    gpu_sync()
    t0 = time.perf_counter()
    runner.forward()
    gpu_sync()
    t_fwd = time.perf_counter() - t0
    dbar = torch.zeros(sim.mesh.n_nodes, dtype=torch.float64, device="cuda")
    dbar.copy_(sim.state.d * (2.0 / sim.mesh.n_nodes))
    tm = {}
    t0 = time.perf_counter()
    runner.backward(dbar, timing=tm)
    gpu_sync()
    t_bwd = time.perf_counter() - t0
    return {"workload": "256x128 plate, FP64, AT2/spectral/plane strain, 500 steps, checkpoint every 50",
            "fwd_s": round(t_fwd, 3), "bwd_s": round(t_bwd, 3), "ratio": round(t_bwd / t_fwd, 3),
            "recompute_s": round(tm["recompute"], 3), "adjoint_s": round(tm["adjoint"], 3),
            "ratio_without_recompute": round(tm["adjoint"] / t_fwd, 3),
            "note": "bwd includes the checkpoint recompute; ratio_without_recompute counts the adjoint steps only"}


def batched_vs_plain(n_inst: int = 64, steps: int = 300, plain: bool = True) -> dict:
    import workloads as w
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.grad import TrajectoryRunner

    probs = w.config4(n_inst)
    # batched: one handle, one forward + backward of all instances (explicit-step shape by the autotuner)
    sim = plate_simulator(probs, DEFAULT_TILE["f32"], "f32")
    runner = TrajectoryRunner(sim, steps=steps, checkpoint_every=50)
    gpu_sync()
    t0 = time.perf_counter()
    runner.forward()
    t_f = time.perf_counter() - t0
    dbar = sim.state.d * 1e-3
    tm = {}
    runner.backward(dbar, timing=tm)
    gpu_sync()
    t_b = time.perf_counter() - t0
    ne = sum(p.n_elems for p in probs)
    if not plain:
        return {"workload": f"{n_inst} plates 128x64..512x256 ({ne} triangles), FP32, {steps} steps fwd+bwd, "
                            "one batched handle", "batched_sims_per_s": round(n_inst / t_b, 3),
                "batched_bwd_over_fwd": round((t_b - t_f) / t_f, 3),
                "batched_bwd_over_fwd_without_recompute": round(tm["adjoint"] / t_f, 3)}
    # plain: the same evaluations one instance at a time
    t_p = 0.0
    for pr in probs:
        s1 = Simulator([pr], dtype="f32")
        r1 = TrajectoryRunner(s1, steps=steps, checkpoint_every=50)
        gpu_sync()
        t0 = time.perf_counter()
        r1.forward()
        r1.backward(s1.state.d * 1e-3)
        gpu_sync()
        t_p += time.perf_counter() - t0
        del r1, s1
    return {"workload": f"{n_inst} plates 128x64..512x256 ({ne} triangles), FP32, {steps} steps fwd+bwd",
            "batched_sims_per_s": round(n_inst / t_b, 3), "plain_sims_per_s": round(n_inst / t_p, 3),
            "speedup": round(t_p / t_b, 3), "batched_bwd_over_fwd": round((t_b - t_f) / t_f, 3),
            "batched_bwd_over_fwd_without_recompute": round(tm["adjoint"] / t_f, 3)}


# --------------------------------------------------------------------------- CPU oracle baseline
def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(problem, warm: int, timed: int) -> dict:
    from oracle.step import Sim, initial_state
    sim = Sim(problem)
    st = initial_state(problem)
    for _ in range(warm):
        st = sim.step(st)
    t0 = time.perf_counter()
    for _ in range(timed):
        st = sim.step(st)
    dt = time.perf_counter() - t0
    return {"elem_steps_per_s": round(problem.n_elems * timed / dt, 1), "seconds": round(dt, 2),
            "warm_up_steps": warm, "timed_steps": timed}


def cpu_baseline(protocol: str = "bounded") -> dict:
    """The FP64 oracle (sparse-LU damage QP) on one core of this host, pinned in-process."""
    import torch
    import workloads as w
    nproc = os.cpu_count()
    aff = os.sched_getaffinity(0)
    core = min(aff)
    threads = torch.get_num_threads()
    limiter = None
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    os.sched_setaffinity(0, {core})
    torch.set_num_threads(1)
    try:
        big = (5, 20) if protocol == "full" else (1, 2)
        c1 = _oracle_rate(w.config1(), *big)
        rows = {"1024x512 plate (headline)": c1}
        c0 = w.config0()
        rows["64x32 plate, all 200 steps"] = _oracle_rate(c0, 0, c0.steps)
        rows["1448x724 perforated plate"] = _oracle_rate(w.config2(), *big)
        sub = w.config4(64)[:4]
        rs = [_oracle_rate(pr, 5, 20) for pr in sub]
        ne = sum(p.n_elems for p in sub)
        rows["4 plates of the 64-plate workload, 5 + 20 steps each"] = {
            "elem_steps_per_s": round(ne * 20 / sum(r["seconds"] for r in rs), 1),
            "seconds": round(sum(r["seconds"] for r in rs), 2)}
    finally:
        os.sched_setaffinity(0, aff)
        torch.set_num_threads(threads)
        if limiter is not None and hasattr(limiter, "unregister"):
            limiter.unregister()
    return {"value": c1["elem_steps_per_s"], "unit": "elem-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"staggered steps (explicit step + exact damage QP by sparse LU) of the 1024x512 plate, FP64, "
                      f"{c1['warm_up_steps']} warm-up step(s) then {c1['timed_steps']} timed ({c1['seconds']} s), "
                      f"one pinned core",
            "host": {"cpu_model": _cpu_model(), "nproc": nproc, "pinned_core": core}, "protocol": protocol,
            "workloads": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"],
                    help="arithmetic of the headline (FP64 is the paper's)")
    ap.add_argument("--tile-nodes", default=None,
                    help="owned nodes per tile (the autotuner then picks the explicit-step workgroup shape), "
                         "or 'auto' (the autotuner picks the whole plan); default 512 (FP32), 448 (FP64)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-protocol", default="bounded", choices=["bounded", "full"])
    ap.add_argument("--sections", default=None,
                    help="comma-separated extra sections to run (default: all; names as on the JSON line), "
                         "e.g. bwd_fwd,batched to profile the backward")
    ap.add_argument("--skip-headline", action="store_true",
                    help="profiling aid: run only the --sections bwd_fwd, batched, batched_bwd (the batched "
                         "forward+backward without the one-plate-at-a-time loop) or perforated, and print their "
                         "results")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also copy a 256 MiB device buffer 3 times (known traffic, for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (the sharded layout is a "
                                   "design only)"}))
        sys.exit(2)
    tile = args.tile_nodes
    if tile is None:
        tile = DEFAULT_TILE[args.dtype]
    elif tile != "auto":
        tile = int(tile)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.copy_calib:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    if args.skip_headline:
        extra = {"bwd_fwd": bwd_fwd_ratio, "batched": batched_vs_plain,
                 "batched_bwd": lambda: batched_vs_plain(plain=False), "perforated": perforated}
        out = {k: extra[k]() for k in (args.sections or "").split(",") if k in extra}
        print(json.dumps(out))
        return
    import workloads as w
    p = w.config1().with_(dtype=args.dtype)
    res = run_headline(p, args.dtype, args.steps, args.warmup, tile)
    print("[bench] headline done", file=sys.stderr, flush=True)
    sim = res["sim"]
    hb = headline_block(res, args.steps)
    prec = "fp64 throughout" if args.dtype == "f64" else "fp32 kernels, fp64 CG reductions"
    out = {
        "metric": "elem-steps/s and % HBM peak; batched vs plain sims/s; bwd/fwd time ratio",
        "value": hb["value"], "unit": "elem-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hb["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "1024x512 jittered plate, 1048576 triangles, AT2 / vol-dev / plane strain, "
                               "full staggered step (explicit + projected-CG damage solve)",
                   "n_elems": res["ne"], "n_nodes": sim.mesh.n_nodes, "precision": prec,
                   "tile_plan": {"tile_nodes": sim.mesh.tile_nodes, "explicit_block": sim.mesh.explicit_block,
                                 "explicit_chunks": sim.mesh.explicit_chunks,
                                 "damage_chunks": sim.mesh.damage_chunks,
                                 "n_tiles": int(sim.mesh.totals.n_tiles),
                                 "chosen_by": "autotuner" if tile == "auto"
                                 else "tile size fixed, workgroup shape by the autotuner, damage element "
                                      "chunks by the library"},
                   "stepping": "the faster of Simulator.run (solver convergence read once per 16 steps, window "
                               "re-run on a miss) and Simulator.step (convergence polled in every solve), timed "
                               "on the same steps from fresh simulators; see 'stepping'"},
        "explicit_step": explicit_only(sim, args.steps, WIDTH[args.dtype]),
        "stepping": hb["stepping"],
        "cg_iters_per_solve": hb["cg_iters_per_solve"],
    }
    res["b2b_s"] = damage_pass_b2b(sim)
    out["roofline"] = roofline(res)
    out["damage_cg"] = damage_cg_rates(res, out, out["explicit_step"]["us_per_step"],
                                       out["roofline"]["avg_launch_us"])
    cp = copy_bandwidth()
    out["roofline"]["copy_kernel_GBps"] = cp["GBps"]
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / cp["GBps"], 4)
    out["copy_kernel"] = cp
    # keep the contract's key order: roofline right after the config
    order = list(out)
    order.remove("roofline")
    order.insert(order.index("config") + 1, "roofline")
    out = {k: out[k] for k in order}
    del sim, res
    sections = [("fp32", lambda: fp32_companion(args.steps, args.warmup, None if args.dtype == "f64" else tile))]
    if not args.no_extras:
        sections += [("perforated", perforated), ("batched_step", batched_step),
                     ("graph_replay", lambda: graph_steps(args.steps, tile, args.dtype)),
                     ("bwd_fwd", bwd_fwd_ratio), ("batched", batched_vs_plain),
                     ("subcycling", lambda: subcycling(100)), ("gc_field", lambda: gc_field(100)),
                     ("energies", energies_cost), ("preconditioners", lambda: preconditioners(60)),
                     ("beyond_cache", beyond_cache)]
    if args.dtype == "f32":
        sections = sections[1:]
    if args.sections is not None:
        want = [x for x in args.sections.split(",") if x]
        sections = [(k, fn) for k, fn in sections if k in want]
    for key, fn in sections:
        try:
            out[key] = fn()
        except Exception as e:   # reported on the line; the headline stands on its own
            out[key] = {"error": f"{type(e).__name__}: {e}"}
        print(f"[bench] {key} done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_protocol)
        print("[bench] cpu_baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

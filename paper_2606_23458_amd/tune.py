"""Tile-size autotuning (pf_tune_tiles) with a per-process cache by size class.

A size class is (dtype, split, number of instances, total triangles rounded
to a quarter octave): meshes of one class share the tuned tile size, since
the time per element of a tile plan depends on the tile shape and the launch
width, not on the mesh's details.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _lib as L
from .sim import _stream, params_of

_CACHE: dict[tuple, dict] = {}


def size_class(problems, dtype: str) -> tuple:
    ne = sum(len(p.tri) for p in problems)
    return (dtype, problems[0].split, len(problems), int(round(4 * math.log2(max(ne, 1)))))


def tune_tiles(problems, dtype: str, candidates=None, reps: int = 20, cg_rounds_per_step: float = 16.0,
               use_cache: bool = True) -> dict:
    """Time each candidate tile size on these meshes; returns the report with key 'best'."""
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    key = size_class(problems, dtype)
    if use_cache and candidates is None and key in _CACHE:
        return _CACHE[key]
    n = len(problems)
    keep = []
    descs = (L.MeshDesc * n)()
    for k, pr in enumerate(problems):
        xy = np.ascontiguousarray(pr.xy, dtype=np.float64)
        tri = np.ascontiguousarray(pr.tri, dtype=np.int32)
        fx = None if getattr(pr, "fixed", None) is None else np.ascontiguousarray(pr.fixed, dtype=np.uint8)
        keep += [xy, tri, fx]
        descs[k] = L.MeshDesc(len(xy), len(tri), xy.ctypes.data, tri.ctypes.data,
                              None if fx is None else fx.ctypes.data)
    params = (L.Params * n)(*[params_of(p) for p in problems])
    opts = L.TuneOpts()
    cand = list(candidates or [])
    if len(cand) > L.PF_TUNE_MAX:
        raise ValueError(f"at most {L.PF_TUNE_MAX} candidates")
    opts.n_candidates = len(cand)
    for k, c in enumerate(cand):
        opts.tile_nodes[k] = int(c)
    opts.reps = int(reps)
    opts.cg_rounds_per_step = float(cg_rounds_per_step)
    res = L.TuneResult()
    L.call("pf_tune_tiles", descs, n, L.PF_F64 if dtype == "f64" else L.PF_F32, params, C.byref(opts),
           C.byref(res), _stream())
    rows = []
    for k in range(res.n_tried):
        rows.append({"tile_nodes": res.tile_nodes[k], "status": L.STATUS_NAMES.get(res.status[k], res.status[k]),
                     "explicit_block": res.explicit_block[k], "explicit_chunks": res.explicit_chunks[k],
                     "explicit_us": round(res.explicit_us[k], 3),
                     "cg_round_us": round(res.cg_round_us[k], 3), "score_us": round(res.score_us[k], 3)})
    out = {"best": int(res.best), "explicit_block": int(res.best_explicit_block),
           "explicit_chunks": int(res.best_explicit_chunks), "size_class": key,
           "candidates": rows}
    if use_cache and candidates is None:
        _CACHE[key] = out
    return out

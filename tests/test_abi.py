"""The C ABI without a GPU: symbols, struct layouts, argument validation."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2606_23458_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?(pf_[a-z_0-9]+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = declared_functions()
    assert "pf_explicit_step" in names and "pf_step_backward" in names and len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.pf_version()


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of every public struct, compiled from pf.h with gcc, equal the ctypes mirrors."""
    prog = tmp_path / "sizes.c"
    checks = {
        "pf_mesh_desc_t": (L.MeshDesc, ["n_nodes", "n_elems", "xy", "tri", "fixed"]),
        "pf_tile_opts_t": (L.TileOpts, ["tile_nodes", "explicit_block"]),
        "pf_params_t": (L.Params, ["E", "nu", "rho", "Gc", "l0", "eta", "gamma_star", "model", "split", "plane",
                                   "bounds"]),
        "pf_state_t": (L.StatePtrs, ["ux", "uy", "vx", "vy", "ax", "ay", "d", "H", "t"]),
        "pf_cg_opts_t": (L.CgOpts, ["tol", "max_iter", "check_every", "start", "monotone", "rounds", "resume"]),
        "pf_cg_stats_t": (L.CgStats, ["iters", "restarts", "n_active", "flags", "resid"]),
        "pf_instance_info_t": (L.InstanceInfo, ["node_offset", "n_nodes", "elem_offset", "n_elems", "tile_offset",
                                                "n_tiles", "h_min", "area"]),
        "pf_mesh_totals_t": (L.Totals, ["n_instances", "n_nodes", "n_elems", "n_tiles", "dtype", "max_tile_nodes",
                                        "max_tile_elems", "tile_elems_total", "device_bytes"]),
        "pf_tune_opts_t": (L.TuneOpts, ["n_candidates", "tile_nodes", "reps", "cg_rounds_per_step"]),
        "pf_tune_result_t": (L.TuneResult, ["best", "best_explicit_block", "n_tried", "tile_nodes", "status",
                                            "explicit_block", "explicit_us", "cg_round_us", "score_us"]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for t, (_, fields) in checks.items():
        lines.append(f'printf("{t} %zu\\n", sizeof({t}));')
        for f in fields:
            lines.append(f'printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines.append("return 0; }")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(prog)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True)
               .stdout.splitlines())
    for t, (cls, fields) in checks.items():
        assert int(out[t]) == C.sizeof(cls), t
        for f in fields:
            assert int(out[f"{t}.{f}"]) == getattr(cls, f).offset, f"{t}.{f}"


def _create(xy, tri, fixed=None, n=1, dtype=L.PF_F64, tile=0):
    keep = [np.ascontiguousarray(xy, np.float64), np.ascontiguousarray(tri, np.int32)]
    descs = (L.MeshDesc * max(n, 1))()
    descs[0] = L.MeshDesc(len(keep[0]), len(keep[1]), keep[0].ctypes.data, keep[1].ctypes.data,
                          None if fixed is None else fixed.ctypes.data)
    h = C.c_void_p()
    st = L.lib().pf_mesh_create(descs, n, dtype, C.byref(L.TileOpts(tile)), None, C.byref(h))
    return st, L.lib().pf_last_error().decode()


def test_mesh_validation_errors():
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float)
    st, msg = _create(xy, np.array([[0, 1, 4]]))
    assert st == L.PF_ERR_MESH and "out of range" in msg
    st, msg = _create(xy, np.array([[0, 1, 1]]))
    assert st == L.PF_ERR_MESH and "repeats" in msg
    st, msg = _create(np.array([[0, 0], [1, 0], [2, 0]], float), np.array([[0, 1, 2]]))
    assert st == L.PF_ERR_MESH and "zero area" in msg
    st, msg = _create(xy, np.array([[0, 1, 2]]))
    assert st == L.PF_ERR_MESH and "belongs to no element" in msg
    bad = xy.copy()
    bad[3, 0] = np.nan
    st, msg = _create(bad, np.array([[0, 1, 2], [1, 3, 2]]))
    assert st == L.PF_ERR_MESH and "non-finite" in msg


def test_argument_errors():
    lib = L.lib()
    xy = np.array([[0, 0], [1, 0], [0, 1]], float)
    st, msg = _create(xy, np.array([[0, 1, 2]]), n=0)
    assert st == L.PF_ERR_ARG
    st, msg = _create(xy, np.array([[0, 1, 2]]), dtype=7)
    assert st == L.PF_ERR_ARG
    st, msg = _create(xy, np.array([[0, 1, 2]]), tile=5000)
    assert st == L.PF_ERR_ARG and "tile_nodes" in msg
    keep = [np.ascontiguousarray(xy, np.float64), np.ascontiguousarray([[0, 1, 2]], np.int32)]
    descs = (L.MeshDesc * 1)(L.MeshDesc(3, 1, keep[0].ctypes.data, keep[1].ctypes.data, None))
    h = C.c_void_p()
    assert lib.pf_mesh_create(descs, 1, 0, C.byref(L.TileOpts(0, 384)), None, C.byref(h)) == L.PF_ERR_ARG
    assert "explicit_block" in lib.pf_last_error().decode()
    assert lib.pf_mesh_create(descs, 1, 0, C.byref(L.TileOpts(0, 0, 3)), None, C.byref(h)) == L.PF_ERR_ARG
    assert "explicit_chunks" in lib.pf_last_error().decode()
    assert lib.pf_mesh_create(descs, 1, 0, C.byref(L.TileOpts(0, 0, 0, 3)), None, C.byref(h)) == L.PF_ERR_ARG
    assert "damage_chunks" in lib.pf_last_error().decode()
    assert lib.pf_mesh_create(None, 1, 0, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_explicit_step(None, None, None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_damage_solve(None, None, None, None, None, None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_step_backward(None, None, None, None, None, None, None, None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_tune_tiles(None, 1, 0, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_subcycle_limit(None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_energies(None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_energies_static(None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_set_gc_field(None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_set_loading(None, None, None, None, None, None) == L.PF_ERR_ARG
    assert lib.pf_damage_pass_repeat(None, None, None, None, 1, None) == L.PF_ERR_ARG
    res = L.TuneResult()
    descs = (L.MeshDesc * 1)()
    params = (L.Params * 1)()
    bad = L.TuneOpts()
    bad.n_candidates = 9
    assert lib.pf_tune_tiles(descs, 1, 0, params, C.byref(bad), C.byref(res), None) == L.PF_ERR_ARG
    bad.n_candidates = 1
    bad.tile_nodes[0] = 32
    assert lib.pf_tune_tiles(descs, 1, 0, params, C.byref(bad), C.byref(res), None) == L.PF_ERR_ARG
    assert "tile_nodes" in lib.pf_last_error().decode()
    assert lib.pf_mesh_destroy(None) == L.PF_OK
    tot = L.Totals()
    assert lib.pf_mesh_totals(None, C.byref(tot)) == L.PF_ERR_ARG

"""ctypes binding of libpfrac (include/pf.h): structures, prototypes, status checks.

Argument marshalling only.  Importing this module raises if the built HIP
library is missing; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpfrac.so")

PF_OK, PF_ERR_ARG, PF_ERR_MESH, PF_ERR_HIP, PF_ERR_NOMEM, PF_ERR_NOT_CONVERGED, PF_ERR_NONFINITE, \
    PF_ERR_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "PF_OK", 1: "PF_ERR_ARG", 2: "PF_ERR_MESH", 3: "PF_ERR_HIP", 4: "PF_ERR_NOMEM",
                5: "PF_ERR_NOT_CONVERGED", 6: "PF_ERR_NONFINITE", 7: "PF_ERR_UNSUPPORTED"}
PF_F32, PF_F64 = 0, 1
SPLITS = {"none": 0, "spectral": 1, "voldev": 2, "starconvex": 3}
PLANES = {"strain": 0, "stress": 1}
BOUNDS = {"projected": 0, "postclamp": 1}
PF_ACTIVE_LOWER, PF_ACTIVE_UPPER = 1, 2
PF_ENERGY_STATIC_MAX_TILES = 32768
PF_FLAG_NOT_CONVERGED, PF_FLAG_NONFINITE = 1, 2


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("xy", C.c_void_p), ("tri", C.c_void_p),
                ("fixed", C.c_void_p)]


class TileOpts(C.Structure):
    _fields_ = [("tile_nodes", C.c_int32), ("explicit_block", C.c_int32), ("explicit_chunks", C.c_int32),
                ("damage_chunks", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double), ("Gc", C.c_double),
                ("l0", C.c_double), ("eta", C.c_double), ("gamma_star", C.c_double), ("model", C.c_int32),
                ("split", C.c_int32), ("plane", C.c_int32), ("bounds", C.c_int32)]


class StatePtrs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("ux", "uy", "vx", "vy", "ax", "ay", "d", "H", "t")]


class CgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32), ("start", C.c_int32),
                ("monotone", C.c_int32), ("rounds", C.c_int32), ("resume", C.c_int32), ("precond", C.c_int32)]


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("n_active", C.c_int32), ("flags", C.c_int32),
                ("resid", C.c_double)]


class InstanceInfo(C.Structure):
    _fields_ = [("node_offset", C.c_int32), ("n_nodes", C.c_int32), ("elem_offset", C.c_int32),
                ("n_elems", C.c_int32), ("tile_offset", C.c_int32), ("n_tiles", C.c_int32),
                ("h_min", C.c_double), ("area", C.c_double)]


class Totals(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("n_nodes", C.c_int32), ("n_elems", C.c_int32),
                ("n_tiles", C.c_int32), ("dtype", C.c_int32), ("max_tile_nodes", C.c_int32),
                ("max_tile_elems", C.c_int32), ("tile_elems_total", C.c_int32), ("device_bytes", C.c_size_t),
                ("damage_chunks", C.c_int32)]


PF_TUNE_MAX = 8


class TuneOpts(C.Structure):
    _fields_ = [("n_candidates", C.c_int32), ("tile_nodes", C.c_int32 * PF_TUNE_MAX), ("reps", C.c_int32),
                ("cg_rounds_per_step", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("best", C.c_int32), ("best_explicit_block", C.c_int32), ("n_tried", C.c_int32),
                ("tile_nodes", C.c_int32 * PF_TUNE_MAX), ("status", C.c_int32 * PF_TUNE_MAX),
                ("explicit_block", C.c_int32 * PF_TUNE_MAX), ("explicit_us", C.c_double * PF_TUNE_MAX),
                ("cg_round_us", C.c_double * PF_TUNE_MAX), ("score_us", C.c_double * PF_TUNE_MAX),
                ("best_explicit_chunks", C.c_int32), ("explicit_chunks", C.c_int32 * PF_TUNE_MAX)]


class PfError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# name -> (argtypes)
PROTOTYPES = {
    "pf_mesh_create": [C.POINTER(MeshDesc), C.c_int32, C.c_int32, C.POINTER(TileOpts), C.c_void_p,
                       C.POINTER(C.c_void_p)],
    "pf_mesh_destroy": [C.c_void_p],
    "pf_mesh_totals": [C.c_void_p, C.POINTER(Totals)],
    "pf_mesh_instance": [C.c_void_p, C.c_int32, C.POINTER(InstanceInfo)],
    "pf_mesh_node_perm": [C.c_void_p, C.c_void_p],
    "pf_mesh_elem_perm": [C.c_void_p, C.c_void_p],
    "pf_explicit_step": [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(StatePtrs),
                         C.POINTER(StatePtrs), C.c_void_p, C.c_void_p],
    "pf_damage_solve": [C.c_void_p, C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                        C.c_void_p, C.POINTER(CgOpts), C.c_void_p, C.c_void_p],
    "pf_step_backward": [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(StatePtrs),
                         C.POINTER(StatePtrs), C.c_void_p, C.POINTER(StatePtrs), C.POINTER(StatePtrs),
                         C.c_void_p, C.POINTER(CgOpts), C.c_void_p, C.c_void_p],
    "pf_cfl_dt": [C.c_void_p, C.POINTER(Params), C.c_double, C.POINTER(C.c_double)],
    "pf_tune_tiles": [C.POINTER(MeshDesc), C.c_int32, C.c_int32, C.POINTER(Params), C.POINTER(TuneOpts),
                      C.POINTER(TuneResult), C.c_void_p],
    "pf_energies": [C.c_void_p, C.POINTER(Params), C.POINTER(StatePtrs), C.c_void_p, C.c_void_p],
    "pf_energies_static": [C.c_void_p, C.POINTER(Params), C.POINTER(StatePtrs), C.c_void_p, C.c_void_p],
    "pf_set_gc_field": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "pf_set_loading": [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.c_void_p],
    "pf_subcycle_limit": [C.c_void_p, C.POINTER(Params), C.POINTER(C.c_int32), C.POINTER(C.c_double)],
    "pf_timer_enable": [C.c_void_p, C.c_int32],
    "pf_timer_read": [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "pf_damage_pass_repeat": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
}


def lib() -> C.CDLL:
    """Load libpfrac.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libpfrac.so not found at {LIB_PATH}; build it with "
                              "`python -m paper_2606_23458_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, argt in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.argtypes = argt
            fn.restype = C.c_int
        L.pf_last_error.restype = C.c_char_p
        L.pf_last_error.argtypes = []
        L.pf_version.restype = C.c_char_p
        L.pf_version.argtypes = []
        _lib = L
    return _lib


def check(status: int, func: str) -> None:
    if status != PF_OK:
        raise PfError(status, func, lib().pf_last_error().decode())


def call(name: str, *args) -> int:
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st

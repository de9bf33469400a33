"""MI355X-native matrix-free explicit phase-field fracture (libpfrac + Python binding).

The hot path (explicit step, damage solve, adjoint step) runs in hand-written
HIP kernels for gfx950 in libpfrac.so; this package marshals arguments to it.
"""
from . import _lib
from .sim import CgConfig, GraphStepper, Loading, Mesh, Simulator, State, params_of
from .tune import tune_tiles
from .inverse import invert_gc, invert_gc_field

__all__ = ["_lib", "CgConfig", "Mesh", "GraphStepper", "Loading", "Simulator", "State", "invert_gc", "invert_gc_field",
           "params_of", "tune_tiles"]

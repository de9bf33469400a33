"""MI355X-native matrix-free explicit phase-field fracture (libpfrac + Python binding).

The hot path (explicit step, damage solve, adjoint step) runs in hand-written
HIP kernels for gfx950 in libpfrac.so; this package marshals arguments to it.

Typical use (problems are objects with the fields of workloads.Problem: mesh,
material, model, split, plane, initial state)::

    sim = Simulator(problems, dtype="f32", tile_nodes="auto")   # one handle, all instances
    sim.run(1000)                         # staggered steps; convergence read once per window
    E_kin, E_el, E_frac = sim.energies()[0]
    user_state = sim.state.to_user()      # per instance, in the caller's numbering

    from paper_2606_23458_amd.grad import loss_and_grad
    L, dL_dGc = loss_and_grad(sim, Gc, target, steps=500, checkpoint_every=50)
    out = invert_gc(sim, target, steps=500, gc0=Gc)                # L-BFGS, all instances at once

Options: CgConfig (tolerance, polling, Chebyshev-Jacobi preconditioner),
Simulator(n_sub=...) (damage subcycling), Simulator.set_loading (ramps),
Simulator.set_gc_field (per-element toughness), GraphStepper (HIP graphs).
"""
from . import _lib
from .sim import CgConfig, GraphStepper, Loading, Mesh, Simulator, State, params_of
from .tune import tune_tiles
from .inverse import invert_gc, invert_gc_field

__all__ = ["_lib", "CgConfig", "Mesh", "GraphStepper", "Loading", "Simulator", "State", "invert_gc", "invert_gc_field",
           "params_of", "tune_tiles"]

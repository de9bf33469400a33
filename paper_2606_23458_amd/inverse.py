"""Inversion of the fracture toughness from an observed final damage field
(Sec. 4, material parameter inversion: L-BFGS on the loss of eq.
inversion_loss), driven by the GPU forward map and its reverse sweep.

invert_gc         one G_c per instance, all instances at once: the instances
                  are independent, so L-BFGS-B on the sum of their losses
                  needs one batched forward + backward per evaluation.
invert_gc_field   a toughness field G_c,e = G_c phi_e with phi = B theta for a
                  caller-given basis B (e.g. region indicators), from the
                  per-element gradient dL/dG_c,e.
Both optimise in log space (the toughness stays positive).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize as so
import torch

from .grad import TrajectoryRunner, field_loss_and_grad, loss_and_grad
from .sim import Simulator


def invert_gc(sim: Simulator, target: torch.Tensor, steps: int, gc0, checkpoint_every: int = 50,
              max_iter: int = 40, gtol: float = 1e-14) -> dict:
    """Recover one G_c per instance; `target` is the observed final damage (internal node order)."""
    runner = TrajectoryRunner(sim, steps, checkpoint_every)
    hist = []

    def fun(x):
        gc = np.exp(x)
        L, g = loss_and_grad(sim, gc, target, steps, runner=runner)
        hist.append((gc.copy(), L.copy()))
        return float(L.sum()), g * gc

    x0 = np.log(np.atleast_1d(np.asarray(gc0, dtype=np.float64)))
    res = so.minimize(fun, x0, jac=True, method="L-BFGS-B",
                      options={"maxiter": max_iter, "ftol": 0.0, "gtol": gtol})
    return {"Gc": np.exp(res.x), "loss": hist[-1][1] if hist else None, "evaluations": len(hist),
            "iterations": int(res.nit), "message": str(res.message), "history": hist}


def invert_gc_field(sim: Simulator, target: torch.Tensor, steps: int, basis, theta0, checkpoint_every: int = 50,
                    max_iter: int = 40, gtol: float = 1e-14) -> dict:
    """Recover phi = basis @ theta (one instance; basis is (n_elems, n_params) in the
    user's element order) so that G_c,e = G_c phi_e reproduces `target`."""
    if sim.mesh.n_instances != 1:
        raise ValueError("invert_gc_field inverts the field of a single instance")
    B = np.asarray(basis, dtype=np.float64)
    gc = float(sim.params[0].Gc)
    runner = TrajectoryRunner(sim, steps, checkpoint_every)
    hist = []

    def fun(x):
        theta = np.exp(x)
        sim.set_gc_field([B @ theta])
        L, ge = field_loss_and_grad(sim, target, steps, runner=runner)
        # dL/dtheta_j = sum_e B_ej dL/dphi_e, dL/dphi_e = G_c dL/dG_c,e
        g = (B.T @ (gc * ge[0])) * theta
        hist.append((theta.copy(), float(L[0])))
        return float(L[0]), g

    x0 = np.log(np.asarray(theta0, dtype=np.float64))
    res = so.minimize(fun, x0, jac=True, method="L-BFGS-B",
                      options={"maxiter": max_iter, "ftol": 0.0, "gtol": gtol})
    theta = np.exp(res.x)
    sim.set_gc_field([B @ theta])
    return {"theta": theta, "loss": hist[-1][1] if hist else None, "evaluations": len(hist),
            "iterations": int(res.nit), "message": str(res.message), "history": hist}

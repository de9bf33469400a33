"""Helpers for the GPU parity tests: seeded states, oracle <-> library conversion."""
import numpy as np
import torch

import oracle
from oracle.step import Sim as OSim, State as OState


def random_state(problem, seed: int, amp_u: float = 2e-6, damage: bool = True) -> dict:
    """A seeded, physically scaled random state in the caller's numbering."""
    r = np.random.default_rng(seed)
    n, ne = problem.n_nodes, problem.n_elems
    fixed = problem.fixed.astype(bool)
    u = r.normal(size=(n, 2)) * amp_u
    v = r.normal(size=(n, 2)) * 0.3
    a = r.normal(size=(n, 2)) * 3e6
    a[fixed] = 0.0
    v[fixed] = problem.v0[fixed]
    d = np.clip(r.uniform(-0.3, 1.0, n), 0.0, 1.0) if damage else np.zeros(n)
    d[problem.d0 == 1.0] = 1.0
    H = r.uniform(0, 3000.0, ne)
    return {"u": u, "v": v, "a": a, "d": d, "H": H}


def to_oracle(st: dict) -> OState:
    f = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64).clone()
    return OState(f(st["u"]), f(st["v"]), f(st["a"]), f(st["d"]), f(st["H"]))


def rel_err(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    if scale == 0:
        return float(np.max(np.abs(got)))
    return float(np.max(np.abs(got - ref)) / scale)

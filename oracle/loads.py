"""Time-dependent loads (Sec. 3, loading protocols): the smooth traction ramp
(eq. smooth_traction_ramp) and the velocity ramp (eq. kalthoff_velocity_ramp).

Oracle: test infrastructure only.

Readings used here:
* the external force of a step is evaluated at the step's end time t_{n+1}
  (it enters a_{n+1} = m^-1 (f_ext - f_int(u_{n+1})));
* a prescribed velocity that ramps is applied at the step's midpoint
  t_n + dt/2 (the displacement increment dt v is then exact for the linear
  ramp).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .step import Sim, State, initial_state


def smooth_ramp(t: float, t_r: float) -> float:
    """S(t): 0 for t <= 0, (1 - cos(pi t / t_r)) / 2 on (0, t_r), 1 for t >= t_r."""
    if t <= 0.0:
        return 0.0
    if t >= t_r:
        return 1.0
    return 0.5 * (1.0 - math.cos(math.pi * t / t_r))


def velocity_ramp(t: float, t_r: float) -> float:
    """v(t)/v0: t/t_r on [0, t_r), 1 afterwards."""
    if t_r <= 0.0 or t >= t_r:
        return 1.0
    return max(t, 0.0) / t_r


def run_loaded(problem, steps: int, traction: np.ndarray | None = None, t_traction: float = 0.0,
               t_velocity: float = 0.0, sim: Sim | None = None) -> State:
    """Staggered steps under ramped loads.

    traction: (N, 2) nodal force reached at full load, scaled by S(t_{n+1});
    t_velocity > 0: the prescribed velocities (problem.v0 on fixed DOFs) are
    scaled by the velocity ramp at t_n + dt/2.
    """
    sim = sim or Sim(problem)
    st = initial_state(problem)
    fixed = torch.as_tensor(np.asarray(problem.fixed, dtype=bool))
    v0 = torch.as_tensor(np.asarray(problem.v0, dtype=np.float64))
    dt = sim.dt
    for n in range(steps):
        if t_velocity > 0.0:
            fac = velocity_ramp(n * dt + 0.5 * dt, t_velocity)
            st = State(st.u, torch.where(fixed, fac * v0, st.v), st.a, st.d, st.H)
        f = None
        if traction is not None:
            f = smooth_ramp((n + 1) * dt, t_traction) * torch.as_tensor(np.asarray(traction, dtype=np.float64))
        st = sim.step(st, f_ext=f)
    return st

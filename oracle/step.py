"""Staggered explicit step, trajectories and the G_c gradient (Sec. 2.2-2.4, Sec. 4).

Oracle: test infrastructure only.

One step n -> n+1 (Sec. 2.2, staggered scheme; Sec. 2.3, velocity-Verlet):
  1. u_{n+1} = u_n + dt v_n + dt^2/2 a_n                       (eq. vv_u)
  2. eps_e from u_{n+1}; d_e = mean of the three nodal d_n; g = (1-d_e)^2 + eta;
     sigma_e = g sigma+ + sigma-; f_int = sum_e A_e B_e' sigma_e
  3. a_{n+1} = m^-1 (f_ext - f_int) on free DOFs, 0 on prescribed DOFs  (eq. vv_a)
  4. v_{n+1} = v_n + dt/2 (a_n + a_{n+1})                       (eq. vv_v)
  5. H_{n+1} = psi+ where psi+ > H_n, else H_n
  6. d_{n+1} = damage QP with lower bound d_n (DamageQP).
Prescribed-velocity DOFs keep their velocity in v and zero acceleration, so
the same formulas advance them by dt * v.

Readings: the element damage inside g(d) is the centroid value (mean of the
three nodal values); H is one value per element; ties of the maximum keep
H_n.  The gradient of the final-damage loss with respect to G_c is taken by
forward-mode differentiation of the whole trajectory; the damage update
contributes through the implicit rule (DamageQP.tangent).

A spatially varying toughness (the per-element G_c(x) inverse problem named
in Sec. 4) is G_c,e = G_c phi_e with a per-element factor phi (Sim.gc_scale);
phi enters only the damage sub-problem and the fracture energy.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch
import torch.autograd.forward_ad as fwAD

from .constitutive import split_energy
from .damage import DamageQP, energies
from .fem import Mesh, cfl_dt, element_strain, internal_force, lumped_mass, make_mesh


@dataclass
class Material:
    E: float
    nu: float
    rho: float
    Gc: float
    l0: float
    eta: float
    model: int
    split: str
    plane: str
    gamma_star: float = 0.0
    bounds: str = "projected"

    @staticmethod
    def of(problem) -> "Material":
        return Material(problem.E, problem.nu, problem.rho, problem.Gc, problem.l0, problem.eta,
                        problem.model, problem.split, problem.plane, problem.gamma_star, problem.bounds)


@dataclass
class State:
    u: torch.Tensor   # (N,2)
    v: torch.Tensor   # (N,2)
    a: torch.Tensor   # (N,2)
    d: torch.Tensor   # (N,)
    H: torch.Tensor   # (Ne,)

    def numpy(self) -> dict:
        return {k: fwAD.unpack_dual(getattr(self, k))[0].detach().numpy().copy()
                for k in ("u", "v", "a", "d", "H")}


def initial_state(problem) -> State:
    f = lambda x: torch.as_tensor(np.asarray(x), dtype=torch.float64).clone()
    return State(f(problem.u0), f(problem.v0), f(problem.a0), f(problem.d0), f(problem.H0))


class Sim:
    """Mesh, material and constant operators of one problem."""

    def __init__(self, problem, dt: float | None = None, material: Material | None = None, gc_scale=None,
                 qp_inner: str = "lu"):
        self.mat = material or Material.of(problem)
        # per-element factor phi of G_c,e = G_c phi_e (None: uniform); a
        # forward-mode dual tensor carries a direction of phi
        self.gc_scale = gc_scale
        self.mesh: Mesh = make_mesh(problem.xy, problem.tri, problem.fixed)
        self.mass = lumped_mass(self.mesh, self.mat.rho)
        self.minv = 1.0 / self.mass
        self.dt = dt if dt is not None else cfl_dt(self.mesh, self.mat.E, self.mat.nu, self.mat.rho,
                                                    self.mat.plane, problem.cfl)
        self.qp = DamageQP(self.mesh, self.mat.l0, self.mat.model, self.mat.bounds, qp_inner)

    def stress(self, u, d):
        """Element strain energy parts and stress for displacement u and damage d."""
        m = self.mat
        exx, eyy, exy = element_strain(self.mesh, u)
        psi_p, psi_m, sp, sm = split_energy(exx, eyy, exy, m.E, m.nu, m.plane, m.split, m.gamma_star)
        de = d[self.mesh.tri].sum(1) / 3.0
        g = (1.0 - de) ** 2 + m.eta
        sig = (g * sp[0] + sm[0], g * sp[1] + sm[1], g * sp[2] + sm[2])
        return psi_p, psi_m, g, sig

    def explicit(self, st: State, f_ext=None):
        """Steps 1-5: returns (u_{n+1}, v_{n+1}, a_{n+1}, H_{n+1}, psi_e(u_{n+1}, d_n))."""
        dt = self.dt
        u1 = st.u + dt * st.v + (0.5 * dt * dt) * st.a
        psi_p, psi_m, g, sig = self.stress(u1, st.d)
        f = internal_force(self.mesh, *sig)
        rhs = -f if f_ext is None else torch.as_tensor(f_ext, dtype=torch.float64) - f
        a1 = self.minv[:, None] * rhs
        a1 = torch.where(self.mesh.fixed, torch.zeros_like(a1), a1)
        v1 = st.v + (0.5 * dt) * (st.a + a1)
        H1 = torch.where(psi_p > st.H, psi_p, st.H)
        return u1, v1, a1, H1, g * psi_p + psi_m

    def damage(self, H, d_prev, Gc):
        """Step 6 with forward-mode tangents passed through the implicit rule."""
        Hp, Ht = fwAD.unpack_dual(H)
        lp, lt = fwAD.unpack_dual(d_prev)
        if isinstance(Gc, torch.Tensor):
            gp, gt = fwAD.unpack_dual(Gc)
            gcv = float(gp)
        else:
            gt, gcv = None, float(Gc)
        phi, pt = None, None
        if self.gc_scale is not None:
            if isinstance(self.gc_scale, torch.Tensor):
                pp, pt = fwAD.unpack_dual(self.gc_scale)
                phi = pp.detach().numpy()
                pt = None if pt is None else pt.detach().numpy()
            else:
                phi = np.asarray(self.gc_scale, dtype=np.float64)
        Hn = Hp.detach().numpy()
        dn, act, upper, x, A = self.qp.solve(Hn, gcv, lp.detach().numpy(), phi)
        out = torch.from_numpy(dn)
        if Ht is None and lt is None and gt is None and pt is None:
            return out, act, upper
        zero_e = np.zeros(self.mesh.n_elems)
        zero_n = np.zeros(self.mesh.n_nodes)
        tan = self.qp.tangent(A, x, act, upper, Hn, gcv,
                              zero_e if Ht is None else Ht.detach().numpy(),
                              0.0 if gt is None else float(gt),
                              zero_n if lt is None else lt.detach().numpy(), phi, pt)
        return fwAD.make_dual(out, torch.from_numpy(tan)), act, upper

    def step(self, st: State, Gc=None, f_ext=None, info: dict | None = None, solve: bool = True) -> State:
        """One staggered step; with solve=False the damage sub-problem is skipped (subcycling:
        d_{n+1} = d_n while the mechanics and the history field advance)."""
        u1, v1, a1, H1, _ = self.explicit(st, f_ext)
        if not solve:
            return State(u1, v1, a1, st.d, H1)
        d1, act, upper = self.damage(H1, st.d, self.mat.Gc if Gc is None else Gc)
        if info is not None:
            info["active"] = act
            info["upper"] = upper
        return State(u1, v1, a1, d1, H1)

    def energies(self, st: State):
        u = fwAD.unpack_dual(st.u)[0]
        d = fwAD.unpack_dual(st.d)[0]
        psi_p, psi_m, g, _ = self.stress(u, d)
        psi = (g * psi_p + psi_m).detach().numpy()
        phi = self.gc_scale
        if isinstance(phi, torch.Tensor):
            phi = fwAD.unpack_dual(phi)[0].detach().numpy()
        return energies(self.mesh, self.mass.numpy(), fwAD.unpack_dual(st.v)[0].detach().numpy(), psi,
                        d.detach().numpy(), self.mat.Gc, self.mat.l0, self.mat.model, K=self.qp.K, M=self.qp.M,
                        phi=phi)


def explicit_step(problem, st: State, dt: float | None = None):
    return Sim(problem, dt).explicit(st)


def staggered_step(problem, st: State, dt: float | None = None) -> State:
    return Sim(problem, dt).step(st)


def run(problem, steps: int | None = None, Gc: float | None = None, dt: float | None = None,
        state: State | None = None, record_every: int = 0, sim: Sim | None = None, n_sub: int = 1):
    """Integrate ``steps`` staggered steps; returns (final State, recorded states, sim).

    With n_sub > 1 the damage sub-problem is solved only on every n_sub-th
    step (steps n_sub, 2 n_sub, ... counted from 1), as in the paper's
    subcycling (Sec. 2.3); the history field is updated every step.
    """
    if n_sub < 1:
        raise ValueError("n_sub must be >= 1")
    sim = sim or Sim(problem, dt)
    st = state or initial_state(problem)
    n = problem.steps if steps is None else steps
    rec = []
    g = sim.mat.Gc if Gc is None else Gc
    for k in range(n):
        st = sim.step(st, Gc=g, solve=(k + 1) % n_sub == 0)
        if record_every and (k + 1) % record_every == 0:
            rec.append(st.numpy())
    return st, rec, sim


def loss_and_grad(problem, d_target: np.ndarray, Gc: float, steps: int | None = None,
                  dt: float | None = None, sim: Sim | None = None):
    """Nodewise MSE of the final damage (eq. inversion_loss) and dL/dG_c.

    The derivative is the forward-mode tangent of L along G_c.
    """
    sim = sim or Sim(problem, dt)
    n = problem.steps if steps is None else steps
    tgt = torch.as_tensor(np.asarray(d_target), dtype=torch.float64)
    with fwAD.dual_level():
        gc = fwAD.make_dual(torch.tensor(float(Gc), dtype=torch.float64), torch.tensor(1.0, dtype=torch.float64))
        st = initial_state(problem)
        for _ in range(n):
            st = sim.step(st, Gc=gc)
        L = ((st.d - tgt) ** 2).mean()
        Lp, Lt = fwAD.unpack_dual(L)
        d_final = fwAD.unpack_dual(st.d)[0].detach().numpy().copy()
    return float(Lp), (0.0 if Lt is None else float(Lt)), d_final


def loss_and_field_derivative(problem, d_target: np.ndarray, Gc: float, gc_scale, direction,
                              steps: int | None = None, dt: float | None = None):
    """Loss of eq. inversion_loss for the toughness field G_c,e = G_c phi_e and its
    directional derivative along a change `direction` of the element toughness
    G_c,e (absolute units), by forward-mode differentiation of the trajectory.

    The GPU adjoint's per-element gradient g_e = dL/dG_c,e satisfies
    sum_e g_e direction_e = this derivative.
    """
    sim = Sim(problem, dt)
    n = problem.steps if steps is None else steps
    tgt = torch.as_tensor(np.asarray(d_target), dtype=torch.float64)
    phi = torch.as_tensor(np.asarray(gc_scale, dtype=np.float64))
    dphi = torch.as_tensor(np.asarray(direction, dtype=np.float64) / float(Gc))
    with fwAD.dual_level():
        sim.gc_scale = fwAD.make_dual(phi, dphi)
        st = initial_state(problem)
        for _ in range(n):
            st = sim.step(st, Gc=float(Gc))
        L = ((st.d - tgt) ** 2).mean()
        Lp, Lt = fwAD.unpack_dual(L)
        d_final = fwAD.unpack_dual(st.d)[0].detach().numpy().copy()
    return float(Lp), (0.0 if Lt is None else float(Lt)), d_final

"""Damage sub-problem as a bound-constrained quadratic programme (Sec. 2.2, Sec. 2.4).

Oracle: test infrastructure only.

For element-constant history H_e on P1 triangles the weak forms of
eq. damage_pde_at2 and eq. damage_pde_at1 give a symmetric system
A d = b with

  AT2: A = G_c l0 K + sum_e (G_c/l0 + 2 H_e) M^e,   b_i = sum_{e ni i} 2 H_e A_e / 3
  AT1: A = 3/4 G_c l0 K + sum_e 2 H_e M^e,           b_i = sum_{e ni i} (2 H_e - 3 G_c/(8 l0)) A_e / 3

with K^e_kl = A_e grad phi_k . grad phi_l and the consistent element mass
M^e_kl = A_e (1 + delta_kl) / 12 of Sec. 2.4.  Irreversibility and the lower
bound make the update the minimiser of 1/2 d'Ad - b'd over d >= lb with
lb = d_n (Sec. 2.4, bound enforcement); the upper bound d <= 1 is imposed
as a second bound of the same programme, so the update is the minimiser over
d_n <= d <= 1 (the phase field lives in [0, 1], Sec. 2.1).  The paper's AT2
alternative (unconstrained solve, then clamp to [d_n, 1]) is the 'postclamp'
mode.

The exact minimiser is found by a primal-dual active-set iteration with a
sparse LU solve on the free set; the result is verified against the KKT
conditions.  For the full-size plates the free-set systems can instead be
solved by SciPy's conjugate gradients (Jacobi-preconditioned, relative
residual 1e-14): the same active-set iteration and KKT check, an order of
magnitude faster at a million unknowns.  Reading: the damage operator uses
g = (1-d)^2 without eta.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from .fem import Mesh


def _pairs(mesh: Mesh):
    tri = mesh.tri.numpy()
    rows = np.repeat(tri, 3, axis=1).ravel()        # k repeated over l
    cols = np.tile(tri, (1, 3)).ravel()
    return rows, cols


def stiffness_matrix(mesh: Mesh, coef: np.ndarray | None = None) -> sp.csr_matrix:
    """K = sum_e coef_e A_e grad phi_k . grad phi_l (coef = 1: unit diffusion)."""
    G = mesh.grad.numpy()
    A = mesh.area.numpy() if coef is None else mesh.area.numpy() * np.asarray(coef)
    ke = A[:, None, None] * np.einsum("ekc,elc->ekl", G, G)
    rows, cols = _pairs(mesh)
    n = mesh.n_nodes
    return sp.coo_matrix((ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def mass_matrix(mesh: Mesh, coef: np.ndarray | None = None) -> sp.csr_matrix:
    """sum_e coef_e M^e with M^e_kl = A_e (1 + delta_kl)/12."""
    A = mesh.area.numpy() if coef is None else mesh.area.numpy() * np.asarray(coef)
    pat = (np.ones((3, 3)) + np.eye(3)) / 12.0
    me = A[:, None, None] * pat[None]
    rows, cols = _pairs(mesh)
    n = mesh.n_nodes
    return sp.coo_matrix((me.ravel(), (rows, cols)), shape=(n, n)).tocsr()


def node_area(mesh: Mesh) -> np.ndarray:
    """sum_{e ni i} A_e/3 (the integral of the hat function phi_i)."""
    w = np.zeros(mesh.n_nodes)
    np.add.at(w, mesh.tri.numpy().ravel(), np.repeat(mesh.area.numpy() / 3.0, 3))
    return w


def damage_coefficients(model: int, Gc: float, l0: float):
    """(kappa, reaction constant, load constant) of the AT2/AT1 weak form.

    AT2: kappa = Gc l0, c_e = Gc/l0 + 2H_e, load 2H_e.
    AT1: kappa = 3/4 Gc l0, c_e = 2H_e, load 2H_e - 3Gc/(8 l0).
    """
    if model == 2:
        return Gc * l0, Gc / l0, 0.0
    if model == 1:
        return 0.75 * Gc * l0, 0.0, -3.0 * Gc / (8.0 * l0)
    raise ValueError(model)


def assemble_damage(mesh: Mesh, H: np.ndarray, Gc: float, l0: float, model: int, K=None, phi=None):
    """Return (A, b) for the current history H (element array).

    phi (element array, optional) makes the fracture energy a field,
    Gc_e = Gc phi_e: every Gc in the element's weak form becomes Gc_e.
    """
    H = np.asarray(H, dtype=np.float64)
    kappa, c0, b0 = damage_coefficients(model, Gc, l0)
    if phi is None:
        if K is None:
            K = stiffness_matrix(mesh)
        A = (kappa * K + mass_matrix(mesh, c0 + 2.0 * H)).tocsr()
        load = 2.0 * H + b0
    else:
        phi = np.asarray(phi, dtype=np.float64)
        A = (stiffness_matrix(mesh, kappa * phi) + mass_matrix(mesh, c0 * phi + 2.0 * H)).tocsr()
        load = 2.0 * H + b0 * phi
    b = np.zeros(mesh.n_nodes)
    np.add.at(b, mesh.tri.numpy().ravel(), np.repeat(load * mesh.area.numpy() / 3.0, 3))
    return A, b


def kkt_residuals(A, b, lb, x, ub=None):
    """Scaled KKT violations of min 1/2 x'Ax - b'x over lb <= x <= ub.

    Returns (bound violation, max |r_i|/A_ii over free nodes, max r_i/A_ii over
    nodes at the lower bound, max -r_i/A_ii over nodes at the upper bound)
    with r = b - A x; nodes with lb_i = ub_i are fixed and carry no sign
    condition.  All are <= 0 or small at the minimiser.
    """
    r = b - A @ x
    dg = A.diagonal()
    ub = np.full(len(x), np.inf) if ub is None else np.asarray(ub, dtype=np.float64)
    fixed = np.asarray(lb) >= ub          # lb = ub: the node is fixed, its multiplier has either sign
    lo = (x <= lb) & ~fixed
    up = (x >= ub) & ~lo & ~fixed
    free = ~(lo | up | fixed)
    viol = float(max(np.max(lb - x), np.max(x - ub))) if len(x) else 0.0
    rf = float(np.max(np.abs(r[free]) / dg[free])) if free.any() else 0.0
    ra = float(np.max(r[lo] / dg[lo])) if lo.any() else -np.inf
    ru = float(np.max(-r[up] / dg[up])) if up.any() else -np.inf
    return viol, rf, ra, ru


def solve_spd(A, rhs, inner: str = "lu") -> np.ndarray:
    """Solve A x = rhs for a sparse SPD matrix: sparse LU ('lu') or Jacobi-preconditioned
    conjugate gradients to a relative residual of 1e-14 ('cg')."""
    if inner == "lu":
        return spla.spsolve(sp.csc_matrix(A), rhs)
    if inner != "cg":
        raise ValueError(inner)
    if not np.any(rhs):
        return np.zeros(len(rhs))
    x, info = spla.cg(A, rhs, rtol=1e-14, atol=0.0, M=sp.diags(1.0 / A.diagonal()), maxiter=50000)
    if info != 0:
        raise RuntimeError(f"conjugate gradients did not converge (info={info})")
    return x


def solve_box_qp(A, b, lb, ub=None, x0=None, max_iter: int = 200, check: bool = True, tol: float = 1e-9,
                 kkt_tol: float = 1e-13, inner: str = "lu"):
    """Exact minimiser of 1/2 x'Ax - b'x subject to lb <= x <= ub (ub = None: no upper bound).

    Primal-dual active set on the gradient g = A x - b: a node is held at its
    lower bound when g_i + A_ii (lb_i - x_i) > 0 and at its upper bound when
    g_i + A_ii (ub_i - x_i) < 0; free nodes solve A_FF x_F = b_F - A_FH x_H
    exactly (solve_spd).  The iteration stops as soon as the iterate satisfies
    the KKT conditions to rounding (free nodes inside the bounds to kkt_tol,
    scaled multipliers of held nodes of the right sign to kkt_tol), or when
    the sets repeat.  Nodes at a degenerate free boundary (x_i at a bound with
    zero multiplier, e.g. the edge of the AT1 support) would otherwise flip
    between the sets on rounding noise.  Returns (x, lower mask, upper mask).
    """
    A = sp.csr_matrix(A)
    lb = np.asarray(lb, dtype=np.float64)
    ub = np.full(len(b), np.inf) if ub is None else np.asarray(ub, dtype=np.float64)
    dg = A.diagonal()
    x = np.clip(lb if x0 is None else np.asarray(x0, dtype=np.float64), lb, ub)
    g = A @ x - b
    lo = (g + dg * (lb - x)) > 0
    up = ((g + dg * (ub - x)) < 0) & ~lo
    seen = set()
    for _ in range(max_iter):
        key = lo.tobytes() + up.tobytes()
        if key in seen:
            raise RuntimeError("active-set iteration cycled")
        seen.add(key)
        held = lo | up
        free = ~held
        x = np.where(lo, lb, np.where(up, ub, 0.0))
        if free.any():
            Aff = A[free][:, free].tocsc()
            rhs = b[free] - A[free][:, held] @ x[held]
            x[free] = solve_spd(Aff, rhs, inner) if free.sum() > 1 else rhs / Aff.toarray()[0, 0]
        g = A @ x - b
        g[free] = 0.0
        if (np.all(x[free] >= lb[free] - kkt_tol) and np.all(x[free] <= ub[free] + kkt_tol)
                and np.all(g[lo] / dg[lo] >= -kkt_tol) and np.all(g[up] / dg[up] <= kkt_tol)):
            break
        new_lo = (g + dg * (lb - x)) > 0
        new_up = ((g + dg * (ub - x)) < 0) & ~new_lo
        if np.array_equal(new_lo, lo) and np.array_equal(new_up, up):
            break
        lo, up = new_lo, new_up
    else:
        raise RuntimeError("active-set iteration did not converge")
    x = np.clip(x, lb, ub)
    if check:
        viol, rf, ra, ru = kkt_residuals(A, b, lb, x, ub)
        if viol > 0 or rf > tol or ra > tol or ru > tol:
            raise RuntimeError(f"KKT check failed: viol={viol} rf={rf} ra={ra} ru={ru}")
    return x, lo, up


def solve_bound_qp(A, b, lb, x0=None, max_iter: int = 200, check: bool = True, tol: float = 1e-9,
                   kkt_tol: float = 1e-13, inner: str = "lu"):
    """Exact minimiser of 1/2 x'Ax - b'x subject to x >= lb; returns (x, active mask)."""
    x, lo, _ = solve_box_qp(A, b, lb, None, x0=x0, max_iter=max_iter, check=check, tol=tol, kkt_tol=kkt_tol,
                            inner=inner)
    return x, lo


@dataclass
class DamageQP:
    """Damage update of one staggered step for a fixed mesh and model."""
    mesh: Mesh
    l0: float
    model: int
    bounds: str = "projected"
    inner: str = "lu"          # free-set solver of the active-set iteration (solve_spd)

    def __post_init__(self):
        self.K = stiffness_matrix(self.mesh)
        self.M = mass_matrix(self.mesh)
        self.w = node_area(self.mesh)

    def system(self, H, Gc, phi=None):
        return assemble_damage(self.mesh, H, Gc, self.l0, self.model, K=self.K, phi=phi)

    def solve(self, H, Gc, d_prev, phi=None):
        """Return (d_new, lower, upper, x, A).

        Projected mode: d_new = x is the minimiser over d_prev <= d <= 1;
        lower / upper mark nodes held at d_prev / at 1.  Post-clamp mode: x is
        the unconstrained solution and d_new = min(max(x, d_prev), 1).
        """
        A, b = self.system(H, Gc, phi)
        if self.bounds == "projected":
            x, lo, up = solve_box_qp(A, b, d_prev, np.ones(len(b)), x0=d_prev, inner=self.inner)
            return x, lo, up, x, A
        if self.bounds == "postclamp":
            x = spla.spsolve(A.tocsc(), b)
            lo = x < d_prev
            xc = np.where(lo, d_prev, x)
            up = xc > 1.0
            return np.minimum(xc, 1.0), lo, up, x, A
        raise ValueError(self.bounds)

    def tangent(self, A, x, act, upper, H, Gc, dH, dGc, dlb, phi=None, dphi=None):
        """Directional derivative of the update (implicit rule, Sec. 4.2).

        Projected mode: nodes held at d_prev follow it, nodes held at 1 do not
        move, and the free nodes F solve
        A_FF xdot_F = (bdot - Adot x - A_F,held xdot_held)_F.
        Post-clamp mode: the linear solve is unconstrained, A xdot = bdot - Adot x,
        and the clamp passes d_prev's tangent where x < d_prev and 0 where x > 1.
        """
        kappa_dg = {2: self.l0, 1: 0.75 * self.l0}[self.model]
        b0_dg = {2: 0.0, 1: -3.0 / (8.0 * self.l0)}[self.model]
        c0_dg = {2: 1.0 / self.l0, 1: 0.0}[self.model]
        # tangent of the element fracture energies Gc_e = Gc phi_e
        ne = self.mesh.n_elems
        ph = np.ones(ne) if phi is None else np.asarray(phi, dtype=np.float64)
        dph = np.zeros(ne) if dphi is None else np.asarray(dphi, dtype=np.float64)
        dgce = dGc * ph + Gc * dph
        Adot_x = (stiffness_matrix(self.mesh, kappa_dg * dgce) @ x
                  + mass_matrix(self.mesh, c0_dg * dgce + 2.0 * dH) @ x)
        bdot = np.zeros(self.mesh.n_nodes)
        np.add.at(bdot, self.mesh.tri.numpy().ravel(),
                  np.repeat((2.0 * dH + dgce * b0_dg) * self.mesh.area.numpy() / 3.0, 3))
        if self.bounds == "projected":
            held = act | upper
            free = ~held
            xdot = np.where(act, dlb, 0.0)
            if free.any():
                rhs = (bdot - Adot_x - A @ xdot)[free]
                xdot[free] = spla.spsolve(A[free][:, free].tocsc(), rhs)
            return xdot
        full = spla.spsolve(A.tocsc(), bdot - Adot_x)
        xdot = np.where(act, dlb, full)
        return np.where(upper, 0.0, xdot)


def energies(mesh: Mesh, mass: np.ndarray, v, psi_total, d, Gc: float, l0: float, model: int, K=None, M=None,
             phi=None):
    """Kinetic, elastic and fracture energy per unit thickness.

    E_kin = 1/2 sum m_i |v_i|^2, E_el = sum_e A_e psi_e,
    E_frac(AT2) = Gc (d'Md/(2 l0) + l0/2 d'Kd),
    E_frac(AT1) = 3Gc/8 (int d / l0 + l0 d'Kd);
    with a field phi (Gc_e = Gc phi_e) each element's share is weighted by phi_e.
    """
    v = np.asarray(v)
    d = np.asarray(d)
    e_kin = 0.5 * float(np.sum(np.asarray(mass)[:, None] * v * v))
    e_el = float(np.sum(mesh.area.numpy() * np.asarray(psi_total)))
    if phi is not None:
        K = stiffness_matrix(mesh, phi)
        M = mass_matrix(mesh, phi)
        w = np.zeros(mesh.n_nodes)
        np.add.at(w, mesh.tri.numpy().ravel(), np.repeat(np.asarray(phi) * mesh.area.numpy() / 3.0, 3))
    else:
        K = stiffness_matrix(mesh) if K is None else K
        M = mass_matrix(mesh) if M is None else M
        w = node_area(mesh)
    if model == 2:
        e_fr = Gc * (float(d @ (M @ d)) / (2.0 * l0) + 0.5 * l0 * float(d @ (K @ d)))
    else:
        e_fr = 3.0 * Gc / 8.0 * (float(w @ d) / l0 + l0 * float(d @ (K @ d)))
    return e_kin, e_el, e_fr

"""P1 triangle geometry, strain, internal force and lumped mass (Sec. 2.3).

Oracle: test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .constitutive import wave_speed


@dataclass
class Mesh:
    xy: torch.Tensor      # (N,2) float64
    tri: torch.Tensor     # (Ne,3) int64, counter-clockwise
    grad: torch.Tensor    # (Ne,3,2) shape-function gradients, row k = grad phi_k
    area: torch.Tensor    # (Ne,)
    fixed: torch.Tensor   # (N,2) bool

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tri.shape[0])


def make_mesh(xy, tri, fixed=None) -> Mesh:
    """Orient every triangle counter-clockwise and precompute eq. grad_phi and A_e.

    A triangle of zero area is an error.
    """
    xy = torch.as_tensor(np.asarray(xy), dtype=torch.float64)
    tri = torch.as_tensor(np.asarray(tri), dtype=torch.int64).clone()
    x = xy[tri]
    two_a = ((x[:, 1, 0] - x[:, 0, 0]) * (x[:, 2, 1] - x[:, 0, 1])
             - (x[:, 2, 0] - x[:, 0, 0]) * (x[:, 1, 1] - x[:, 0, 1]))
    if bool((two_a == 0).any()):
        raise ValueError("degenerate triangle")
    cw = two_a < 0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    two_a = two_a.abs()
    x = xy[tri]
    x1, y1 = x[:, 0, 0], x[:, 0, 1]
    x2, y2 = x[:, 1, 0], x[:, 1, 1]
    x3, y3 = x[:, 2, 0], x[:, 2, 1]
    grad = torch.stack([torch.stack([y2 - y3, x3 - x2], 1),
                        torch.stack([y3 - y1, x1 - x3], 1),
                        torch.stack([y1 - y2, x2 - x1], 1)], 1) / two_a[:, None, None]
    if fixed is None:
        fixed_t = torch.zeros(xy.shape, dtype=torch.bool)
    else:
        fixed_t = torch.as_tensor(np.asarray(fixed)).bool()
    return Mesh(xy=xy, tri=tri, grad=grad, area=0.5 * two_a, fixed=fixed_t)


def lumped_mass(mesh: Mesh, rho: float) -> torch.Tensor:
    """m_i = rho * sum over elements containing i of A_e/3."""
    m = torch.zeros(mesh.n_nodes, dtype=torch.float64)
    m.index_add_(0, mesh.tri.reshape(-1), (rho * mesh.area / 3.0).repeat_interleave(3))
    return m


def h_min(mesh: Mesh) -> float:
    """Smallest incircle diameter, 4 A_e / perimeter_e."""
    x = mesh.xy[mesh.tri]
    per = ((x[:, 0] - x[:, 1]).norm(dim=1) + (x[:, 1] - x[:, 2]).norm(dim=1)
           + (x[:, 2] - x[:, 0]).norm(dim=1))
    return float((4.0 * mesh.area / per).min())


def cfl_dt(mesh: Mesh, E: float, nu: float, rho: float, plane: str, factor: float) -> float:
    """dt = factor * h_min / c_p (Sec. 2.3, CFL condition)."""
    return factor * h_min(mesh) / wave_speed(E, nu, rho, plane)


def element_strain(mesh: Mesh, u: torch.Tensor):
    """Constant P1 strain eps = sym(sum_k u_k (x) grad phi_k); returns (exx, eyy, exy)."""
    ue = u[mesh.tri]                        # (Ne,3,2)
    G = mesh.grad
    exx = (ue[:, :, 0] * G[:, :, 0]).sum(1)
    eyy = (ue[:, :, 1] * G[:, :, 1]).sum(1)
    exy = 0.5 * (ue[:, :, 0] * G[:, :, 1] + ue[:, :, 1] * G[:, :, 0]).sum(1)
    return exx, eyy, exy


def element_forces(mesh: Mesh, sxx, syy, sxy) -> torch.Tensor:
    """f^e_k = A_e sigma grad phi_k, shape (Ne,3,2)."""
    G = mesh.grad
    A = mesh.area[:, None]
    fx = A * (sxx[:, None] * G[:, :, 0] + sxy[:, None] * G[:, :, 1])
    fy = A * (sxy[:, None] * G[:, :, 0] + syy[:, None] * G[:, :, 1])
    return torch.stack([fx, fy], 2)


def internal_force(mesh: Mesh, sxx, syy, sxy) -> torch.Tensor:
    """Scatter-add the element forces into the global internal force (N,2)."""
    fe = element_forces(mesh, sxx, syy, sxy)
    f = torch.zeros((mesh.n_nodes, 2), dtype=fe.dtype)
    return f.index_add(0, mesh.tri.reshape(-1), fe.reshape(-1, 2))

"""Pins of the oracle's P1 geometry, mass and internal force (Sec. 2.3)."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.constitutive import split_energy
from oracle.fem import element_strain, h_min, internal_force, lumped_mass, make_mesh
from oracle.damage import mass_matrix, stiffness_matrix
from tests._helpers import rel
from tests.test_oracle_constitutive import hooke_D

E, NU = 32e9, 0.2


def jittered(nx=12, ny=7, jitter=0.2, seed=11, random_diag=True):
    m = w.plate_mesh(nx, ny, 1e-3, jitter, seed, random_diag=random_diag)
    return m, make_mesh(m["xy"], m["tri"])


def test_geometry_against_shape_function_solve():
    """eq. grad_phi against the inverse of [1 x y] at the three vertices, and the area."""
    m, mesh = jittered()
    X = mesh.xy.numpy()[mesh.tri.numpy()]
    for e in range(mesh.n_elems):
        P = np.hstack([np.ones((3, 1)), X[e]])
        C = np.linalg.inv(P)          # column k holds (a, b, c) of phi_k = a + b x + c y
        assert np.allclose(C[1:, :].T, mesh.grad[e].numpy(), rtol=1e-12, atol=1e-9)
        assert abs(abs(np.linalg.det(P)) / 2 - float(mesh.area[e])) < 1e-14 * float(mesh.area[e]) * 10
    assert torch.all(mesh.area > 0)


def test_mesh_identities():
    """P5: sum grad phi = 0, sum m = rho sum A, K 1 = 0, 1'M1 = sum A, unjittered h_min."""
    m, mesh = jittered()
    assert float(mesh.grad.sum(1).abs().max()) < 1e-12 * float(mesh.grad.abs().max())
    rho = 2450.0
    assert abs(float(lumped_mass(mesh, rho).sum()) - rho * float(mesh.area.sum())) < 1e-12 * rho * float(mesh.area.sum())
    K = stiffness_matrix(mesh)
    assert np.abs(K @ np.ones(mesh.n_nodes)).max() < 1e-12 * np.abs(K.diagonal()).max()
    M = mass_matrix(mesh)
    assert abs(np.ones(mesh.n_nodes) @ (M @ np.ones(mesh.n_nodes)) - float(mesh.area.sum())) < 1e-15
    plain = w.plate_mesh(10, 6, 1e-3, 0.0, 0)
    pm = make_mesh(plain["xy"], plain["tri"])
    assert abs(h_min(pm) - (2 - np.sqrt(2)) * 1e-3) < 1e-15


def test_orientation_is_counter_clockwise():
    m, _ = jittered()
    tri = m["tri"].copy()
    tri[::3] = tri[::3][:, [0, 2, 1]]          # flip some triangles clockwise
    mesh = make_mesh(m["xy"], tri)
    X = mesh.xy.numpy()[mesh.tri.numpy()]
    e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
    cross = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    assert np.all(cross > 0)
    bad = m["tri"].copy()
    bad[0] = [bad[0, 0], bad[0, 0], bad[0, 1]]
    with pytest.raises(ValueError):
        make_mesh(m["xy"], bad)


@pytest.mark.parametrize("split", ["none", "spectral", "voldev", "starconvex"])
@pytest.mark.parametrize("plane", ["strain", "stress"])
def test_patch_test(split, plane):
    """P1: an affine displacement gives the same strain in every element and zero interior force."""
    m, mesh = jittered(16, 9, 0.2, 5)
    X = mesh.xy
    eps0 = torch.tensor([[3e-4, 1.2e-4], [1.2e-4, -2e-4]], dtype=torch.float64)
    u = X @ eps0.T + torch.tensor([1e-5, -2e-5], dtype=torch.float64)
    exx, eyy, exy = element_strain(mesh, u)
    assert float((exx - 3e-4).abs().max()) < 1e-14 * 3e-4 * 10
    assert float((eyy + 2e-4).abs().max()) < 1e-14 * 2e-4 * 10
    assert float((exy - 1.2e-4).abs().max()) < 1e-14 * 1.2e-4 * 10
    pp, pm, sp, sm = split_energy(exx, eyy, exy, E, NU, plane, split, 1.0)
    sig = [sp[i] + sm[i] for i in range(3)]
    f = internal_force(mesh, *sig).numpy()
    ij = m["ij"]
    inner = (ij[:, 0] > 0) & (ij[:, 0] < 16) & (ij[:, 1] > 0) & (ij[:, 1] < 9)
    fe_scale = float(max(s.abs().max() for s in sig)) * float(mesh.area.max()) / 1e-3
    assert np.abs(f[inner]).max() < 1e-12 * fe_scale
    # the boundary force is the traction sigma n integrated along the edge: total is zero
    assert np.abs(f.sum(0)).max() < 1e-12 * fe_scale * mesh.n_nodes


def test_cst_stiffness_textbook():
    """P4: with no split the internal force is K_CST u, K_CST = A B' D B (textbook CST)."""
    m, mesh = jittered(6, 4, 0.2, 9)
    r = np.random.default_rng(0)
    u = torch.tensor(r.normal(size=(mesh.n_nodes, 2)) * 1e-6)
    for plane in ("strain", "stress"):
        exx, eyy, exy = element_strain(mesh, u)
        pp, pm, sp, sm = split_energy(exx, eyy, exy, E, NU, plane, "none")
        f = internal_force(mesh, *sp).numpy()
        D = hooke_D(E, NU, plane)
        fref = np.zeros((mesh.n_nodes, 2))
        X = mesh.xy.numpy()
        for e, t in enumerate(mesh.tri.numpy()):
            P = np.hstack([np.ones((3, 1)), X[t]])
            C = np.linalg.inv(P)
            b, c = C[1], C[2]
            B = np.zeros((3, 6))
            B[0, 0::2] = b
            B[1, 1::2] = c
            B[2, 0::2] = c
            B[2, 1::2] = b
            A = abs(np.linalg.det(P)) / 2
            ue = u.numpy()[t].ravel()
            fe = A * B.T @ D @ B @ ue
            fref[t] += fe.reshape(3, 2)
        assert rel(f, fref) < 1e-12


def test_internal_force_is_linear_without_split():
    """P6: with psi+ = psi and d fixed, f(u + p) - f(u) = f(p) and f(0) = 0."""
    m, mesh = jittered(8, 5, 0.2, 3)
    r = np.random.default_rng(1)
    u = torch.tensor(r.normal(size=(mesh.n_nodes, 2)) * 1e-6)
    p = torch.tensor(r.normal(size=(mesh.n_nodes, 2)) * 1e-6)
    d = torch.tensor(r.uniform(0, 1, mesh.n_nodes))
    g = (1 - d[mesh.tri].mean(1)) ** 2 + 1e-7

    def f(v):
        exx, eyy, exy = element_strain(mesh, v)
        _, _, sp, _ = split_energy(exx, eyy, exy, E, NU, "strain", "none")
        return internal_force(mesh, *[g * s for s in sp])
    assert float(f(torch.zeros_like(u)).abs().max()) == 0.0
    assert rel((f(u + p) - f(u)).numpy(), f(p).numpy()) < 1e-10

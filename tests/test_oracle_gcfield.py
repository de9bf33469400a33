"""Pins of the oracle's spatially varying toughness G_c,e = G_c phi_e (the
per-element G_c(x) inverse problem named in Sec. 4)."""
import numpy as np
import pytest

import workloads as w
from oracle.damage import DamageQP, assemble_damage, energies, mass_matrix, stiffness_matrix
from oracle.step import Sim, initial_state, loss_and_field_derivative, run
from tests._helpers import rel
from tests.test_oracle_damage import GC, L0, mesh_of, quadrature_system


def quadrature_system_field(mesh, H, gce, l0, model):
    """Element-by-element quadrature assembly with each element's own toughness."""
    n = mesh.n_nodes
    A = np.zeros((n, n))
    b = np.zeros(n)
    for e in range(mesh.n_elems):
        # a one-element mesh carries the element's contribution
        sub = type("M", (), {})()
        sub.n_nodes, sub.xy, sub.tri = n, mesh.xy, mesh.tri[e:e + 1]
        Ae, be = quadrature_system(sub, H[e:e + 1], gce[e], l0, model)
        A += Ae
        b += be
    return A, b


@pytest.mark.parametrize("model", [1, 2])
def test_field_assembly_against_quadrature(model):
    """Every G_c of an element's weak form becomes that element's G_c,e."""
    m, mesh = mesh_of(6, 4, 2.5e-4, 0.2, 4, random_diag=True)
    r = np.random.default_rng(2)
    H = r.uniform(0, 5000, mesh.n_elems)
    phi = r.uniform(0.3, 2.5, mesh.n_elems)
    A, b = assemble_damage(mesh, H, GC, L0, model, phi=phi)
    Aq, bq = quadrature_system_field(mesh, H, GC * phi, L0, model)
    assert rel(A.toarray(), Aq) < 1e-13
    assert rel(b, bq) < 1e-13


@pytest.mark.parametrize("model", [1, 2])
def test_uniform_field_is_the_scalar_toughness(model):
    m, mesh = mesh_of(5, 4, 2.5e-4, 0.1, 1)
    H = np.random.default_rng(0).uniform(0, 3000, mesh.n_elems)
    A1, b1 = assemble_damage(mesh, H, GC, L0, model, phi=np.full(mesh.n_elems, 1.7))
    A2, b2 = assemble_damage(mesh, H, 1.7 * GC, L0, model)
    assert rel(A1.toarray(), A2.toarray()) < 1e-15 and rel(b1, b2) < 1e-15


def test_field_tangent_by_finite_differences():
    """Implicit rule along a change of the element toughness field."""
    m, mesh = mesh_of(6, 4, 2.5e-4, 0.2, 8, random_diag=True)
    r = np.random.default_rng(5)
    for model in (1, 2):
        qp = DamageQP(mesh, L0, model)
        H = r.uniform(0, 4000, mesh.n_elems)
        lb = np.where(r.random(mesh.n_nodes) < 0.3, r.uniform(0, 0.4, mesh.n_nodes), 0.0)
        phi = r.uniform(0.5, 2.0, mesh.n_elems)
        dphi = r.normal(size=mesh.n_elems) * 0.2
        d, act, upper, x, A = qp.solve(H, GC, lb, phi)
        t = qp.tangent(A, x, act, upper, H, GC, np.zeros(mesh.n_elems), 0.0, np.zeros(mesh.n_nodes), phi, dphi)
        eps = 1e-6
        dp = qp.solve(H, GC, lb, phi + eps * dphi)[0]
        dm = qp.solve(H, GC, lb, phi - eps * dphi)[0]
        fd = (dp - dm) / (2 * eps)
        assert np.abs(t).max() > 0
        assert np.max(np.abs(fd - t)) < 1e-6 * max(1.0, np.abs(t).max())


def test_field_energy_is_linear_in_the_field():
    """E_frac is a sum of element terms, each proportional to G_c,e."""
    m, mesh = mesh_of(5, 4, 2.5e-4, 0.1, 2)
    r = np.random.default_rng(1)
    d = r.uniform(0, 1, mesh.n_nodes)
    v = np.zeros((mesh.n_nodes, 2))
    mass = np.ones(mesh.n_nodes)
    psi = np.zeros(mesh.n_elems)
    p1, p2 = r.uniform(0.2, 2, mesh.n_elems), r.uniform(0.2, 2, mesh.n_elems)
    for model in (1, 2):
        e = lambda phi: energies(mesh, mass, v, psi, d, GC, L0, model, phi=phi)[2]
        assert abs(e(p1 + 2 * p2) - (e(p1) + 2 * e(p2))) < 1e-13 * abs(e(p1 + 2 * p2))
        assert abs(e(np.full(mesh.n_elems, 1.3)) - 1.3 * energies(mesh, mass, v, psi, d, GC, L0, model)[2]) \
            < 1e-14 * abs(e(p1))
        # a field that is 1 on some elements and 0 elsewhere counts those elements only
        sel = np.zeros(mesh.n_elems)
        sel[: mesh.n_elems // 2] = 1.0
        assert abs(e(sel) + e(1.0 - sel) - e(np.ones(mesh.n_elems))) < 1e-13 * abs(e(np.ones(mesh.n_elems)))


def test_uniform_field_trajectory_equals_scalar():
    p = w.small_plate(12, 6, seed=3).with_(steps=20)
    a, _, _ = run(p, steps=20, Gc=2.0 * p.Gc)
    sim = Sim(p, gc_scale=np.full(len(p.tri), 2.0))
    b, _, _ = run(p, steps=20, sim=sim)
    for k in ("u", "v", "d", "H"):
        assert rel(a.numpy()[k], b.numpy()[k]) < 1e-12, k


@pytest.mark.parametrize("model,split", [(2, "spectral"), (1, "voldev")])
def test_field_directional_derivative_against_central_differences(model, split):
    """Forward-mode derivative of the loss along a toughness-field direction against
    central differences (the step stays within one smooth piece of the trajectory)."""
    p = w.small_plate(16, 8, model=model, split=split, seed=5).with_(steps=30)
    r = np.random.default_rng(7)
    ne = len(p.tri)
    st, _, _ = run(p, steps=30)
    target = st.d.numpy()
    phi = r.uniform(0.6, 1.4, ne)
    direc = r.normal(size=ne) * p.Gc
    L, dL, _ = loss_and_field_derivative(p, target, p.Gc, phi, direc, steps=30)
    h = 1e-7
    Lp = loss_and_field_derivative(p, target, p.Gc, phi + h * direc / p.Gc, direc, steps=30)[0]
    Lm = loss_and_field_derivative(p, target, p.Gc, phi - h * direc / p.Gc, direc, steps=30)[0]
    fd = (Lp - Lm) / (2 * h)
    assert L > 0 and abs(dL) > 0
    assert abs(fd - dL) / abs(dL) < 1e-5

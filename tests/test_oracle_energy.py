"""Pins of the oracle's energy budget and wave speeds (Sec. 2.1, Sec. 2.3, energy histories of Sec. 3).

Each energy is checked against a value fixed by something other than the
oracle's own formula: the plate's exact area, the textbook plane-strain /
plane-stress stiffness, an independent quadrature assembly of the damage
functional, and the regularised functional's limit, the fracture energy
G_c times the crack length (Sec. 2.1).
"""
import math

import numpy as np
import pytest
import torch

import workloads as w
from oracle.constitutive import wave_speed
from oracle.damage import DamageQP, energies
from oracle.fem import lumped_mass, make_mesh
from oracle.step import Sim, State
from tests.test_oracle_constitutive import hooke_D
from tests.test_oracle_damage import quadrature_system

GC, L0 = 3.0, 5e-4
SPLITS = ["none", "spectral", "voldev", "starconvex"]


def plate(nx=14, ny=9, jitter=0.2, seed=5, **kw):
    args = dict(random_diag=True)
    args.update(kw)
    return w.small_plate(nx, ny, jitter=jitter, seed=seed, **args)


def state(p, u=None, v=None, d=None):
    n, ne = p.n_nodes, p.n_elems
    f = lambda x, shape: torch.zeros(shape, dtype=torch.float64) if x is None else \
        torch.as_tensor(np.asarray(x, dtype=np.float64)).clone()
    return State(f(u, (n, 2)), f(v, (n, 2)), torch.zeros((n, 2), dtype=torch.float64), f(d, (n,)),
                 torch.zeros(ne, dtype=torch.float64))


def plate_area(p):
    """Jitter moves boundary nodes only along the boundary and keeps the corners, so the
    meshed area is the rectangle's."""
    return p.meta["nx"] * p.meta["h"] * p.meta["ny"] * p.meta["h"]


def test_kinetic_energy_of_a_uniform_velocity():
    """E_kin = 1/2 rho |v|^2 times the plate area: the lumped masses add up to rho A."""
    p = plate()
    sim = Sim(p)
    v = np.array([0.7, -1.3])
    ek, _, _ = sim.energies(state(p, v=np.tile(v, (p.n_nodes, 1))))
    assert abs(ek - 0.5 * p.rho * plate_area(p) * float(v @ v)) <= 1e-13 * ek


def test_kinetic_energy_of_one_moving_node():
    """One node moving: E_kin = 1/2 m_i |v_i|^2 with m_i = rho sum A_e/3 over the triangles
    around i, the areas taken by the shoelace formula."""
    p = plate()
    sim = Sim(p)
    i = int(np.argmin(np.abs(p.xy[:, 0] - p.xy[:, 0].mean()) + np.abs(p.xy[:, 1] - p.xy[:, 1].mean())))
    v = np.zeros((p.n_nodes, 2))
    v[i] = (2.0, 0.5)
    m_i = 0.0
    for t in p.tri:
        if i in t:
            (x0, y0), (x1, y1), (x2, y2) = p.xy[t]
            m_i += p.rho * abs((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)) / 2 / 3
    ek, _, _ = sim.energies(state(p, v=v))
    assert abs(ek - 0.5 * m_i * 4.25) <= 1e-13 * ek


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("plane", ["strain", "stress"])
def test_elastic_energy_of_an_affine_field(split, plane):
    """Undamaged (d = 0, eta = 0): u = eps0 x gives E_el = A * 1/2 eps0' D eps0 for every split,
    with the textbook D and the exact plate area."""
    p = plate(split=split, plane=plane, gamma_star=0.6).with_(eta=0.0)
    sim = Sim(p)
    for eps in ([1.1e-4, -0.4e-4, 0.3e-4], [-2e-4, -1e-4, 0.5e-4], [0.5e-4, 0.8e-4, -0.2e-4]):
        exx, eyy, exy = eps
        u = np.stack([exx * p.xy[:, 0] + exy * p.xy[:, 1], exy * p.xy[:, 0] + eyy * p.xy[:, 1]], 1)
        _, ee, _ = sim.energies(state(p, u=u))
        vgt = np.array([exx, eyy, 2 * exy])
        ref = plate_area(p) * 0.5 * vgt @ hooke_D(p.E, p.nu, plane) @ vgt
        assert abs(ee - ref) <= 1e-12 * ref, (split, plane, eps)


@pytest.mark.parametrize("plane", ["strain", "stress"])
def test_elastic_energy_of_a_broken_plate(plane):
    """Fully damaged (d = 1, so g = eta), spectral split: a tensile affine field keeps only
    eta psi; a compressive one keeps all of psi (psi+ = 0)."""
    p = plate(split="spectral", plane=plane)
    sim = Sim(p)
    D = hooke_D(p.E, p.nu, plane)
    ones = np.ones(p.n_nodes)
    for eps, factor in (([1e-4, 0.6e-4, 0.2e-4], p.eta), ([-1e-4, -0.6e-4, 0.2e-4], 1.0)):
        exx, eyy, exy = eps
        u = np.stack([exx * p.xy[:, 0] + exy * p.xy[:, 1], exy * p.xy[:, 0] + eyy * p.xy[:, 1]], 1)
        _, ee, _ = sim.energies(state(p, u=u, d=ones))
        vgt = np.array([exx, eyy, 2 * exy])
        ref = factor * plate_area(p) * 0.5 * vgt @ D @ vgt
        assert abs(ee - ref) <= 1e-12 * ref, (plane, eps)


@pytest.mark.parametrize("model", [1, 2])
@pytest.mark.parametrize("field", [False, True])
def test_fracture_energy_is_the_damage_functional(model, field):
    """With H = 0 the damage programme's objective is the fracture energy:
    AT2 E_frac = 1/2 d'Ad, AT1 E_frac = 1/2 d'Ad - b'd, with A and b from an
    independent edge-midpoint quadrature of the weak form (per element G_c,e = G_c phi_e)."""
    p = plate(model=model)
    mesh = make_mesh(p.xy, p.tri)
    r = np.random.default_rng(11)
    d = r.uniform(0, 1, p.n_nodes)
    phi = r.uniform(0.5, 1.5, p.n_elems) if field else None
    A, b = quadrature_system(mesh, np.zeros(p.n_elems), GC if phi is None else GC * phi, L0, model)
    ref = 0.5 * d @ A @ d - (0.0 if model == 2 else b @ d)
    _, _, ef = energies(mesh, lumped_mass(mesh, 1.0).numpy(), np.zeros((p.n_nodes, 2)), np.zeros(p.n_elems),
                        d, GC, L0, model, phi=phi)
    assert abs(ef - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("model", [1, 2])
def test_fracture_energy_of_a_crack_tends_to_gc_times_length(model):
    """A full-width crack row (d_prev = 1) across an unjittered plate, H = 0: the damage
    programme's minimiser is the regularised crack, and its fracture energy tends to
    G_c times the crack length (Sec. 2.1) as h/l0 -> 0.

    The continuum AT2 profile on a strip of half-height L is cosh((L - y)/l0)/cosh(L/l0)
    with energy G_c W tanh(L/l0) over both sides; AT1 reaches G_c W exactly.  P1
    elements approach it from above at second order in h/l0."""
    errs = []
    for ratio in (2, 4, 8):
        h = L0 / ratio
        N, nx = 12 * ratio, 40 * ratio
        m = w.plate_mesh(nx, 2 * N, h, 0.0, 0)
        mesh = make_mesh(m["xy"], m["tri"])
        lb = np.where(m["ij"][:, 1] == N, 1.0, 0.0)
        d = DamageQP(mesh, L0, model).solve(np.zeros(mesh.n_elems), GC, lb)[0]
        _, _, ef = energies(mesh, lumped_mass(mesh, 1.0).numpy(), np.zeros((mesh.n_nodes, 2)),
                            np.zeros(mesh.n_elems), d, GC, L0, model)
        limit = GC * nx * h * (math.tanh(N * h / L0) if model == 2 else 1.0)
        errs.append(ef / limit - 1.0)
        assert 0.0 < errs[-1] < 0.05 / ratio ** 2, (model, ratio, errs[-1])
    assert all(3.5 < errs[k] / errs[k + 1] < 4.5 for k in range(2)), errs


@pytest.mark.parametrize("nu", [0.0, 0.2, 0.35, 0.45])
def test_dilatational_wave_speed_closed_forms(nu):
    """c_p of the 2D media: plane strain sqrt(E (1-nu) / (rho (1+nu)(1-2nu))),
    plane stress sqrt(E / (rho (1 - nu^2)))."""
    E, rho = 32e9, 2450.0
    ps = math.sqrt(E / (rho * (1 - nu * nu)))
    pe = math.sqrt(E * (1 - nu) / (rho * (1 + nu) * (1 - 2 * nu)))
    assert abs(wave_speed(E, nu, rho, "stress") - ps) <= 1e-14 * ps
    assert abs(wave_speed(E, nu, rho, "strain") - pe) <= 1e-14 * pe

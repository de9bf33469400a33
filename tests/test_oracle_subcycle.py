"""Oracle pins for damage subcycling (Sec. 2.3): the Rayleigh speed behind N_max, and the schedule."""
import math

import numpy as np
import pytest
import torch

import workloads as w
from oracle.constitutive import rayleigh_speed, shear_wave_speed, subcycle_limit, wave_speed
from oracle.damage import DamageQP
from oracle.step import Sim, initial_state, run
from tests._helpers import golden

E, RHO = 32e9, 2450.0


def test_rayleigh_poisson_solid_closed_form():
    """nu = 1/4 in plane strain (lambda = mu): c_R / c_s = sqrt(2 - 2/sqrt(3)), a textbook closed form."""
    xi = rayleigh_speed(E, 0.25, RHO, "strain") / shear_wave_speed(E, 0.25, RHO)
    assert abs(xi - math.sqrt(2.0 - 2.0 / math.sqrt(3.0))) < 1e-13


@pytest.mark.parametrize("plane", ["strain", "stress"])
@pytest.mark.parametrize("nu", [0.05, 0.2, 0.3, 0.35, 0.45])
def test_rayleigh_matches_rationalised_cubic(nu, plane):
    """Squaring the Rayleigh equation gives eta^3 - 8 eta^2 + (24 - 16 k) eta - 16 (1 - k) = 0
    in eta = xi^2; its root in (0, 1), from numpy.roots, must equal the bisection root."""
    cs, cp = shear_wave_speed(E, nu, RHO), wave_speed(E, nu, RHO, plane)
    k = (cs / cp) ** 2
    roots = np.roots([1.0, -8.0, 24.0 - 16.0 * k, -16.0 * (1.0 - k)])
    eta = [r.real for r in roots if abs(r.imag) < 1e-12 and 0.0 < r.real < 1.0]
    assert len(eta) == 1
    assert abs(rayleigh_speed(E, nu, RHO, plane) / cs - math.sqrt(eta[0])) < 1e-12


@pytest.mark.parametrize("nu", [0.1, 0.2, 0.3, 0.4, 0.45])
def test_rayleigh_viktorov_approximation(nu):
    """The classical approximation (0.862 + 1.14 nu)/(1 + nu) is within 1 % (plane strain)."""
    xi = rayleigh_speed(E, nu, RHO, "strain") / shear_wave_speed(E, nu, RHO)
    assert abs(xi - (0.862 + 1.14 * nu) / (1.0 + nu)) < 1e-2 * xi


def test_rayleigh_textbook_limits():
    """Plane strain: nu = 0 gives c_R/c_s = 0.8740, the incompressible limit 0.9553."""
    assert abs(rayleigh_speed(E, 0.0, RHO, "strain") / shear_wave_speed(E, 0.0, RHO) - 0.8740) < 1e-4
    nu = 0.4999999
    assert abs(rayleigh_speed(E, nu, RHO, "strain") / shear_wave_speed(E, nu, RHO) - 0.9553) < 1e-4


def test_subcycle_limit_paper_pmma():
    g = golden("paper_constants.txt")
    for plane in ("strain", "stress"):
        assert subcycle_limit(E, g["pmma_nu"], RHO, plane) == int(g["pmma_n_max"])


def test_subcycling_schedule_and_history():
    """n_sub = 3: d changes only on steps 3, 6, ...; each of those equals the exact damage QP for
    (H of that step, d of the last solve); H never decreases and moves on the skipped steps too."""
    p = w.small_plate(24, 12, seed=4).with_(steps=12)
    sim = Sim(p)
    st = initial_state(p)
    last_d = st.d.clone()
    h_moved_on_skip = False
    for k in range(12):
        solve = (k + 1) % 3 == 0
        nxt = sim.step(st, solve=solve)
        assert torch.all(nxt.H >= st.H)
        if solve:
            d_ref, _, _ = sim.damage(nxt.H, last_d, p.Gc)
            assert torch.equal(nxt.d, d_ref)
            last_d = nxt.d.clone()
        else:
            assert torch.equal(nxt.d, st.d)
            h_moved_on_skip |= bool(torch.any(nxt.H > st.H))
        st = nxt
    assert h_moved_on_skip


def test_subcycling_one_is_the_plain_scheme():
    p = w.small_plate(16, 8, seed=2).with_(steps=6)
    a, _, _ = run(p, steps=6)
    b, _, _ = run(p, steps=6, n_sub=1)
    for f in ("u", "v", "a", "d", "H"):
        assert torch.equal(getattr(a, f), getattr(b, f))

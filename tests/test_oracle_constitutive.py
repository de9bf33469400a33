"""Pins of the oracle's constitutive law against textbook forms (Sec. 2.1)."""
import numpy as np
import pytest
import torch

from oracle.constitutive import elastic_constants, split_energy
from tests._helpers import golden, rel

E, NU = 32e9, 0.2
SPLITS = ["none", "spectral", "voldev", "starconvex"]
PLANES = ["strain", "stress"]


def hooke_D(E, nu, plane):
    """Textbook plane strain / plane stress matrix for (exx, eyy, gamma_xy = 2 exy)."""
    if plane == "strain":
        f = E / ((1 + nu) * (1 - 2 * nu))
        return f * np.array([[1 - nu, nu, 0], [nu, 1 - nu, 0], [0, 0, (1 - 2 * nu) / 2]])
    f = E / (1 - nu * nu)
    return f * np.array([[1, nu, 0], [nu, 1, 0], [0, 0, (1 - nu) / 2]])


def strains(n=100000, seed=0):
    r = np.random.default_rng(seed)
    e = r.normal(size=(n, 3)) * 1e-3
    special = np.array([
        [1e-3, 1e-3, 0.0],      # equal principal strains
        [-1e-3, -1e-3, 0.0],
        [1e-3, -1e-3, 0.0],     # trace zero
        [0.0, 0.0, 1e-3],       # pure shear
        [0.0, 0.0, 0.0],
        [2e-3, 0.0, 0.0],       # one principal strain zero
        [-2e-3, 0.0, 0.0],
    ])
    e = np.vstack([special, e])
    return [torch.tensor(e[:, k]) for k in range(3)]


def energy_textbook(exx, eyy, exy, plane):
    D = hooke_D(E, NU, plane)
    v = np.stack([exx.numpy(), eyy.numpy(), 2 * exy.numpy()], 1)
    return 0.5 * np.einsum("ni,ij,nj->n", v, D, v)


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("plane", PLANES)
def test_split_sums_to_plane_energy(split, plane):
    """P2: psi+ + psi- equals the undamaged plane energy 1/2 eps:C:eps."""
    exx, eyy, exy = strains()
    pp, pm, _, _ = split_energy(exx, eyy, exy, E, NU, plane, split, gamma_star=1.0)
    ref = energy_textbook(exx, eyy, exy, plane)
    err = np.abs((pp + pm).numpy() - ref) / np.maximum(np.abs(ref), 1e-30)
    assert err[np.abs(ref) > 0].max() < 1e-13
    assert np.all(np.abs((pp + pm).numpy()[ref == 0]) == 0)


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("plane", PLANES)
def test_stress_is_energy_derivative(split, plane):
    """P3: sigma+- = d psi+- / d eps by central differences, away from kinks."""
    exx, eyy, exy = strains(2000, seed=1)
    h = 1e-9
    pp, pm, sp, sm = split_energy(exx, eyy, exy, E, NU, plane, split, gamma_star=1.0)
    for which, sig in ((0, sp), (1, sm)):
        for comp in range(3):
            dv = [torch.zeros_like(exx) for _ in range(3)]
            dv[comp] = torch.full_like(exx, h)
            up = split_energy(exx + dv[0], eyy + dv[1], exy + dv[2], E, NU, plane, split, 1.0)[which]
            dn = split_energy(exx - dv[0], eyy - dv[1], exy - dv[2], E, NU, plane, split, 1.0)[which]
            fd = ((up - dn) / (2 * h)).numpy()
            an = sig[comp].numpy() * (2.0 if comp == 2 else 1.0)   # d psi / d exy = 2 sigma_xy
            scale = np.abs(np.stack([s.numpy() for s in sig])).max(0) + 1e3
            err = np.abs(fd - an) / scale
            assert np.median(err) < 1e-6 and np.quantile(err, 0.99) < 1e-5, (which, comp, err.max())


@pytest.mark.parametrize("plane", PLANES)
def test_spectral_matches_eigendecomposition(plane):
    """Spectral split against numpy.linalg.eigh: E+ = sum <e_a>+ n_a n_a'."""
    exx, eyy, exy = strains(5000, seed=2)
    k = elastic_constants(E, NU, plane)
    pp, pm, sp, sm = split_energy(exx, eyy, exy, E, NU, plane, "spectral")
    T = np.stack([np.stack([exx, exy], 1), np.stack([exy, eyy], 1)], 1)
    w, V = np.linalg.eigh(T)
    Ep = np.einsum("na,nia,nja->nij", np.maximum(w, 0), V, V)
    tr = w.sum(1)
    psi_p = 0.5 * k["lam"] * np.maximum(tr, 0) ** 2 + k["mu"] * (np.maximum(w, 0) ** 2).sum(1)
    sig_p = k["lam"] * np.maximum(tr, 0)[:, None, None] * np.eye(2) + 2 * k["mu"] * Ep
    assert rel(pp.numpy(), psi_p) < 1e-13
    assert rel(sp[0].numpy(), sig_p[:, 0, 0]) < 1e-12
    assert rel(sp[1].numpy(), sig_p[:, 1, 1]) < 1e-12
    assert rel(sp[2].numpy(), sig_p[:, 0, 1]) < 1e-12


def test_special_cases():
    """P4: branch identities of the splits."""
    exx, eyy, exy = strains(20000, seed=3)
    tr = (exx + eyy).numpy()
    for plane in PLANES:
        k = elastic_constants(E, NU, plane)
        ref = energy_textbook(exx, eyy, exy, plane)
        # spectral: both principal strains >= 0 -> psi+ = psi
        pp, pm, _, _ = split_energy(exx, eyy, exy, E, NU, plane, "spectral")
        T = np.stack([np.stack([exx, exy], 1), np.stack([exy, eyy], 1)], 1)
        wmin = np.linalg.eigvalsh(T)[:, 0]
        m = wmin > 1e-12
        assert rel(pp.numpy()[m], ref[m]) < 1e-13 and np.all(pm.numpy()[m] == 0)
        # vol-dev: compression -> psi- = K/2 (c tr)^2 with K = E / (3 (1 - 2 nu))
        Kb = E / (3 * (1 - 2 * NU))
        c = 1.0 if plane == "strain" else (1 - 2 * NU) / (1 - NU)
        pp, pm, _, _ = split_energy(exx, eyy, exy, E, NU, plane, "voldev")
        neg = tr < 0
        assert rel(pm.numpy()[neg], 0.5 * Kb * (c * tr[neg]) ** 2) < 1e-13
        assert np.all(pm.numpy()[~neg] == 0)
        # star-convex: psi- = (1 + gamma) K/2 (c tr)^2 in compression
        g = 0.7
        pp2, pm2, _, _ = split_energy(exx, eyy, exy, E, NU, plane, "starconvex", gamma_star=g)
        assert rel(pm2.numpy()[neg], (1 + g) * 0.5 * Kb * (c * tr[neg]) ** 2) < 1e-13
        # star-convex with gamma = 0 is vol-dev, bit for bit
        out0 = split_energy(exx, eyy, exy, E, NU, plane, "starconvex", gamma_star=0.0)
        out1 = split_energy(exx, eyy, exy, E, NU, plane, "voldev")
        assert torch.equal(out0[0], out1[0]) and torch.equal(out0[1], out1[1])
        for a, b in zip(out0[2] + out0[3], out1[2] + out1[3]):
            assert torch.equal(a, b)


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("plane", PLANES)
def test_undamaged_stress_is_hooke(split, plane):
    """sigma+ + sigma- equals the textbook plane Hooke law for every split."""
    exx, eyy, exy = strains(5000, seed=4)
    _, _, sp, sm = split_energy(exx, eyy, exy, E, NU, plane, split, gamma_star=1.0)
    D = hooke_D(E, NU, plane)
    v = np.stack([exx.numpy(), eyy.numpy(), 2 * exy.numpy()], 1)
    s = v @ D.T
    got = np.stack([(sp[i] + sm[i]).numpy() for i in range(3)], 1)
    assert rel(got, s) < 1e-12


def test_paper_constants_and_threshold():
    """Printed parameters (Table 'benchmark overview', Sec. 2.1) and the AT1 threshold identity.

    A uniaxial stress sigma_c = sqrt(3 Gc E/(8 l0)) stores psi = sigma_c^2/(2E), which is
    the AT1 threshold 3 Gc/(16 l0): the two printed formulas agree.
    """
    g = golden("paper_constants.txt")
    assert g["eta"] == 1e-7
    Gc = g["glass_Gc_N_per_mm"] * 1e3       # N/mm -> J/m^2
    l0 = g["glass_l0_mm"] * 1e-3
    sigma_c = np.sqrt(3 * Gc * g["glass_E_Pa"] / (8 * l0))
    assert abs(sigma_c ** 2 / (2 * g["glass_E_Pa"]) - 3 * Gc / (16 * l0)) < 1e-9
    # lambda_PE and lambda_PS of Sec. 2.1 against the textbook D matrices
    for plane in PLANES:
        k = elastic_constants(g["glass_E_Pa"], g["glass_nu"], plane)
        D = hooke_D(g["glass_E_Pa"], g["glass_nu"], plane)
        assert abs(D[0, 1] - k["lam"]) < 1e-6 * k["lam"]
        assert abs(D[2, 2] - k["mu"]) < 1e-6 * k["mu"]

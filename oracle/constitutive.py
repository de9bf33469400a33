"""Elastic constants and energy splits (Sec. 2.1, eq. spectral_split, eq. amor_split).

Oracle: test infrastructure only.

Strains are passed as the three independent components (exx, eyy, exy) of
the symmetric 2x2 tensor; stresses are returned the same way.  All
functions are plain torch float64 expressions so that forward-mode
differentiation passes through them.

Readings of the paper used here:
* plane stress for the volumetric-deviatoric and star-convex splits: the
  out-of-plane strain s*tr with s = -nu/(1-nu) enters the 3D trace
  c*tr (c = 1 + s) and the deviatoric norm; the stress is the exact
  derivative of that energy with respect to the in-plane strain;
* the spectral split under plane stress uses lambda_PS and the 2D principal
  strains (the plane choice only changes the first Lame parameter);
* star-convex: psi+ = K/2 c^2 (<tr>+^2 - gamma <tr>-^2) + mu*dev:dev,
  psi- = (1+gamma) K/2 c^2 <tr>-^2; gamma = 0 is the vol-dev split;
* Macaulay brackets <x>+ = x if x > 0 else 0 (derivative 0 at x = 0).
"""
from __future__ import annotations

import math

import torch


def elastic_constants(E: float, nu: float, plane: str) -> dict:
    """Lame parameters, 3D bulk modulus and plane-stress trace factors (Sec. 2.1, plane assumptions)."""
    mu = E / (2.0 * (1.0 + nu))
    lam_pe = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    lam_ps = E * nu / (1.0 - nu * nu)
    K = E / (3.0 * (1.0 - 2.0 * nu))
    if plane == "strain":
        lam, s = lam_pe, 0.0
    elif plane == "stress":
        lam, s = lam_ps, -nu / (1.0 - nu)
    else:
        raise ValueError(plane)
    c = 1.0 + s
    return {"mu": mu, "lam": lam, "lam_pe": lam_pe, "lam_ps": lam_ps, "K": K, "s": s, "c": c}


def wave_speed(E: float, nu: float, rho: float, plane: str) -> float:
    """Dilatational wave speed c_p = sqrt((lambda + 2 mu)/rho) with the plane's lambda (Sec. 2.3)."""
    k = elastic_constants(E, nu, plane)
    return math.sqrt((k["lam"] + 2.0 * k["mu"]) / rho)


def shear_wave_speed(E: float, nu: float, rho: float) -> float:
    """Shear wave speed c_s = sqrt(mu/rho) (the same in both plane assumptions)."""
    return math.sqrt(elastic_constants(E, nu, "strain")["mu"] / rho)


def rayleigh_speed(E: float, nu: float, rho: float, plane: str) -> float:
    """Rayleigh surface-wave speed c_R of the plane's 2D elastic medium.

    c_R = xi c_s, where xi in (0, 1) is the root of the Rayleigh equation
        (2 - xi^2)^2 = 4 sqrt(1 - xi^2) sqrt(1 - kappa xi^2),  kappa = c_s^2 / c_p^2,
    with c_p the plane's dilatational speed.  Found by bisection: the function
    f(xi) = (2 - xi^2)^2 - 4 sqrt(1 - xi^2) sqrt(1 - kappa xi^2) behaves like
    -2 (1 - kappa) xi^2 < 0 near 0 and equals 1 at xi = 1; its one root in
    (0, 1) (besides xi = 0) lies above 0.5 for 0 < kappa < 1/2.
    """
    cs = shear_wave_speed(E, nu, rho)
    cp = wave_speed(E, nu, rho, plane)
    kappa = (cs / cp) ** 2

    def f(x):
        return (2.0 - x * x) ** 2 - 4.0 * math.sqrt(1.0 - x * x) * math.sqrt(1.0 - kappa * x * x)

    lo, hi = 0.5, 1.0
    assert f(lo) < 0.0 < f(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-16:
            break
    return 0.5 * (lo + hi) * cs


def subcycle_limit(E: float, nu: float, rho: float, plane: str) -> int:
    """Largest admissible damage subcycling factor N_max = floor(c_p / (0.6 c_R)) (Sec. 2.3, subcycling)."""
    return int(math.floor(wave_speed(E, nu, rho, plane) / (0.6 * rayleigh_speed(E, nu, rho, plane))))


def _pos(x):
    return torch.where(x > 0, x, torch.zeros_like(x))


def _neg(x):
    return torch.where(x < 0, x, torch.zeros_like(x))


def _split_none(exx, eyy, exy, k):
    lam, mu = k["lam"], k["mu"]
    tr = exx + eyy
    ee = exx * exx + eyy * eyy + 2.0 * exy * exy
    psi_p = 0.5 * lam * tr * tr + mu * ee
    z = torch.zeros_like(exx)
    sp = (lam * tr + 2.0 * mu * exx, lam * tr + 2.0 * mu * eyy, 2.0 * mu * exy)
    return psi_p, z, sp, (z, z, z)


def _split_spectral(exx, eyy, exy, k):
    lam, mu = k["lam"], k["mu"]
    tr = exx + eyy
    hd = 0.5 * (exx - eyy)
    R2 = hd * hd + exy * exy
    has_r = R2 > 0
    R = torch.where(has_r, torch.sqrt(torch.where(has_r, R2, torch.ones_like(R2))), torch.zeros_like(R2))
    e1 = 0.5 * tr + R
    e2 = 0.5 * tr - R
    both_pos = e2 >= 0
    both_neg = e1 <= 0
    mixed = (~both_pos) & (~both_neg)
    # mixed branch: E+ = e1 * (eps - e2 I) / (e1 - e2); there e1 - e2 = 2R > 0
    f = e1 / (2.0 * torch.where(mixed, R, torch.ones_like(R)))
    z = torch.zeros_like(exx)
    Ep = (torch.where(both_pos, exx, torch.where(mixed, f * (exx - e2), z)),
          torch.where(both_pos, eyy, torch.where(mixed, f * (eyy - e2), z)),
          torch.where(both_pos, exy, torch.where(mixed, f * exy, z)))
    Em = (exx - Ep[0], eyy - Ep[1], exy - Ep[2])
    tp, tm = _pos(tr), _neg(tr)
    p1, p2, m1, m2 = _pos(e1), _pos(e2), _neg(e1), _neg(e2)
    psi_p = 0.5 * lam * tp * tp + mu * (p1 * p1 + p2 * p2)
    psi_m = 0.5 * lam * tm * tm + mu * (m1 * m1 + m2 * m2)
    sp = (lam * tp + 2.0 * mu * Ep[0], lam * tp + 2.0 * mu * Ep[1], 2.0 * mu * Ep[2])
    sm = (lam * tm + 2.0 * mu * Em[0], lam * tm + 2.0 * mu * Em[1], 2.0 * mu * Em[2])
    return psi_p, psi_m, sp, sm


def _split_voldev(exx, eyy, exy, k, gamma):
    K, mu, c, s = k["K"], k["mu"], k["c"], k["s"]
    tr = exx + eyy
    tp, tm = _pos(tr), _neg(tr)
    dev = exx * exx + eyy * eyy + 2.0 * exy * exy + (s * s - c * c / 3.0) * tr * tr
    kc2 = K * c * c
    psi_p = 0.5 * kc2 * (tp * tp - gamma * tm * tm) + mu * dev
    psi_m = 0.5 * (1.0 + gamma) * kc2 * tm * tm
    iso = kc2 * (tp - gamma * tm) + 2.0 * mu * (s * s - c * c / 3.0) * tr
    sp = (iso + 2.0 * mu * exx, iso + 2.0 * mu * eyy, 2.0 * mu * exy)
    im = (1.0 + gamma) * kc2 * tm
    z = torch.zeros_like(exx)
    return psi_p, psi_m, sp, (im, im, z)


def split_energy(exx, eyy, exy, E: float, nu: float, plane: str, split: str, gamma_star: float = 1.0):
    """Return (psi+, psi-, sigma+, sigma-) for the chosen split.

    sigma+- = d psi+- / d eps, so the stress is g(d) sigma+ + sigma- (Sec. 2.2).
    """
    k = elastic_constants(E, nu, plane)
    if split == "none":
        return _split_none(exx, eyy, exy, k)
    if split == "spectral":
        return _split_spectral(exx, eyy, exy, k)
    if split == "voldev":
        return _split_voldev(exx, eyy, exy, k, 0.0)
    if split == "starconvex":
        return _split_voldev(exx, eyy, exy, k, gamma_star)
    raise ValueError(split)

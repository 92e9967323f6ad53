"""Independent numerical references used to pin the oracle (test helpers only).

Nothing here re-types the oracle's formulas: the classical two-body
scattering integral and the closest-approach root are evaluated with scipy's
adaptive quadrature and root finder on whatever potential the caller passes
(normally the oracle's own V(r)), and the published closed forms (Rutherford,
Lindhard's reduced electronic stopping, the ZBL universal nuclear stopping fit)
are written from their textbook definitions.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

COULOMB = 14.3996454784  # e^2/(4 pi eps0), eV*A (CODATA 2018)
BOHR = 0.529177210903    # A


def closest_approach(V, Ec, p=0.0, r_hi=50.0):
    """Root of g(r) = 1 - V(r)/Ec - p^2/r^2 (classical turning point).  For a repulsive,
    decreasing V, g increases with r, so the root is unique: bracket it by halving r
    from above, then refine with Brent's method."""
    g = lambda r: 1.0 - V(r) / Ec - (p / r) ** 2
    hi = max(r_hi, 2.0 * p + 10.0)
    while g(hi) <= 0.0:
        hi *= 2.0
    lo = hi
    while g(lo) > 0.0:
        lo *= 0.5
        if lo < 1e-12:
            raise RuntimeError("no turning point")
    return optimize.brentq(g, lo, 2.0 * lo, xtol=1e-15, rtol=1e-15, maxiter=500)


def cm_deflection(V, Ec, p):
    """Centre-of-mass scattering angle from the classical deflection integral
    theta = pi - 2 p int_{r_min}^inf dr / (r^2 sqrt(1 - V/Ec - p^2/r^2)),
    with u = r_min/r and u = 1 - t^2 to remove the turning-point singularity."""
    if p == 0.0:
        return math.pi
    rm = closest_approach(V, Ec, p)

    def f(t):
        u = 1.0 - t * t
        if u <= 0.0:
            return 0.0
        r = rm / u
        g = 1.0 - V(r) / Ec - (p * u / rm) ** 2
        return 2.0 * t / math.sqrt(max(g, 1e-300))

    val, _ = integrate.quad(f, 0.0, 1.0, limit=400, epsabs=1e-13, epsrel=1e-12)
    return math.pi - 2.0 * (p / rm) * val


def lab_angle(theta_cm, M1, M2):
    """Projectile lab deflection for a target initially at rest."""
    return math.atan2(math.sin(theta_cm), math.cos(theta_cm) + M1 / M2)


def rutherford_cm(Z1, Z2, Ec, p):
    """Closed-form Coulomb deflection: tan(theta/2) = b / (2 p), b = Z1 Z2 e^2 / Ec."""
    b = Z1 * Z2 * COULOMB / Ec
    return 2.0 * math.atan(b / (2.0 * p))


def lindhard_kL(Z1, Z2, M1, M2):
    """Lindhard-Scharff electronic stopping S_e = kL sqrt(E) (eV A^2, E in eV), written from
    the reduced-unit form  d eps / d rho = k eps^(1/2),
    k = xi_e 0.0793 Z1^(1/2) Z2^(1/2) (M1+M2)^(3/2) / ((Z1^(2/3)+Z2^(2/3))^(3/4) M1^(3/2) M2^(1/2)),
    xi_e = Z1^(1/6), with Lindhard's units eps = a_L E M2/(Z1 Z2 e^2 (M1+M2)),
    rho = R N 4 pi a_L^2 M1 M2 / (M1+M2)^2, a_L = 0.8853 a0 (Z1^(2/3)+Z2^(2/3))^(-1/2)."""
    k = Z1 ** (1 / 6) * 0.0793 * Z1 ** 0.5 * Z2 ** 0.5 * (M1 + M2) ** 1.5 / (
        (Z1 ** (2 / 3) + Z2 ** (2 / 3)) ** 0.75 * M1 ** 1.5 * M2 ** 0.5)
    aL = 0.8853 * BOHR / math.sqrt(Z1 ** (2 / 3) + Z2 ** (2 / 3))
    c_eps = aL * M2 / (Z1 * Z2 * COULOMB * (M1 + M2))
    c_rho = 4.0 * math.pi * aL ** 2 * M1 * M2 / (M1 + M2) ** 2
    # dE/dR = k sqrt(c_eps E) N c_rho / c_eps, and S_e = (dE/dR) / N
    return k * c_rho / math.sqrt(c_eps)


def zbl_reduced_energy(Z1, Z2, M1, M2, E_eV):
    """ZBL reduced energy as printed with the universal stopping:
    eps = 32.53 M2 E[keV] / (Z1 Z2 (M1+M2) (Z1^0.23 + Z2^0.23))."""
    return 32.53 * M2 * (E_eV / 1000.0) / (Z1 * Z2 * (M1 + M2) * (Z1 ** 0.23 + Z2 ** 0.23))


def zbl_universal_sn(eps):
    """ZBL universal reduced nuclear stopping fit."""
    if eps <= 30.0:
        return math.log(1.0 + 1.1383 * eps) / (
            2.0 * (eps + 0.01321 * eps ** 0.21226 + 0.19593 * eps ** 0.5))
    return math.log(eps) / (2.0 * eps)


def reduced_nuclear_stopping(phi, eps):
    """s_n(eps) = 2 eps int_0^inf sin^2(theta(b)/2) b db for the screened potential
    V(x)/E_c = phi(x) / (x eps) in units of the screening length."""
    Vred = lambda x: phi(x) / x

    def th(b):
        return cm_deflection(Vred, eps, b)

    f = lambda b: math.sin(th(b) / 2.0) ** 2 * b
    edges = [0.0, 0.01, 0.1, 0.5, 1, 2, 4, 8, 16, 32, 64]
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        val, _ = integrate.quad(f, lo, hi, limit=200, epsrel=1e-9)
        tot += val
    return 2.0 * eps * tot


def weighted_ks(x1, w1, x2, w2):
    """Two-sample Kolmogorov-Smirnov statistic for weighted samples and its p-value
    with effective sample sizes n_eff = (sum w)^2 / sum w^2."""
    x1, w1, x2, w2 = map(np.asarray, (x1, w1, x2, w2))
    o1, o2 = np.argsort(x1), np.argsort(x2)
    x1, w1, x2, w2 = x1[o1], w1[o1], x2[o2], w2[o2]
    allx = np.concatenate([x1, x2])
    c1 = np.concatenate([[0.0], np.cumsum(w1)]) / w1.sum()
    c2 = np.concatenate([[0.0], np.cumsum(w2)]) / w2.sum()
    F1 = c1[np.searchsorted(x1, allx, side="right")]
    F2 = c2[np.searchsorted(x2, allx, side="right")]
    D = float(np.max(np.abs(F1 - F2)))
    n1 = w1.sum() ** 2 / (w1 ** 2).sum()
    n2 = w2.sum() ** 2 / (w2 ** 2).sum()
    ne = n1 * n2 / (n1 + n2)
    from scipy.stats import kstwobign
    p = float(kstwobign.sf(D * math.sqrt(ne)))
    return D, p


def family_moments(z, w, family):
    """Weighted mean and standard deviation of z, with standard errors that treat primary
    families (a primary and all of its clones, which share their early path) as the
    independent units: per family W_f = sum w, S_f = sum w z, Q_f = sum w z^2; the mean
    m = sum S / sum W and std = sqrt(sum Q / sum W - m^2) are ratio estimators, and their
    standard errors come from the first-order (delta-method) expansion over families,
    SE(m)^2 = sum_f (S_f - m W_f)^2 / (sum W)^2 and
    SE(std)^2 = sum_f ((Q_f - E2 W_f) - 2 m (S_f - m W_f))^2 / (2 std sum W)^2."""
    z, w = np.asarray(z, float), np.asarray(w, float)
    fam = np.unique(np.asarray(family), return_inverse=True)[1]
    nf = fam.max() + 1
    Wf = np.bincount(fam, weights=w, minlength=nf)
    Sf = np.bincount(fam, weights=w * z, minlength=nf)
    Qf = np.bincount(fam, weights=w * z * z, minlength=nf)
    W = Wf.sum()
    m = Sf.sum() / W
    E2 = Qf.sum() / W
    sd = math.sqrt(max(E2 - m * m, 0.0))
    se_m = math.sqrt(((Sf - m * Wf) ** 2).sum()) / W
    r = (Qf - E2 * Wf) - 2.0 * m * (Sf - m * Wf)
    se_sd = math.sqrt((r ** 2).sum()) / (2.0 * sd * W) if sd > 0 else float("nan")
    return m, sd, se_m, se_sd

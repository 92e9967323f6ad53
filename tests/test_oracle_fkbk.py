"""Pins of the oracle's Firsov + Brandt-Kitagawa stopping (CPU only).

The model (paper Sec. 2, "Third": a local inelastic loss after Firsov and Kishinevskii plus a
Brandt-Kitagawa loss in the interstitial electron density; the paper prints no parameters):
friction gamma = k (gamma_F(x) + (zeta Z1)^2 gamma_p), with gamma_F a sum over the domain atoms
of the kernel C 3 b^3 / (pi (1 + b r)^5), C = S_F / v from Firsov's stopping cross-section.

Pinned here against things other than the oracle's own code: Firsov's per-collision loss and
its impact-parameter integral (scipy quadrature of the published formula), the kernel's volume
integral, molecular-dynamics flybys past one atom against the line integral of the published
kernel (closed form head-on, quadrature off axis) and their independence of the speed, the
impact-parameter integral of those line integrals against the stopping cross-section, the
Brandt-Kitagawa limits (bare ion: zeta = 1 and the loss scales as Z1^2; slow ion: constant
zeta, friction independent of the speed), the atomic velocity unit from the electron mass, a
free ion's exponential slowing-down under the Brandt-Kitagawa friction alone, and k = 0
against the stopping switched off.  The absolute stopping (and so the range profile) is
parity unpinned against the paper."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

B, P, AS = 0, 1, 2
SPECIES3 = ("B", "P", "As")
ZS = {"B": 5, "P": 15, "As": 33}
N_E_SI = 32.0 / 5.431 ** 3      # four valence electrons per silicon atom


def cfg(**kw):
    kw.setdefault("species", SPECIES3)
    kw.setdefault("stop_mode", oracle.STOP_FKBK)
    return oracle.Config(**kw)


def _firsov_kernel(zsum, r):
    """The published Firsov constants: b = 0.31 (Z1+Z2)^(1/3) per A, S_F / v =
    0.3254 (Z1+Z2) / sqrt(2) with v in sqrt(eV/amu); unit-volume kernel 3 b^3 / (pi (1+br)^5)."""
    b = 0.31 * zsum ** (1.0 / 3.0)
    C = 0.3254 * zsum / math.sqrt(2.0)
    return C * 3.0 * b ** 3 / (math.pi * (1.0 + b * r) ** 5)


@pytest.mark.parametrize("name", ["B", "P", "As"])
def test_firsov_cross_section_is_the_impact_parameter_integral_of_the_collision_loss(name):
    """Firsov's loss per collision, 0.05973 (Z1+Z2)^(5/3) sqrt(E/M1) / (1 + 0.31 (Z1+Z2)^(1/3) p)^5
    eV, integrated over 2 pi p dp, is the cross-section 0.3254 (Z1+Z2) sqrt(E/M1) eV A^2 the
    kernel is normalised to (0.3254 is the rounded closed form)."""
    zs = ZS[name] + 14
    b = 0.31 * zs ** (1.0 / 3.0)
    val, _ = integrate.quad(lambda p: 2 * math.pi * p * 0.05973 * zs ** (5.0 / 3.0) / (1 + b * p) ** 5, 0, np.inf,
                            epsabs=0, epsrel=1e-12)
    assert abs(val / (0.3254 * zs) - 1.0) < 2e-4


@pytest.mark.parametrize("sp", [B, P, AS])
def test_firsov_kernel_matches_published_constants_and_has_unit_volume_integral(sp):
    c = cfg()
    zs = ZS[SPECIES3[sp]] + 14
    for r in (0.0, 0.3, 1.0, 2.35, 5.0, 12.0):
        assert abs(oracle.firsov_weight(c, sp, r) / _firsov_kernel(zs, r) - 1.0) < 1e-13
    vol, _ = integrate.quad(lambda r: 4 * math.pi * r * r * oracle.firsov_weight(c, sp, r), 0, np.inf,
                            epsabs=0, epsrel=1e-12)
    assert abs(vol / (0.3254 * zs / math.sqrt(2.0)) - 1.0) < 1e-10


def _flyby(c, sp, E, p, r0=60.0):
    """An ion passing one atom (no nuclear force, so the path is straight) at impact
    parameter p from z = -r0: returns Gamma = M1 (v_in - v_out), the line integral of the
    friction, and the end point z1."""
    t = oracle.Track.start(c, sp, E, [p, 0.0, -r0], [0.0, 0.0, 1.0], 1)
    v_in = np.linalg.norm(t.state()["v"])
    m1 = 2.0 * E / v_in ** 2
    n = int(math.ceil(2.0 * r0 / c.dx_max)) + 10
    t.advance(n, events=False)
    st = t.state()
    assert st["x"][2] > r0 and abs(st["x"][0] - p) < 1e-12
    return m1 * (v_in - np.linalg.norm(st["v"])), st["x"][2]


def _line_integral(zs, p, s0=-np.inf, s1=np.inf):
    f = lambda s: _firsov_kernel(zs, math.hypot(p, s))
    if s0 == -np.inf and s1 == np.inf:
        return 2.0 * integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-12)[0]
    return integrate.quad(f, s0, 0, epsabs=0, epsrel=1e-12)[0] + integrate.quad(f, 0, s1, epsabs=0, epsrel=1e-12)[0]


@pytest.mark.parametrize("sp", [B, AS])
def test_flyby_loss_is_the_line_integral_of_the_firsov_kernel(sp):
    """Force -gamma v along a straight path gives dv/ds = -gamma / M1, so the speed drops by
    exactly the line integral of gamma over M1 along the path travelled (z from -r0 to z1).
    Head on the integral has the closed form C 3 b^2 / (4 pi) (2 - (1 + b r0)^-4 -
    (1 + b z1)^-4); off axis it is compared with quadrature of the published kernel.  The
    step-size error falls as dx_max^2: at 0.002 A it is below 1e-5 head on (the kernel's cusp at
    the atom) and below 1e-6 off axis."""
    c = cfg(structure=oracle.ISOLATED, pot_mode=oracle.POT_NONE, n_e=0.0, dx_max=0.002, E_stop=1e-6)
    zs = ZS[SPECIES3[sp]] + 14
    b = 0.31 * zs ** (1.0 / 3.0)
    C = 0.3254 * zs / math.sqrt(2.0)
    g0, z1 = _flyby(c, sp, 2000.0, 0.0)
    head_on = 3.0 * C * b * b / (4.0 * math.pi) * (2.0 - (1.0 + b * 60.0) ** -4 - (1.0 + b * z1) ** -4)
    assert abs(g0 / head_on - 1.0) < 1e-5, (g0, head_on)
    for p in (0.5, 1.5, 3.0):
        g, z1 = _flyby(c, sp, 2000.0, p)
        assert abs(g / _line_integral(zs, p, -60.0, z1) - 1.0) < 1e-6


def test_flyby_loss_is_proportional_to_the_speed():
    """The Firsov friction does not depend on the speed, so the momentum it takes in one
    flyby is the same at 500 eV and at 50 keV (the energy lost is proportional to v)."""
    c = cfg(structure=oracle.ISOLATED, pot_mode=oracle.POT_NONE, n_e=0.0, dx_max=0.004, E_stop=1e-6)
    g_lo = _flyby(c, P, 500.0, 0.8)[0]
    g_hi = _flyby(c, P, 50000.0, 0.8)[0]
    assert abs(g_hi / g_lo - 1.0) < 1e-6


def test_impact_parameter_integral_of_the_local_loss_is_the_stopping_cross_section():
    """Integrating the flyby loss over 2 pi p dp gives back the volume integral of the kernel:
    the local loss reproduces Firsov's stopping cross-section S_F = C v."""
    zs = 5 + 14
    b = 0.31 * zs ** (1.0 / 3.0)
    # p = t / (b (1 - t)) maps [0, 1) onto [0, inf)
    f = lambda t: 2 * math.pi * (t / (b * (1 - t))) * _line_integral(zs, t / (b * (1 - t))) / (b * (1 - t) ** 2)
    val, _ = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-9, limit=200)
    assert abs(val / (0.3254 * zs / math.sqrt(2.0)) - 1.0) < 1e-7


def test_atomic_velocity_unit():
    """The velocity unit of the Brandt-Kitagawa formulas: one atomic unit is the speed of an
    electron with kinetic energy of half a Hartree, sqrt(E_h / m_e) = 222.72 sqrt(eV/amu)
    (m_e = 5.48579909065e-4 amu).  A bare ion (zeta = 1) at speed v_au atomic units has the
    same Brandt-Kitagawa friction whichever route converts the unit."""
    v_au = math.sqrt(27.211386245988 / 5.48579909065e-4)
    c = cfg(n_e=N_E_SI)
    # well above the Fermi speed (relative speed ~ v) and fully stripped (zeta = 1 to 1e-12)
    v = 60.0 * v_au * 33 ** (2.0 / 3.0)
    assert abs(oracle.bk_zeta(c, AS, v) - 1.0) < 1e-12
    assert abs(oracle.bk_gamma(c, AS, v) / (33 ** 2 * oracle.bk_proton_friction(c)) - 1.0) < 1e-12
    # the Fermi speed of silicon's valence gas, vF = (3 pi^2 n)^(1/3) a0 in atomic units, separates
    # the two relative-speed branches: zeta is continuous there
    n_au = N_E_SI * 0.529177210903 ** 3
    vF = (3 * math.pi ** 2 * n_au) ** (1.0 / 3.0) * v_au
    z_lo, z_hi = oracle.bk_zeta(c, B, vF * (1 - 1e-9)), oracle.bk_zeta(c, B, vF * (1 + 1e-9))
    assert abs(z_hi - z_lo) < 1e-7


@pytest.mark.parametrize("sp", [B, P, AS])
def test_brandt_kitagawa_effective_charge_limits(sp):
    """zeta lies in [0, 1], grows with the speed, tends to 1 for a bare ion and to a
    constant for a slow one (so the loss of a slow ion is proportional to its speed)."""
    c = cfg(n_e=N_E_SI)
    vs = np.geomspace(1e-3, 1e5, 200)
    z = np.array([oracle.bk_zeta(c, sp, v) for v in vs])
    assert (z > 0).all() and (z <= 1.0 + 1e-15).all()
    assert (np.diff(z) >= -1e-15).all()
    assert z[-1] > 1 - 1e-9
    g = [oracle.bk_gamma(c, sp, v) for v in (1e-6, 1e-4, 1e-2)]
    assert abs(g[2] / g[0] - 1.0) < 1e-8 and abs(g[1] / g[0] - 1.0) < 1e-12
    # no electrons: no Brandt-Kitagawa loss
    assert oracle.bk_gamma(cfg(n_e=0.0), sp, 10.0) == 0.0


def test_free_ion_slows_exponentially_under_brandt_kitagawa_friction():
    """Far from any atom the Firsov sum is below 1e-15 of its contact value and the
    Brandt-Kitagawa friction of a slow ion is constant to 1e-10: the speed decays as
    exp(-k gamma t / M1), which the split friction reproduces step by step."""
    k = 0.7
    c = cfg(structure=oracle.ISOLATED, pot_mode=oracle.POT_NONE, n_e=N_E_SI, k=k, dx_max=0.05, dt_max=0.5,
            E_stop=1e-9)
    E = 1e-4
    t = oracle.Track.start(c, B, E, [0.0, 1000.0, 0.0], [1.0, 0.0, 0.0], 1)
    v0 = np.linalg.norm(t.state()["v"])
    T = 0.0
    for _ in range(400):
        T += t.step()
    v = np.linalg.norm(t.state()["v"])
    g = oracle.bk_gamma(c, B, v0)
    m1 = 2.0 * E / v0 ** 2
    assert abs(math.log(v / v0) / (-k * g * T / m1) - 1.0) < 1e-9


def test_zero_scale_equals_stopping_off():
    """k = 0 removes the whole stopping force: 300 steps of a 5 keV As track in the crystal are
    bitwise those with the stopping switched off."""
    pr = oracle.sample_primaries(oracle.SamplerCfg(choice=(2,), E_min=5000.0, E_max=5000.0), 3, 1)
    a = oracle.Track.start(cfg(k=0.0, n_e=N_E_SI), 2, float(pr["E0"][0]), pr["pos"][:, 0], pr["dir"][:, 0],
                           int(pr["key"][0]))
    b = oracle.Track.start(cfg(stop_mode=oracle.STOP_OFF), 2, float(pr["E0"][0]), pr["pos"][:, 0],
                           pr["dir"][:, 0], int(pr["key"][0]))
    a.advance(300, events=False)
    b.advance(300, events=False)
    ra, rb = a.record(), b.record()
    ra[9] = rb[9] = 0.0          # the Firsov sum vs the LS density: different weights, unused at k = 0
    assert np.array_equal(ra.view(np.int64), rb.view(np.int64))


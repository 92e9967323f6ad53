"""Pins of the oracle's fluorite (UO2) target, two-species stopping, recoil start and radial
range (CPU only), each against something other than the oracle's own formulas: textbook
fluorite geometry, the Coulomb limit and the printed ZBL reduced energy for the anion
constants, Lindhard's reduced form for both stopping constants, closed-form friction paths,
the atomic densities of the structure, energy and momentum ledgers, and exact record
round trips.
"""
import math

import numpy as np
import pytest
from scipy import stats as sps

import oracle
from tests import physref

U, B = 0, 1


def ucfg(**kw):
    d = dict(oracle.UO2)
    d.update(species=("U", "B"))
    d.update(kw)
    return oracle.Config(**d)


def _domain(t, c):
    st = t.state()
    ex = oracle.slot_exists(st["center"], c.structure, st["vac_cell"], st["vac_basis"])
    return st, ex


# --------------------------------------------------------------------------- geometry
def test_fluorite_geometry_and_domain_size():
    """27 cells x (4 cations + 8 anions) = 324 atoms; nearest cation-anion distance a sqrt(3)/4,
    anion-anion a/2, cation-cation a/sqrt(2); every anion has 4 cation neighbours
    (tetrahedron) and every cation 8 anion neighbours (cube) at a sqrt(3)/4."""
    c = ucfg(sigma=0.0, sigma_b=0.0)
    t = oracle.Track.start(c, U, 1000.0, [10.2 * c.a, 10.6 * c.a, 10.3 * c.a], [0, 0, 1], 3)
    st, ex = _domain(t, c)
    assert ex.sum() == 324
    assert ex[:108].all() and not ex[108:128].any() and ex[128:].all()
    X = st["ax"].T
    cat, an = X[:108], X[128:]
    def dists(A, Bm):
        d = np.sqrt(((A[:, None, :] - Bm[None, :, :]) ** 2).sum(-1))
        d[d < 1e-9] = np.inf
        return d
    a = c.a
    assert abs(dists(cat, an).min() - a * math.sqrt(3) / 4) < 1e-12
    assert abs(dists(an, an).min() - a / 2) < 1e-12
    assert abs(dists(cat, cat).min() - a / math.sqrt(2)) < 1e-12
    nn = a * math.sqrt(3) / 4 + 1e-9
    d_ac = dists(an, cat)
    centre = np.array(st["center"]) * a
    inner_an = np.all((an > centre + 0.1) & (an < centre + a - 0.1), axis=1)
    assert inner_an.sum() == 8
    assert np.all((d_ac[inner_an] <= nn).sum(1) == 4)
    d_ca = dists(cat, an)
    inner_cat = np.all((cat > centre - 0.1) & (cat < centre + a + 0.1), axis=1)
    assert np.all((d_ca[inner_cat] <= nn).sum(1) == 8)
    # stoichiometry of the target species at the sites
    types = [oracle.site(c, b)[1] for b in range(12)]
    assert types == [0] * 4 + [1] * 8


def test_fluorite_record_round_trip_is_exact():
    c = ucfg(vacancy=1)
    t = oracle.Track.start(c, U, 85000.0, [0.0, 0.0, 40 * c.a], [0.3, 0.5, 0.8], 77)
    t.advance(300, events=False)
    r1 = t.record()
    r2 = oracle.Track.from_record(c, r1).record()
    assert r1.shape[0] == oracle.RECORD_WORDS_FLUORITE
    assert np.array_equal(r1.view(np.int64), r2.view(np.int64))


# --------------------------------------------------------------------------- anion constants
def test_anion_pair_constants():
    """Target species 1 uses Z2b: r V(r) -> Z1 Z2b e^2 as r -> 0, its screening length gives
    the printed ZBL reduced energy, and its stopping constant Lindhard's reduced form."""
    c = ucfg()
    for sp, (Z1, M1) in ((U, (92, 238.03)), (B, (5, 10.81))):
        for ty, (Z2, M2) in ((0, (92, 238.03)), (1, (8, 15.999))):
            V, _ = oracle.zbl(c, sp, 1e-10, type=ty)
            assert abs(V * 1e-10 / (Z1 * Z2 * physref.COULOMB) - 1.0) < 1e-8
            aU = oracle.screening_length(c, sp, type=ty)
            E = 85_000.0
            eps = aU * E * M2 / (M2 + M1) / (Z1 * Z2 * physref.COULOMB)
            assert abs(eps / physref.zbl_reduced_energy(Z1, Z2, M1, M2, E) - 1.0) < 5e-4
            assert abs(oracle.lss_kL(c, sp, type=ty) / physref.lindhard_kL(Z1, Z2, M1, M2) - 1.0) < 2e-3


# --------------------------------------------------------------------------- stopping
def _free(c, sp, E0, pos, d):
    return oracle.Track.start(c, sp, E0, pos, d, 1)


def test_compound_uniform_stopping_path_closed_form():
    """ZBL off, uniform stopping in UO2 (Bragg additivity): the path to E_stop is
    2 (sqrt(E0) - sqrt(E_stop)) / (k (N_U kL_U + N_O kL_O)) with N_U = 4/a^3, N_O = 8/a^3."""
    for sp, name, E0, k in ((U, "U", 85000.0, 1.0), (B, "B", 3000.0, 0.6)):
        c = ucfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM, k=k, dx_max=0.05)
        t = _free(c, sp, E0, [0.0, 0.0, -3.0], [0.0, 0.0, 1.0])
        t.advance(10**8, events=True)
        st = t.state()
        assert st["status"] == oracle.STOPPED
        S = 4 / c.a**3 * oracle.lss_kL(c, sp, 0) + 8 / c.a**3 * oracle.lss_kL(c, sp, 1)
        L = 2 * (math.sqrt(E0) - math.sqrt(c.E_stop)) / (k * S)
        assert abs((st["z_stop"] + 3.0) / L - 1.0) < 1e-7
        # local stopping gives the same coefficient on average (next test), and gamma(rho)
        # is linear with gamma(uniform density) equal to the uniform one
        cl = ucfg(stop_mode=oracle.STOP_LOCAL, k=k)
        M1 = oracle.SPECIES[name][1]
        kL0 = oracle.lss_kL(c, sp, 0)
        rho_u = S / kL0
        assert abs(oracle.gamma(cl, sp, rho_u) / (k * S * math.sqrt(M1 / 2)) - 1.0) < 1e-14


def test_compound_local_density_averages_to_weighted_atomic_density():
    """rho = sum_t (kL_t / kL_0) sum_{j in t} w_t(r_j) with unit-integral kernels: its mean over
    ion positions in a cell is N_U + N_O kL_O / kL_U (midpoint grid, B ions)."""
    c = ucfg(sigma=0.0, sigma_b=0.0)
    ref = 4 / c.a**3 + 8 / c.a**3 * oracle.lss_kL(c, B, 1) / oracle.lss_kL(c, B, 0)
    n = 32
    g = (np.arange(n) + 0.5) / n
    vals = []
    for i in g:
        for j in g:
            for k in g:
                x = (np.array([10.0, 10.0, 10.0]) + np.array([i, j, k])) * c.a
                vals.append(oracle.Track.start(c, B, 1000.0, x, [0, 0, 1], 1).state()["rho"])
    assert abs(np.mean(vals) / ref - 1.0) < 5e-4


# --------------------------------------------------------------------------- recoil start
def test_vacancy_at_the_start_site_stays_empty():
    """A recoil starts on the basis-0 site of its cell and that site stays empty, also when
    the cell is created again after leaving the domain."""
    c = ucfg(vacancy=1, pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_OFF, sigma=0.0, sigma_b=0.0)
    z0 = 40 * c.a
    t = oracle.Track.start(c, U, 2000.0, [0.0, 0.0, z0], [1.0, 0.0, 0.0], 5)
    st, ex = _domain(t, c)
    assert ex.sum() == 323
    assert list(st["vac_cell"]) == [0, 0, 40] and st["vac_basis"] == 0
    X = st["ax"][:, ex].T
    assert np.sqrt(((X - np.array([0.0, 0.0, z0])) ** 2).sum(1)).min() > 2.3   # nearest: anion at a sqrt(3)/4
    # fly two cells away, then put the ion back next to the start site
    while t.state()["center"][0] < 2:
        t.advance(50, events=False)
    rec = t.record()
    rec[0] = 0.3
    t2 = oracle.Track.from_record(c, rec)
    t2.step()
    st2, ex2 = _domain(t2, c)
    assert list(st2["center"]) == [0, 0, 40]
    assert ex2.sum() == 323
    X = st2["ax"][:, ex2].T
    assert np.sqrt(((X - np.array([0.0, 0.0, z0])) ** 2).sum(1)).min() > 2.3


def test_recoil_sampler_is_on_site_and_isotropic():
    sc = oracle.SamplerCfg(choice=(0,), E_min=85000.0, E_max=85000.0, dir_mode=oracle.DIR_ISOTROPIC,
                           start_mode=oracle.START_SITE, a=oracle.UO2["a"], z_start=40 * oracle.UO2["a"])
    n = 20000
    pr = oracle.sample_primaries(sc, 11, n)
    assert np.all(pr["pos"][0] == 0.0) and np.all(pr["pos"][1] == 0.0)
    assert np.all(pr["pos"][2] == 40 * oracle.UO2["a"])
    d = pr["dir"]
    assert np.allclose((d * d).sum(0), 1.0, atol=1e-14)
    assert np.abs(d.mean(1)).max() < 5 / math.sqrt(3 * n)
    for ax in range(3):   # every Cartesian component of a uniform unit vector is uniform on [-1, 1]
        assert sps.kstest(d[ax], "uniform", args=(-1, 2)).pvalue > 1e-3


def test_radial_range_of_a_free_ion_is_its_path_length():
    """ZBL off, uniform stopping, isotropic recoils: with the radial range the stopping
    coordinate is the closed-form path length in every direction; with the depth range it
    is z0 + L cos(theta)."""
    sc = oracle.SamplerCfg(choice=(0,), E_min=20000.0, E_max=20000.0, dir_mode=oracle.DIR_ISOTROPIC,
                           start_mode=oracle.START_SITE, a=oracle.UO2["a"], z_start=400 * oracle.UO2["a"])
    pr = oracle.sample_primaries(sc, 2, 6)
    base = dict(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM, vacancy=1, z_start=0.0)
    cr = ucfg(range_mode=oracle.RANGE_RADIAL, **base)
    cd = ucfg(range_mode=oracle.RANGE_DEPTH, **base)
    S = 4 / cr.a**3 * oracle.lss_kL(cr, U, 0) + 8 / cr.a**3 * oracle.lss_kL(cr, U, 1)
    L = 2 * (math.sqrt(20000.0) - math.sqrt(cr.E_stop)) / S
    for i in range(6):
        p0, d = pr["pos"][:, i], pr["dir"][:, i]
        tr = oracle.Track.start(cr, U, 20000.0, p0, d, 1)
        tr.advance(10**8, events=True)
        td = oracle.Track.start(cd, U, 20000.0, p0, d, 1)
        td.advance(10**8, events=True)
        assert tr.state()["status"] == oracle.STOPPED and td.state()["status"] == oracle.STOPPED
        assert abs(tr.state()["z_stop"] / L - 1.0) < 1e-7
        assert abs(td.state()["z_stop"] - (p0[2] + L * d[2])) < 1e-7 * L
        assert np.array_equal(tr.state()["x0"], p0)


# --------------------------------------------------------------------------- invariants
def test_fluorite_energy_and_momentum_conservation_without_stopping():
    """Stopping off, thermal UO2 domain with the recoil vacancy, two atom masses: the energy
    ledger is constant to 1e-8 relative and the momentum ledger to round-off over several
    domain shifts."""
    c = ucfg(stop_mode=oracle.STOP_OFF, dx_max=4e-4, vacancy=1)
    z0 = 40 * c.a
    t = oracle.Track.start(c, U, 2000.0, [0.0, 0.0, z0], [0.55, 0.35, 0.76], 4242)
    E0, p0 = t.ledger()
    shifts = 0
    center = t.state()["center"].copy()
    worst = 0.0
    while np.linalg.norm(t.state()["x"] - np.array([0.0, 0.0, z0])) < 20.0:
        t.advance(4000, events=False)
        st = t.state()
        if (st["center"] != center).any():
            shifts += 1
            center = st["center"].copy()
        E, pm = t.ledger()
        worst = max(worst, abs(E - E0) / E0)
        assert np.abs(pm - p0).max() < 1e-12 * np.linalg.norm(p0) * 100
        if t.state()["steps"] > 400000:
            break
    assert shifts >= 3
    assert worst < 1e-8

"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what it pins and the reference it is checked against: a
library routine (numpy's Philox, scipy quadrature / root finding), a closed
form (Rutherford, Coulomb turning point, pure-friction decay), a published
independent form (Lindhard's reduced stopping, the ZBL universal nuclear
stopping fit and reduced energy), an invariant (energy, momentum, weight), or
brute force (splitting vs no splitting).
"""
import math

import numpy as np
import pytest

import oracle
from tests import physref

B, P, AS = 0, 1, 2
SPECIES3 = ("B", "P", "As")


def cfg(**kw):
    kw.setdefault("species", SPECIES3)
    return oracle.Config(**kw)


# --------------------------------------------------------------------------- RNG
def test_philox_matches_numpy():
    """Philox4x64-10 (Salmon et al. 2011) vs numpy's independent implementation."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64) * 2 + rng.integers(0, 2, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        # numpy increments its counter before each block: start one below
        c = ctr[:]
        i = 0
        while True:
            c[i] = (c[i] - 1) % 2**64
            if c[i] != 2**64 - 1:
                break
            i += 1
            if i == 4:
                break
        bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
        assert [int(x) for x in bg.random_raw(4)] == oracle.philox4x64(ctr, key)


def test_uniform_open_interval_exact():
    L = oracle.lib()
    assert L.or_u01(0) == 2.0**-53
    assert L.or_u01(2**64 - 1) == 1.0 - 2.0**-53
    assert 0.0 < L.or_u01(2**63) < 1.0


def test_thermal_displacements_are_gaussian():
    """Created atoms sit at ideal diamond sites plus N(0, sigma^2) per axis."""
    c = cfg(sigma=0.076)
    c0 = cfg(sigma=0.0)
    dev = []
    for key in range(300):
        pos = [10.3 * c.a, 7.6 * c.a, 12.2 * c.a]
        t = oracle.Track.start(c, 0, 1000.0, pos, [0, 0, 1], key + 1)
        t0 = oracle.Track.start(c0, 0, 1000.0, pos, [0, 0, 1], key + 1)
        dev.append((t.state()["ax"] - t0.state()["ax"]).ravel())
    d = np.concatenate(dev) / 0.076
    n = d.size
    assert abs(d.mean()) < 5 / math.sqrt(n)
    assert abs(d.std() - 1.0) < 5 / math.sqrt(2 * n)
    kurt = np.mean(d**4) / np.mean(d**2) ** 2
    assert abs(kurt - 3.0) < 5 * math.sqrt(24.0 / n)


# --------------------------------------------------------------------------- ZBL
def test_zbl_coulomb_limit():
    """phi(0) = 1: r V(r) -> Z1 Z2 e^2 as r -> 0."""
    c = cfg()
    for sp, Z in ((B, 5), (P, 15), (AS, 33)):
        V, _ = oracle.zbl(c, sp, 1e-10)
        assert abs(V * 1e-10 / (Z * 14 * physref.COULOMB) - 1.0) < 1e-8


def test_zbl_force_is_derivative_of_potential():
    c = cfg()
    for sp in (B, P, AS):
        for r in (0.05, 0.2, 0.7, 1.5, 3.0, 6.0):
            h = 1e-4 * r
            Vf = lambda x: oracle.zbl(c, sp, x)[0]
            d1 = (Vf(r + h) - Vf(r - h)) / (2 * h)
            d2 = (Vf(r + h / 2) - Vf(r - h / 2)) / h
            rich = (4 * d2 - d1) / 3
            assert abs(oracle.zbl(c, sp, r)[1] - rich) <= 1e-9 * abs(rich)


def test_zbl_screening_length_matches_published_reduced_energy():
    """eps = a_U E_cm / (Z1 Z2 e^2) must equal the printed ZBL reduced energy
    32.53 M2 E[keV] / (Z1 Z2 (M1+M2)(Z1^0.23+Z2^0.23)) (pins 0.8854 a0 and the 0.23 exponent)."""
    c = cfg()
    for sp, (Z1, M1) in enumerate([(5, 10.81), (15, 30.97), (33, 74.92)]):
        aU = oracle.screening_length(c, sp)
        E = 10_000.0
        eps = aU * E * c.M2 / (c.M2 + M1) / (Z1 * c.Z2 * physref.COULOMB)
        ref = physref.zbl_reduced_energy(Z1, c.Z2, M1, c.M2, E)
        assert abs(eps / ref - 1.0) < 5e-4   # the printed 32.53 carries 4 digits
    c2 = cfg(s=1.7)
    assert abs(oracle.screening_length(c2, 0) / oracle.screening_length(c, 0) - 1.7) < 1e-15


@pytest.mark.parametrize("eps", [0.01, 0.1, 1.0])
def test_zbl_nuclear_stopping_matches_universal_fit(eps):
    """Reduced nuclear stopping computed by quadrature over the oracle's screening
    function agrees with the ZBL universal fit (pins the c_i, d_i pairs)."""
    c = cfg()
    sp, Z1 = B, 5
    aU = oracle.screening_length(c, sp)
    zz = Z1 * c.Z2 * physref.COULOMB
    phi = lambda x: oracle.zbl(c, sp, x * aU)[0] * (x * aU) / zz
    sn = physref.reduced_nuclear_stopping(phi, eps)
    assert abs(sn / physref.zbl_universal_sn(eps) - 1.0) < 0.02


# --------------------------------------------------------------------------- stopping
def test_lss_constant_matches_lindhard_reduced_form():
    c = cfg()
    for sp, (Z1, M1) in enumerate([(5, 10.81), (15, 30.97), (33, 74.92)]):
        ref = physref.lindhard_kL(Z1, c.Z2, M1, c.M2)
        assert abs(oracle.lss_kL(c, sp) / ref - 1.0) < 2e-3


def _free_ion_track(c, sp, E0):
    return oracle.Track.start(c, sp, E0, [0.0, 0.0, -3.0], [0.0, 0.0, 1.0], 1)


def test_uniform_stopping_closed_form():
    """ZBL off, uniform stopping: |v(t)| = v0 exp(-gamma t / M1) exactly, and the path to
    E_stop is L = 2 (sqrt(E0) - sqrt(E_stop)) / (k N kL)."""
    for sp, name, E0, k in ((B, "B", 1000.0, 1.0), (P, "P", 5000.0, 1.0), (AS, "As", 10000.0, 0.7)):
        c = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM, k=k, dx_max=0.05)
        t = _free_ion_track(c, sp, E0)
        M1 = oracle.SPECIES[name][1]
        N = 8 / c.a**3
        kL = oracle.lss_kL(c, sp)
        gamma = k * N * kL * math.sqrt(M1 / 2)
        v0 = math.sqrt(2 * E0 / M1)
        tt = 0.0
        for _ in range(500):
            tt += t.step()
        v = np.linalg.norm(t.state()["v"])
        assert abs(v / (v0 * math.exp(-gamma * tt / M1)) - 1.0) < 1e-12
        # path length to the stop
        t = _free_ion_track(c, sp, E0)
        t.advance(10**8, events=True)
        st = t.state()
        assert st["status"] == oracle.STOPPED
        L = 2 * (math.sqrt(E0) - math.sqrt(c.E_stop)) / (k * N * kL)
        assert abs((st["z_stop"] - (-3.0)) / L - 1.0) < 1e-7


def test_time_step_follows_kinetic_scale():
    """Fig. 2: the step grows as the ion slows; for a free ion dt = dx_max / |v|."""
    c = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM)
    for E in (100.0, 1000.0, 10000.0):
        t = _free_ion_track(c, B, E)
        dt = t.step()
        v0 = math.sqrt(2 * E / 10.81)
        assert abs(dt * v0 / c.dx_max - 1.0) < 1e-12


@pytest.mark.parametrize("r", [0.4, 1.0, 2.0])
@pytest.mark.parametrize("dx_max", [0.05, 0.01])
def test_time_step_acceleration_branch(r, dx_max):
    """Fig. 2 / collisional scale: an ion at rest at distance r from one free atom moves by
    a t^2 / 2 in a step, so the step that keeps that below dx_max is
    dt = sqrt(2 dx_max / a) with a = |V'(r)| / M of the particle that accelerates most.
    B (10.81 u) on Si (28.0855 u): the ion, a = |V'| / M1.  B on a light target (4 u): the
    atom, a = |V'| / M2.  |V'(r)| is the ZBL derivative, itself pinned against Richardson
    differences of V(r) (test_zbl_force_is_derivative_of_potential)."""
    for M2 in (28.0855, 4.0):
        c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF, dx_max=dx_max, M2=M2)
        t = oracle.Track.start(c, B, 0.0, [0.0, 0.0, -r], [0.0, 0.0, 1.0], 1)
        F = abs(oracle.zbl(c, B, r)[1])
        M = min(10.81, M2)                     # the lighter particle accelerates most
        ref = math.sqrt(2.0 * dx_max * M / F)
        assert ref < c.dt_max
        dt = t.step()
        assert abs(dt / ref - 1.0) < 1e-13, (M2, dt, ref)
    # far from the atom and at rest nothing limits the step but dt_max
    c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF, dx_max=dx_max)
    t = oracle.Track.start(c, B, 0.0, [0.0, 0.0, -200.0], [0.0, 0.0, 1.0], 1)
    assert t.step() == c.dt_max


def test_time_step_takes_the_smaller_branch():
    """A slow ion near an atom: the acceleration branch is below the speed branch and wins;
    a fast one far away: dx_max / |v|."""
    c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF)
    r, E = 0.6, 0.5
    t = oracle.Track.start(c, B, E, [0.0, 0.0, -r], [1.0, 0.0, 0.0], 1)
    F = abs(oracle.zbl(c, B, r)[1])
    da = math.sqrt(2.0 * c.dx_max * 10.81 / F)
    dv = c.dx_max / math.sqrt(2.0 * E / 10.81)
    assert da < dv
    assert abs(t.step() / da - 1.0) < 1e-13
    t = oracle.Track.start(c, B, 5000.0, [0.0, 0.0, -40.0], [1.0, 0.0, 0.0], 1)
    assert abs(t.step() * math.sqrt(2.0 * 5000.0 / 10.81) / c.dx_max - 1.0) < 1e-12


def _free_track_status(c, z0, dz, nsteps):
    t = oracle.Track.start(c, B, 1000.0, [1.7, 2.3, z0], [0.0, 0.0, dz], 5)
    t.advance(nsteps, events=True)
    st = t.state()
    return st["status"], st["steps"], st["x"][2]


def test_backscatter_rule():
    """Termination on backscatter (z < z_start while moving outward, v_z < 0), decided after
    each step.  A free ion (no forces, no stopping) moves exactly dx_max per step:
    - from z = -2.93 A outward it is at -2.98 A after one step (still above z_start = -3 A,
      active) and at -3.03 A after the second, where it ends as backscattered;
    - from z = -5 A (below z_start) moving inward it never backscatters;
    - moving parallel to the surface below z_start (v_z = 0) it never backscatters."""
    c = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_OFF)
    st, n, z = _free_track_status(c, -2.93, -1.0, 50)
    assert st == oracle.BACKSCATTERED and n == 2 and z < c.z_start
    st, n, z = _free_track_status(c, -2.93, -1.0, 1)
    assert st == oracle.ACTIVE and n == 1 and z > c.z_start
    st, n, z = _free_track_status(c, -5.0, 1.0, 30)
    assert st == oracle.ACTIVE and n == 30 and z < c.z_start
    t = oracle.Track.start(c, B, 1000.0, [1.7, 2.3, -3.5], [1.0, 0.0, 0.0], 5)
    t.advance(30, events=True)
    assert t.state()["status"] == oracle.ACTIVE and t.state()["steps"] == 30
    # the rule follows z_start: with z_start = -4 A the outward ion from -3.93 A ends on step 2
    c4 = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_OFF, z_start=-4.0)
    st, n, z = _free_track_status(c4, -3.93, -1.0, 50)
    assert st == oracle.BACKSCATTERED and n == 2


def test_local_density_averages_to_atomic_density():
    """rho(x) = sum_j w(|x - x_j|) with a unit-integral kernel: its mean over ion positions in
    a cell equals the atomic density N up to the kernel mass outside the domain (midpoint grid)."""
    c = cfg(sigma=0.0)
    N = 8 / c.a**3
    n = 24
    g = (np.arange(n) + 0.5) / n
    vals = []
    for i in g:
        for j in g:
            for k in g:
                x = (np.array([10.0, 10.0, 10.0]) + np.array([i, j, k])) * c.a
                vals.append(oracle.Track.start(c, B, 1000.0, x, [0, 0, 1], 1).state()["rho"] / N)
    assert abs(np.mean(vals) - 1.0) < 5e-4


# --------------------------------------------------------------------------- lattice / domain
def test_lattice_geometry_and_domain_size():
    c = cfg(sigma=0.0)
    t = oracle.Track.start(c, B, 1000.0, [10.2 * c.a, 10.6 * c.a, 10.3 * c.a], [0, 0, 1], 3)
    st = t.state()
    ex = oracle.slot_exists(st["center"])
    assert ex.sum() == 216
    X = st["ax"][:, ex].T
    d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    d[np.arange(len(X)), np.arange(len(X))] = np.inf
    assert abs(d.min() - c.a * math.sqrt(3) / 4) < 1e-12
    assert list(st["center"]) == [10, 10, 10]
    # above the surface only the top layer of cells exists
    t = oracle.Track.start(c, B, 1000.0, [1.0, 2.0, -3.0], [0, 0, 1], 3)
    st = t.state()
    assert oracle.slot_exists(st["center"]).sum() == 72
    assert st["center"][2] == -1


def test_force_is_lattice_periodic():
    """sigma = 0: translating the ion by a lattice vector leaves the force unchanged."""
    c = cfg(sigma=0.0)
    x = np.array([10.37, 11.81, 9.55]) * c.a / 1.0
    x = np.array([56.3, 61.2, 53.9])
    F0 = oracle.Track.start(c, AS, 1000.0, x, [0, 0, 1], 9).state()["F"]
    for e in np.eye(3):
        F1 = oracle.Track.start(c, AS, 1000.0, x + c.a * e * 2, [0, 0, 1], 9).state()["F"]
        assert np.allclose(F1, F0, rtol=1e-9, atol=1e-12 * np.abs(F0).max())


# --------------------------------------------------------------------------- two-body
def _two_body(c, sp, E, p, r0=20.0):
    return oracle.Track.start(c, sp, E, [p, 0.0, -r0], [0.0, 0.0, 1.0], 1)


def _separation(st):
    return np.linalg.norm(st["x"] - st["ax"][:, 0])


def _min_separation(t):
    """Steps until the separation grows, then fits a parabola through the 3 samples
    around the smallest one."""
    hist = [_separation(t.state())]
    while True:
        t.step()
        hist.append(_separation(t.state()))
        if len(hist) > 3 and hist[-1] > hist[-2] > hist[-3]:
            break
    i = int(np.argmin(hist))
    y0, y1, y2 = hist[i - 1], hist[i], hist[i + 1]
    # minimum of the parabola through equally spaced? samples are not equally spaced in
    # time, but near the turning point dt is constant to high accuracy
    den = y0 - 2 * y1 + y2
    return y1 - (y0 - y2) ** 2 / (8 * den) if den > 0 else y1


@pytest.mark.parametrize("sp,name,E", [(B, "B", 1000.0), (P, "P", 5000.0), (AS, "As", 10000.0)])
def test_head_on_closest_approach_zbl(sp, name, E):
    """Head-on collision with a free target atom: the MD turning point equals the root of
    V(r) = E_cm + V(r0) (energy conservation in the centre-of-mass frame)."""
    c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF, dx_max=1e-4)
    M1 = oracle.SPECIES[name][1]
    Ec = E * c.M2 / (M1 + c.M2)
    V = lambda r: oracle.zbl(c, sp, r)[0]
    rmin_ref = physref.closest_approach(lambda r: V(r) - V(20.0), Ec)
    rmin = _min_separation(_two_body(c, sp, E, 0.0))
    assert abs(rmin / rmin_ref - 1.0) < 1e-6


def test_head_on_closest_approach_coulomb_closed_form():
    """Screening removed (s -> infinity): r_min = Z1 Z2 e^2 / (E_cm + Z1 Z2 e^2 / r0)."""
    c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF, dx_max=1e-4, s=1e12)
    E, M1, Z1 = 1000.0, 10.81, 5
    zz = Z1 * 14 * physref.COULOMB
    Ec = E * c.M2 / (M1 + c.M2)
    ref = zz / (Ec + zz / 20.0)
    rmin = _min_separation(_two_body(c, B, E, 0.0))
    assert abs(rmin / ref - 1.0) < 1e-6


def test_quadrature_reference_reproduces_rutherford():
    """The deflection-integral helper itself, on a pure Coulomb potential."""
    zz = 5 * 14 * physref.COULOMB
    for p in (0.05, 0.3, 1.0):
        th = physref.cm_deflection(lambda r: zz / r, 700.0, p)
        assert abs(th - physref.rutherford_cm(5, 14, 700.0, p)) < 1e-9


@pytest.mark.parametrize("p", [0.1, 0.3, 0.8])
def test_scattering_angle_matches_quadrature(p):
    """MD two-body deflection vs the classical scattering integral (BCA angle)."""
    c = cfg(structure=oracle.ISOLATED, stop_mode=oracle.STOP_OFF, dx_max=2e-4)
    sp, M1, E = B, 10.81, 1000.0
    Ec = E * c.M2 / (M1 + c.M2)
    th = physref.cm_deflection(lambda r: oracle.zbl(c, sp, r)[0], Ec, p)
    psi_ref = physref.lab_angle(th, M1, c.M2)
    t = _two_body(c, sp, E, p)
    while True:
        t.advance(2000, events=False)
        st = t.state()
        rel = st["x"] - st["ax"][:, 0]
        if _separation(st) > 20.0 and rel @ (st["v"] - st["av"][:, 0]) > 0:
            break
    v = st["v"]
    psi = math.acos(v[2] / np.linalg.norm(v))
    assert abs(psi - psi_ref) < 1e-6


# --------------------------------------------------------------------------- conservation
def test_energy_and_momentum_conservation_without_stopping():
    """Stopping off, full thermal domain, dx_max = 2e-4 A over > 20 A of track: the energy
    ledger (ion + atoms + potential + dropped - created) is constant to 1e-8 relative and
    the momentum ledger to round-off."""
    c = cfg(stop_mode=oracle.STOP_OFF, dx_max=2e-4)
    t = oracle.Track.start(c, B, 1000.0, [1.3, 2.1, -3.0], [math.sin(0.12), 0.0, math.cos(0.12)], 12345)
    E0, p0 = t.ledger()
    shifts = 0
    center = t.state()["center"].copy()
    worst = 0.0
    while t.state()["x"][2] < 20.0:
        t.advance(5000, events=False)
        st = t.state()
        if (st["center"] != center).any():
            shifts += 1
            center = st["center"].copy()
        E, pm = t.ledger()
        worst = max(worst, abs(E - E0) / E0)
        assert np.abs(pm - p0).max() < 1e-12 * np.linalg.norm(p0) * 100
    assert shifts >= 3
    assert worst < 1e-8


# --------------------------------------------------------------------------- splitting
def _run(c, prim, log=True):
    return oracle.run(c, prim, nthreads=8, log=log)


def test_weight_ledger_is_exact():
    """Weights are halved per cloning (Sec. 2): per primary the final weights sum to 1
    exactly, and histogram + under/overflow + backscatter + quarantine = primaries."""
    c = cfg(species=("B",), dx_max=0.1, thresholds=[[40.0, 70.0, 100.0]], n_bins=256)
    prim = oracle.sample_primaries(oracle.SamplerCfg(E_min=1000.0, E_max=1000.0), 0, 96)
    r = _run(c, prim)
    st, log = r["stats"], r["log"]
    assert st["clones"] > 0
    tot = r["hist"].sum() + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + st["w_quarantined"]
    assert tot == 96.0
    assert st["w_stopped"] == r["hist"].sum() + st["w_underflow"] + st["w_overflow"]
    per = np.zeros(96)
    np.add.at(per, log["lineage"], log["w"])
    assert (per == 1.0).all()
    assert len(log) == st["finished"] == 96 + st["clones"]
    # a clone's weight is 2^-(number of thresholds it has crossed)
    assert (log["w"] == 2.0 ** (-log["next_k"].astype(float))).all()


def test_splitting_is_unbiased_against_brute_force():
    """Brute force without splitting vs REED splitting on a tiny case: the weighted
    probabilities of the depth intervals agree within their statistical errors, and the
    weighted two-sample KS test passes."""
    base = dict(species=("B",), dx_max=0.1, n_bins=512)
    sc = oracle.SamplerCfg()
    n = 1536
    prim = oracle.sample_primaries(sc, 11, n)
    brute = _run(cfg(**base), prim)["log"]
    thr = [60.0, 100.0, 140.0]
    prim2 = oracle.sample_primaries(sc, 12, n)
    split = _run(cfg(thresholds=[thr], **base), prim2)["log"]
    b = brute[brute["status"] == oracle.STOPPED]
    s = split[split["status"] == oracle.STOPPED]
    edges = [-10.0] + thr + [1e9]
    for lo, hi in zip(edges[:-1], edges[1:]):
        mb = (b["z_stop"] >= lo) & (b["z_stop"] < hi)
        pb = mb.sum() / n
        eb = math.sqrt(max(pb * (1 - pb), 1.0 / n) / n)
        # per-primary sums of weight in the interval give an unbiased estimator
        per = np.zeros(n)
        ms = (s["z_stop"] >= lo) & (s["z_stop"] < hi)
        np.add.at(per, s["lineage"][ms], s["w"][ms])
        ps = per.mean()
        es = max(per.std(ddof=1) / math.sqrt(n), 1.0 / n)
        assert abs(ps - pb) < 4.0 * math.hypot(eb, es), (lo, hi, ps, pb)
    D, pval = physref.weighted_ks(b["z_stop"], b["w"], s["z_stop"], s["w"])
    assert pval > 0.01
    # splitting puts more samples into the deepest interval than brute force
    assert (s["z_stop"] >= thr[-1]).sum() > 2 * (b["z_stop"] >= thr[-1]).sum()


def test_clones_share_material_until_new_cells_are_created():
    """Clones copy the full system and differ only through material created after the
    cloning (Sec. 2): with different keys, the two evolve bitwise identically until the
    domain shifts; at the shift the kept atoms still agree and only new atoms differ."""
    c = cfg(species=("B",))
    t1 = oracle.Track.start(c, B, 1000.0, [2.0, 2.5, -3.0], [0.05, 0.02, 1.0], 77)
    t1.advance(600, events=True)
    rec = t1.record()
    ir = rec.view(np.int64)
    rec2 = rec.copy()
    rec2.view(np.int64)[15] = 991   # a different crystal-realisation key
    a = oracle.Track.from_record(c, rec)
    b = oracle.Track.from_record(c, rec2)
    c0 = a.state()["center"].copy()
    for _ in range(5000):
        ra, rb = a.record(), b.record()
        a.step()
        b.step()
        sa, sb = a.state(), b.state()
        if (sa["center"] != c0).any():
            ex_old = oracle.slot_exists(c0)
            ex_new = oracle.slot_exists(sa["center"])
            # slots whose cell is unchanged keep their atoms
            kept = np.zeros(216, bool)
            for i in (-1, 0, 1):
                for j in (-1, 0, 1):
                    for k in (-1, 0, 1):
                        cc = sa["center"] + np.array([i, j, k])
                        if all(abs(cc - c0) <= 1) and cc[2] >= 0:
                            base = ((cc[0] % 3) * 9 + (cc[1] % 3) * 3 + (cc[2] % 3)) * 8
                            kept[base:base + 8] = True
            assert kept.sum() > 0 and (ex_new & ~kept).sum() > 0
            assert np.array_equal(sa["ax"][:, kept], sb["ax"][:, kept])
            assert np.array_equal(sa["av"][:, kept], sb["av"][:, kept])
            new = ex_new & ~kept
            assert (sa["ax"][:, new] != sb["ax"][:, new]).all()
            assert not np.array_equal(sa["F"], sb["F"])
            return
        assert np.array_equal(ra, rb) or np.array_equal(ra[:15], rb[:15])
        assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["ax"], sb["ax"])
    pytest.fail("no domain shift")


# --------------------------------------------------------------------------- sampler
def test_sampler_distributions():
    sc = oracle.SamplerCfg(choice=(0, 1, 2), E_min=1000.0, E_max=100000.0, n_energy_tables=2,
                           dir_mode=oracle.DIR_MIXED, n_cone=2000, half_angle=math.radians(0.5),
                           axis=(0.0, 1 / math.sqrt(2), 1 / math.sqrt(2)))
    n = 4000
    pr = oracle.sample_primaries(sc, 0, n)
    d = pr["dir"]
    assert np.allclose((d**2).sum(0), 1.0, atol=1e-14)
    ax = np.array([0.0, 1 / math.sqrt(2), 1 / math.sqrt(2)])
    cone = np.degrees(np.arccos(np.clip(ax @ d[:, :2000], -1, 1)))
    assert cone.max() <= 0.5 + 1e-9 and cone.mean() > 0.3
    tilt = np.degrees(np.arccos(d[2, 2000:]))
    assert np.allclose(tilt, 7.0, atol=1e-12)
    assert (pr["pos"][2] == -3.0).all() and pr["pos"][:2].min() >= 0 and pr["pos"][:2].max() < 5.431
    cnt = np.bincount(pr["species"], minlength=3)
    assert (abs(cnt - n / 3) < 5 * math.sqrt(n * 2 / 9)).all()
    lg = np.log10(pr["E0"] / 1000.0)
    assert lg.min() >= 0 and lg.max() <= 2
    band = pr["table"] % 2
    assert ((lg >= 1) == (band == 1)).mean() > 0.999
    assert (pr["table"] // 2 == pr["species"]).all()
    # distinct primaries get distinct keys; the same id always gets the same key
    assert len(set(pr["key"].tolist())) == n
    assert oracle.sample_primaries(sc, 0, 5, id0=10)["key"].tolist() == pr["key"][10:15].tolist()


# --------------------------------------------------------------------------- derivative
def test_forward_mode_derivative_matches_closed_form_without_collisions():
    """Nuclear force off, uniform stopping: the stopping depth is z0 + L with
    L = 2 (sqrt(E0) - sqrt(E_stop)) / (k N kL), so dz/dk = -L / k and dz/ds = 0.  The
    forward-mode derivative of the discrete map approaches the closed form as the step
    shrinks (O(dx_max): 2-3e-4 at 0.05 A, 3-5e-5 at 0.01 A, 1e-5 at 0.002 A); at
    dx_max = 0.05 A, where no step count changes within +-h, it equals central differences
    of the same map to 1e-7."""
    for sp, E0, k in ((B, 1000.0, 1.0), (P, 5000.0, 1.3)):
        errs = []
        for dx in (0.05, 0.01):
            c = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM, k=k, dx_max=dx)
            st, z, dk, ds, n = oracle.grad_track(c, sp, E0, [0.0, 0.0, -3.0], [0.0, 0.0, 1.0], 1)
            assert st == oracle.STOPPED and ds == 0.0
            errs.append(abs(dk / (-(z + 3.0) / k) - 1.0))
        assert errs[1] < 1e-4 and errs[1] < errs[0] / 3, (sp, errs)
    for sp, E0, k in ((B, 1000.0, 1.0), (P, 5000.0, 1.3)):
        def z_of(kk):
            c = cfg(pot_mode=oracle.POT_NONE, stop_mode=oracle.STOP_UNIFORM, k=kk)
            return oracle.grad_track(c, sp, E0, [0.0, 0.0, -3.0], [0.0, 0.0, 1.0], 1)
        dk = z_of(k)[2]
        fd = (z_of(k + 1e-6)[1] - z_of(k - 1e-6)[1]) / 2e-6
        assert abs(dk / fd - 1.0) < 1e-7, (sp, dk, fd)


def test_forward_mode_derivative_matches_finite_differences_on_short_tracks():
    """ZBL collisions and local stopping on: on short 300 eV B tracks the forward-mode
    derivatives equal central differences of the oracle's own stopping depth to 2e-5,
    on the tracks where differences at two step sizes agree to 1e-5 (the linear regime of
    the discrete map: the paths are chaotic, so d/ds needs h <= 1e-7)."""
    c = cfg(species=("B",))
    sc = oracle.SamplerCfg(choice=(0,), E_min=300.0, E_max=300.0, tilt=math.radians(7.0))
    pr = oracle.sample_primaries(sc, 3, 16)
    steps = {"k": (1e-6, 1e-7), "s": (1e-7, 1e-8)}
    checked = {"k": 0, "s": 0}
    for i in range(16):
        args = (0, pr["E0"][i], pr["pos"][:, i], pr["dir"][:, i], int(pr["key"][i]))
        st, z, dk, ds, n = oracle.grad_track(c, *args)
        if st != oracle.STOPPED:
            continue
        for name, d in (("k", dk), ("s", ds)):
            fd = []
            for h in steps[name]:
                zz = []
                for sign in (1, -1):
                    kw = {"k": c.k, "s": c.s}
                    kw[name] += sign * h
                    r = oracle.grad_track(cfg(species=("B",), **kw), *args)
                    zz.append(r[1] if r[0] == oracle.STOPPED else float("nan"))
                fd.append((zz[0] - zz[1]) / (2 * h))
            scale = max(abs(fd[0]), 1e-3)
            if not np.all(np.isfinite(fd)) or abs(fd[0] - fd[1]) > 1e-5 * scale:
                continue
            checked[name] += 1
            assert abs(d - fd[0]) <= 2e-5 * scale, (i, name, d, fd)
    assert checked["k"] >= 4 and checked["s"] >= 4, checked


# --------------------------------------------------------------------------- adaptive depths
def test_refined_depths_match_exponential_quantiles():
    """Survival exp(-z/mu) booked into 1 A bins: the re-placed depths are the quantiles
    -mu ln p up to the linear-in-S interpolation inside a bin (error <= dz^2 / (8 mu))."""
    mu, nb, dz = 200.0, 4096, 1.0
    S = np.exp(-np.arange(nb + 1) * dz / mu)
    ts = np.array([np.concatenate([S[:-1] - S[1:], [S[-1]], [1.0]])])
    probs = [2.0 ** -k for k in range(1, 9)]
    d = oracle.refine_depths(ts, nb, dz, probs, np.zeros((1, 8)), 1.0, min_weight=0.0)
    assert np.allclose(d[0], [-mu * math.log(p) for p in probs], atol=dz * dz / (8 * mu) + 1e-9)


def test_refined_depths_keep_unresolved_targets_and_spacing():
    """A target the histogram does not resolve keeps its old depth shifted by the move of the
    last placed one, an empty table keeps its depths, and the depths are raised to the
    previous one plus min_gap."""
    nb = 10
    ts = np.zeros((2, nb + 2))
    ts[0, :nb] = 1.0            # 10 units stopped uniformly in [0, 10) A
    ts[0, nb + 1] = 10.0        # everything booked for table 0; table 1 has no data
    old = np.array([[1.0, 2.0, 50.0], [7.0, 8.0, 9.0]])
    d = oracle.refine_depths(ts, nb, 1.0, [0.5, 0.25, 1e-4], old, 0.0, min_weight=0.0)
    # S(z) = (10 - z) / 10: 0.5 at 5 A, 0.25 at 7.5 A, 1e-4 at 9.999 A
    assert np.allclose(d[0], [5.0, 7.5, 9.999], rtol=0, atol=1e-12)
    assert np.array_equal(d[1], old[1])
    ts[0, nb] = 5.0             # 5 more units stopped beyond the histogram
    ts[0, nb + 1] = 15.0
    d = oracle.refine_depths(ts, nb, 1.0, [0.5, 0.25, 1e-4], old, 3.0, min_weight=0.0)
    # S(z) = (15 - z) / 15 on [0, 10]: 0.5 at 7.5 A (moved by 6.5 A); S never falls below 1/3,
    # so the deeper targets keep 2.0 and 50.0 shifted by 6.5 A, raised by the 3 A spacing
    assert np.allclose(d[0], [7.5, 10.5, 56.5], rtol=0, atol=1e-12)
    assert np.array_equal(d[1], [7.0, 10.0, 13.0])


def test_refined_depths_hold_targets_the_statistics_are_too_thin_for():
    """A target is placed only where target x booked weight reaches min_weight (less than that
    much weight expected beyond the depth: the depth moves with the last placed one); scaling
    the statistics up resolves the deeper targets at the same places, since S does not change."""
    nb = 10
    ts = np.zeros((1, nb + 2))
    ts[0, :nb] = 1.0            # 10 units stopped uniformly in [0, 10) A
    ts[0, nb + 1] = 10.0
    old = np.array([[1.0, 2.0, 30.0, 40.0]])
    probs = [0.5, 0.25, 0.05, 1e-4]
    # S(z) = (10 - z) / 10: 0.5 at 5 A, 0.25 at 7.5 A, 0.05 at 9.5 A, 1e-4 at 9.999 A
    d = oracle.refine_depths(ts, nb, 1.0, probs, old, 0.0)           # min_weight 1: two placed
    assert np.allclose(d[0], [5.0, 7.5, 35.5, 45.5], rtol=0, atol=1e-12)
    d = oracle.refine_depths(ts, nb, 1.0, probs, old, 0.0, min_weight=2.6)   # one placed
    assert np.allclose(d[0], [5.0, 6.0, 34.0, 44.0], rtol=0, atol=1e-12)
    d = oracle.refine_depths(ts * 100.0, nb, 1.0, probs, old, 0.0)   # 1,000 units booked
    assert np.allclose(d[0], [5.0, 7.5, 9.5, 19.5], rtol=0, atol=1e-12)
    d = oracle.refine_depths(ts * 1e4, nb, 1.0, probs, old, 0.0)     # 1e5 units
    assert np.allclose(d[0], [5.0, 7.5, 9.5, 9.999], rtol=0, atol=1e-12)


def test_family_moment_errors_reduce_to_textbook_forms():
    """The family-grouped standard errors used by the statistical parity tests: with one
    unit-weight sample per family they are the textbook SE of a mean, s / sqrt(n), and (to
    first order) of a standard deviation, sqrt(mu4 - sigma^4) / (2 sigma sqrt(n)); duplicating
    every sample inside its family (a clone pair of half weight each) changes nothing."""
    from tests.physref import family_moments
    rng = np.random.default_rng(4)
    z = rng.gamma(3.0, 20.0, 20000)
    m, sd, se_m, se_sd = family_moments(z, np.ones_like(z), np.arange(z.size))
    assert abs(m - z.mean()) < 1e-9 * m and abs(sd - z.std()) < 1e-9 * sd
    assert abs(se_m / (z.std() / math.sqrt(z.size)) - 1.0) < 1e-9
    mu4 = ((z - z.mean()) ** 4).mean()
    ref = math.sqrt(mu4 - z.var() ** 2) / (2.0 * z.std() * math.sqrt(z.size))
    assert abs(se_sd / ref - 1.0) < 1e-9
    z2 = np.repeat(z, 2)
    out2 = family_moments(z2, np.full(z2.size, 0.5), np.repeat(np.arange(z.size), 2))
    assert np.allclose(out2, (m, sd, se_m, se_sd), rtol=1e-9)


# --------------------------------------------------------------------------- interaction cut-off
def test_cutoff_beyond_the_domain_changes_nothing():
    """A cut-off larger than any ion-atom distance in the 27-cell domain (whose diagonal is
    3 a sqrt(3) = 28.2 A) skips no atom: every record of a track with domain moves equals the
    27-cell one bit for bit."""
    pr = oracle.sample_primaries(oracle.SamplerCfg(choice=(0, 1, 2), E_min=2000.0, E_max=20000.0), 4, 6)
    for i in range(6):
        args = (int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i], pr["dir"][:, i], int(pr["key"][i]))
        a = oracle.Track.start(cfg(), *args)
        b = oracle.Track.start(cfg(r_cut=1000.0), *args)
        for _ in range(4):
            a.advance(60, events=True)
            b.advance(60, events=True)
            assert np.array_equal(a.record().view(np.int64), b.record().view(np.int64))


@pytest.mark.parametrize("rc", [4.0, 5.0, 6.0])
def test_cutoff_keeps_exactly_the_atoms_within_range(rc):
    """With a cut-off, the ion force and density are the sums over the atoms within rc only
    (pair force -V'(r) (x_ion - x_j)/r and density weight from the pinned ZBL and density
    routines), atoms beyond rc carry zero force, atoms within carry their pair force."""
    c = cfg(r_cut=rc)
    c0 = cfg()
    pr = oracle.sample_primaries(oracle.SamplerCfg(choice=(0, 1, 2), E_min=1000.0, E_max=1000.0), 6, 4)
    for i in range(4):
        sp = int(pr["species"][i])
        x = np.array([30.1, 27.4, 40.3]) + np.array([0.37, 0.11, 0.73]) * i
        st = oracle.Track.start(c, sp, 1000.0, x, pr["dir"][:, i], int(pr["key"][i])).state()
        full = oracle.Track.start(c0, sp, 1000.0, x, pr["dir"][:, i], int(pr["key"][i])).state()
        ex = oracle.slot_exists(st["center"])
        assert np.array_equal(st["ax"], full["ax"])      # same crystal
        F = np.zeros(3)
        rho = 0.0
        n_in = 0
        for s in np.nonzero(ex)[0]:
            d = st["x"] - st["ax"][:, s]
            r = float(np.sqrt(d @ d))
            if r > rc:
                assert np.all(st["af"][:, s] == 0.0)
                continue
            n_in += 1
            _, dV = oracle.zbl(c, sp, r)
            F += -dV * d / r
            rho += oracle.density_weight(c, sp, r)
            assert np.allclose(st["af"][:, s], dV * d / r, rtol=1e-12, atol=0)
        assert 10 < n_in < int(ex.sum())
        assert np.allclose(st["F"], F, rtol=1e-12, atol=1e-12 * np.abs(full["F"]).max())
        assert abs(st["rho"] / rho - 1.0) < 1e-12


def test_track_log_holds_every_finished_track():
    """A shallow depth table makes the families split far more often than the log's first size
    guess (1 + n_clones x n_thresh tracks per primary): the log still holds every finished
    track once, and each family's weights sum to 1."""
    n = 16
    prim = oracle.sample_primaries(oracle.SamplerCfg(choice=(0,), E_min=1000.0, E_max=1000.0), 7, n)
    cfg = oracle.Config(species=("B",), thresholds=[[10.0, 20.0, 30.0, 40.0, 50.0, 60.0]])
    r = oracle.run(cfg, prim, nthreads=4, log=True)
    lg = r["log"]
    assert r["stats"]["finished"] > n * 13
    assert len(lg) == r["stats"]["finished"]
    per_family = np.bincount(lg["lineage"], weights=lg["w"], minlength=n)
    assert np.array_equal(per_family, np.ones(n))

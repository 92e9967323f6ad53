"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Per-step quantities are deterministic and compared element by element at
1e-10 relative (positions, velocities, forces, density; integers exactly).
Whole runs are chaotic and compared statistically (weighted two-sample KS
p > 0.01, mean and standard deviation of the depth within 1 %), plus exact
ledgers and bitwise launch-configuration invariance.
"""
import gzip
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from tests import physref
from tests.clone_keys import check_clone_keys as _check_clone_keys
from tests.workloads import C1_THRESHOLDS, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0810_4737_amd as R
    R._abi.load()
    return R


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context()
    yield c
    c.close()


SPECIES3 = ("B", "P", "As")


def ocfg(**kw):
    kw.setdefault("species", SPECIES3)
    return oracle.Config(**kw)


def rcfg(R, **kw):
    return R.RunConfig(**kw)


def _prims(n, seed=3):
    sc = oracle.SamplerCfg(choice=(0, 1, 2), E_min=1000.0, E_max=20000.0)
    return oracle.sample_primaries(sc, seed, n)


def _exists(rec):
    ir = rec.view(np.int64)
    return oracle.slot_exists(ir[12:15])


def assert_records_close(got, ref, rtol=1e-10, what=""):
    """Compares two exchange records: integers exactly, floats to rtol relative to the
    larger of the value and a floor of 1e-9 times the field's largest magnitude."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    gi, ri = got.view(np.int64), ref.view(np.int64)
    assert np.array_equal(gi[12:22], ri[12:22]), (what, gi[12:22], ri[12:22])
    ex = _exists(ref)

    def cmp(a, b, name):
        scale = np.maximum(np.abs(b), 1e-9 * max(np.abs(b).max(), 1e-300))
        err = np.abs(a - b) / scale
        assert err.max() <= rtol, (what, name, float(err.max()), int(np.argmax(err)))

    cmp(got[0:3], ref[0:3], "x")
    cmp(got[3:6], ref[3:6], "v")
    # the ion force is a sum of cancelling terms: relative to the largest term
    fa = got[32 + 6 * 216: 32 + 9 * 216].reshape(3, 216)[:, ex]
    fb = ref[32 + 6 * 216: 32 + 9 * 216].reshape(3, 216)[:, ex]
    fscale = max(np.abs(fb).max(), np.abs(ref[6:9]).max(), 1e-300)
    assert np.abs(got[6:9] - ref[6:9]).max() <= rtol * fscale, (what, "F", got[6:9], ref[6:9])
    assert abs(got[9] - ref[9]) <= rtol * abs(ref[9]) + 1e-300, (what, "rho")
    assert got[10] == ref[10]
    A = got[32:].reshape(9, 216)[:, ex]
    B = ref[32:].reshape(9, 216)[:, ex]
    for f, name in ((slice(0, 3), "ax"), (slice(3, 6), "av"), (slice(6, 9), "af")):
        cmp(A[f].ravel(), B[f].ravel(), name)


# ----------------------------------------------------------------------------- exp
@pytest.mark.parametrize("pair", [False, True])
def test_library_exponential_is_accurate(R, pair):
    """The kernels' exp(-y) (Cody-Waite + minimax polynomial) against numpy's exp over the
    argument range of the force terms and the gradual-underflow tail: the friction factors'
    exponential to <= 4 ulp; the pair terms' base-2 one (degree 8) to its minimax bound
    1.08e-12 plus the rounding of the base-2 rate and of the result (<= 1.15e-12), 90 x inside
    the per-step tolerance of 1e-10."""
    y = np.concatenate([np.linspace(0.0, 50.0, 200001), np.geomspace(1e-12, 700.0, 100001),
                        np.linspace(700.0, 745.0, 1001)])
    got = R.eval_exp_neg(torch.as_tensor(y, device="cuda"), pair=pair).cpu().numpy()
    ref = np.exp(-y)
    normal = ref > 2.3e-308
    rel = np.abs(got[normal] - ref[normal]) / ref[normal]
    _say(f"exp_neg pair={pair}: worst relative error {rel.max():.3g}")
    bound = 1.15e-12 if pair else 4 * 2.0**-52
    assert rel.max() <= bound, rel.max()
    assert rel.max() > (1e-13 if pair else 0.0) or not pair   # the degree-8 polynomial really ran
    # gradual underflow: the relative bound of the polynomial plus the rounding to the grid of
    # subnormals (ldexp rounds once)
    sub = ~normal
    assert np.all(np.abs(got[sub] - ref[sub]) <= bound * ref[sub] + 4 * 5e-324)


def test_library_logarithm_is_accurate(R):
    """The logarithm of the Brandt-Kitagawa stopping (atanh series after the binary exponent
    is split off) against numpy over the normal range and around 1, and ln(1 + x) down to
    x = 1e-300: within 4 ulp of the value (the series' truncation is below 1e-19, the rest is
    the rounding of the division, the series and the final sums)."""
    x = np.concatenate([np.geomspace(2.3e-308, 1.7e308, 200001), 1.0 + np.linspace(-0.3, 0.3, 100001),
                        np.linspace(0.5, 4.0, 100001)])
    got = R.eval_log(torch.as_tensor(x, device="cuda")).cpu().numpy()
    ref = np.log(x)
    scale = np.maximum(np.abs(ref), 1e-300)
    rel = np.abs(got - ref) / scale
    _say(f"log: worst relative error {rel.max():.3g}")
    assert rel.max() <= 4 * 2.0 ** -52
    assert got[x == 1.0].max() == 0.0 and np.count_nonzero(x == 1.0) == 1
    y = np.concatenate([np.geomspace(1e-300, 1e300, 200001), np.linspace(0.0, 10.0, 100001)])
    got1 = R.eval_log(torch.as_tensor(y, device="cuda"), one_plus=True).cpu().numpy()
    ref1 = np.log1p(y)
    rel1 = np.abs(got1 - ref1) / np.maximum(np.abs(ref1), 1e-300)
    _say(f"log1p: worst relative error {rel1.max():.3g}")
    assert rel1[y > 0].max() <= 4 * 2.0 ** -52 and got1[y == 0.0].max() == 0.0


# ----------------------------------------------------------------------------- sampler
def test_sampler_matches_oracle(R, ctx):
    sc = dict(choice=(0, 1, 2), E_min=1000.0, E_max=100000.0, n_energy_tables=2, dir_mode=2,
              n_cone=3000, half_angle=math.radians(0.5), axis=(0.0, 2 ** -0.5, 2 ** -0.5),
              tilt=math.radians(7.0))
    n = 6000
    ref = oracle.sample_primaries(oracle.SamplerCfg(**sc), 5, n, id0=7)
    got = R.sample_primaries(ctx, R.SamplerConfig(**sc), 5, n, id0=7)
    torch.cuda.synchronize()
    assert np.array_equal(got["species"].cpu().numpy(), ref["species"])
    assert np.array_equal(got["table"].cpu().numpy(), ref["table"])
    assert np.array_equal(got["key"].cpu().numpy().view(np.uint64), ref["key"])
    for k in ("energy", "pos"):
        g = got[k].cpu().numpy()
        r = ref["E0" if k == "energy" else k]
        assert np.allclose(g, r, rtol=1e-14, atol=1e-15), k
    # cone directions go through 1 - cos(theta)^2 with cos(theta) ~ 1 - 4e-5: the sine
    # component carries ~1e-12 relative rounding (absolute ~1e-14)
    g = got["dir"].cpu().numpy()
    assert np.abs(g - ref["dir"]).max() < 5e-13


def test_empty_batch_and_argument_errors(R, ctx):
    b = R.empty_batch(0)
    h, s, _ = R.run(ctx, ("B",), b, rcfg(R))
    torch.cuda.synchronize()
    assert float(h.sum()) == 0.0 and R.parse_stats(s)["finished"] == 0
    with pytest.raises(R.ReedmdError):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, lanes_per_track=48))
    with pytest.raises(R.ReedmdError):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, n_bins=0))
    with pytest.raises(R.ReedmdError):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, thresholds=[[10.0, 20.0]], n_clones=1))
    # recoil options are fluorite-only; unknown modes and precisions are rejected
    with pytest.raises(R.ReedmdError, match="fluorite"):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, range_mode=R.RANGE_RADIAL))
    with pytest.raises(R.ReedmdError, match="fluorite"):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, vacancy=1))
    with pytest.raises(R.ReedmdError, match="range_mode"):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, range_mode=7))
    with pytest.raises(R.ReedmdError, match="force_precision"):
        R.run(ctx, ("B",), R.empty_batch(4), rcfg(R, force_precision=3))
    with pytest.raises(R.ReedmdError, match="start mode"):
        R.sample_primaries(ctx, R.SamplerConfig(start_mode=5), 0, 4)
    with pytest.raises(R.ReedmdError, match="direction mode"):
        R.sample_primaries(ctx, R.SamplerConfig(dir_mode=9), 0, 4)


# ----------------------------------------------------------------------------- per step
@pytest.mark.parametrize("lanes", [64, 32, 16])
def test_initial_domain_and_forces_match_oracle(R, ctx, lanes):
    n = 48
    pr = _prims(n)
    # put some starts deep inside the crystal as well
    pr["pos"][2, ::3] = 37.3 + 11.0 * np.arange(len(pr["pos"][2, ::3]))
    got = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr), rcfg(R, lanes_per_track=lanes)).cpu().numpy()
    c = ocfg()
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        assert_records_close(got[i], t.record(), what=f"init {i} lanes {lanes}")


def _oracle_states(n, seed=4, max_adv=2500, near_shift=False):
    """Oracle records of tracks advanced a random number of steps (atoms recoiling)."""
    pr = _prims(n, seed)
    c = ocfg()
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        t.advance(int(rng.integers(0, max_adv)), events=True)
        if near_shift:
            # stop right before a step that moves the domain
            c0 = t.state()["center"].copy()
            for _ in range(4000):
                prev = t.record()
                t.step()
                if (t.state()["center"] != c0).any():
                    t = oracle.Track.from_record(c, prev)
                    break
        recs.append(t.record())
    return c, np.array(recs)


@pytest.mark.parametrize("near_shift", [False, True])
def test_one_step_matches_oracle(R, ctx, near_shift):
    c, recs = _oracle_states(40, seed=5 + int(near_shift), near_shift=near_shift)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, rcfg(R, lanes_per_track=64), nsteps=1)
    got = dev.cpu().numpy()
    shifted = 0
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.step()
        ref = t.record()
        shifted += int((ref.view(np.int64)[12:15] != recs[i].view(np.int64)[12:15]).any())
        assert_records_close(got[i], ref, what=f"step {i}")
    if near_shift:
        assert shifted >= 0.9 * len(recs)   # a few tracks stop before their next shift


def test_twenty_steps_match_oracle(R, ctx):
    c, recs = _oracle_states(24, seed=9)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, rcfg(R), nsteps=20)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.advance(20, events=False)
        assert_records_close(got[i], t.record(), rtol=1e-8, what=f"20 steps {i}")


@pytest.mark.parametrize("lanes", [32, 16])
def test_lane_layouts_agree_bitwise(R, ctx, lanes):
    """The segment sums (ion force, density) follow one fixed order over the domain slots for
    every lane layout, so starting records and steps are bitwise identical at 64, 32 and 16
    lanes per track (the launch shape the autotuner picks changes no result)."""
    c, recs = _oracle_states(16, seed=11)
    a = torch.as_tensor(recs.copy(), device="cuda")
    b = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, a, rcfg(R, lanes_per_track=64), nsteps=5)
    R.debug_step(ctx, SPECIES3, b, rcfg(R, lanes_per_track=lanes), nsteps=5)
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    for i in range(len(recs)):
        assert np.array_equal(gb[i].view(np.int64), ga[i].view(np.int64)), f"lanes {lanes} record {i}"
    pr = _prims(24, seed=13)
    ia = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr), rcfg(R, lanes_per_track=64)).cpu().numpy()
    ib = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr), rcfg(R, lanes_per_track=lanes)).cpu().numpy()
    assert np.array_equal(ia.view(np.int64), ib.view(np.int64))


# ------------------------------------------------------------------ FP32 pair-term variant
# Force precision option: the pair term (distance, screening exponentials, density weight)
# in FP32, integration and step control in FP64; per-step tolerance 1e-5 relative.
@pytest.mark.parametrize("lanes", [64, 16])
def test_fp32_initial_forces_match_oracle(R, ctx, lanes):
    n = 48
    pr = _prims(n, seed=13)
    pr["pos"][2, ::3] = 37.3 + 11.0 * np.arange(len(pr["pos"][2, ::3]))
    cfg = rcfg(R, lanes_per_track=lanes, force_precision=R.FORCE_FP32)
    got = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr), cfg).cpu().numpy()
    c = ocfg()
    worst = 0.0
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        ref = t.record()
        assert_records_close(got[i], ref, rtol=1e-5, what=f"fp32 init {i} lanes {lanes}")
        ex = _exists(ref)
        # the domain itself does not depend on the force precision: FP64 tolerance
        xa = got[i][32:32 + 3 * 216].reshape(3, 216)[:, ex]
        xb = ref[32:32 + 3 * 216].reshape(3, 216)[:, ex]
        assert np.abs(xa - xb).max() <= 1e-10 * np.abs(xb).max(), ("fp32 init domain", i)
        fa = got[i][32 + 6 * 216:].reshape(3, 216)[:, ex]
        fb = ref[32 + 6 * 216:].reshape(3, 216)[:, ex]
        worst = max(worst, float((np.abs(fa - fb) / np.maximum(np.abs(fb), 1e-300)).max()))
    _say(f"fp32 init lanes {lanes}: worst atom-force relative error {worst:.3g}")
    assert worst > 0.0     # the FP32 path really ran


def test_fp32_one_step_matches_oracle(R, ctx):
    c, recs = _oracle_states(40, seed=21)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, rcfg(R, lanes_per_track=64, force_precision=R.FORCE_FP32), nsteps=1)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.step()
        assert_records_close(got[i], t.record(), rtol=1e-5, what=f"fp32 step {i}")


def test_fp32_rejected_by_the_adjoint(R, ctx):
    b = R.sample_primaries(ctx, R.SamplerConfig(), 0, 8)
    with pytest.raises(R.ReedmdError, match="FP64"):
        R.grad(ctx, ("B",), b, rcfg(R, force_precision=R.FORCE_FP32), k=1.0, s=1.0)


# ----------------------------------------------------------------------------- whole runs
def _load_golden(name):
    meta = json.load(open(os.path.join(GOLDEN, name + ".json")))
    zw = np.loadtxt(gzip.open(os.path.join(GOLDEN, name + "_stopped.txt.gz"), "rt"))
    return meta, zw[:, 0], zw[:, 1]


def _moments(z, w):
    W = w.sum()
    m = (w * z).sum() / W
    return m, math.sqrt((w * (z - m) ** 2).sum() / W)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c0_acceptance_set_matches_oracle_statistics(R, ctx, precision):
    """65,536 B at 1 keV (the 256-ion workload's sampler, extended): exact ledger, weighted
    KS p > 0.01 and mean/std of the stopping depth within 1 % of the stored FP64 oracle run,
    for the FP64 path and for the FP32 pair-term variant."""
    meta, zo, wo = _load_golden("c0_accept")
    w = WORKLOADS["c0_b1kev"]
    n = meta["workload"]["n"]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    fp = R.FORCE_FP32 if precision == "fp32" else R.FORCE_FP64
    hist, stats, log, _ = R.run(ctx, w["species"], batch, rcfg(R, n_bins=w["n_bins"], force_precision=fp),
                                log_cap=n + 16)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    _say(f"c0 {precision} gpu stats {st}")
    assert st["primaries"] == n and st["finished"] == n
    assert st["w_stopped"] + st["w_backscattered"] + st["w_quarantined"] == n
    assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] == st["w_stopped"]
    lg = R.parse_log(log, st["log_count"])
    s = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    mg, sg = _moments(s["z_stop"], s["w"])
    _say(f"c0 KS D={D:.4g} p={p:.3g} mean {mg:.4f} vs {meta['mean']:.4f} std {sg:.4f} vs {meta['std']:.4f}")
    assert p > 0.01
    assert abs(mg / meta["mean"] - 1) < 0.01 and abs(sg / meta["std"] - 1) < 0.01
    assert abs(st["n_backscattered"] - meta["stats"]["n_backscattered"]) < 5 * math.sqrt(meta["stats"]["n_backscattered"] + 1)


def test_adaptive_depths_follow_the_oracle_rule_and_statistics(R, ctx):
    """Cloning depths re-placed between epochs (2,048 B at 1 keV, 6 depths at survival 2^-k,
    4 epochs from a shallow first table): every table the GPU ran with equals the oracle's
    rule (oracle.refine_depths) applied to the GPU's own tracks of the earlier epochs, to
    1e-6 A; the ledger is exact; the weighted stopping depths match the stored oracle run of
    the same procedure (KS p > 0.01)."""
    meta, zo, wo = _load_golden("c0_refined")
    w = WORKLOADS["c0_b1kev"]
    m = meta["workload"]
    n, E, probs, first, gap = m["n"], m["n_epochs"], m["probs"], m["first"], m["min_gap"]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    cfg = rcfg(R, n_bins=w["n_bins"], thresholds=[first], form=R.FORM_PERSISTENT)
    hist, stats, depths, log = R.run_refined(ctx, w["species"], batch, cfg, E, probs, gap, log_cap=200000)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    assert st["primaries"] == n
    assert st["w_stopped"] + st["w_backscattered"] + st["w_quarantined"] == n
    assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] == st["w_stopped"]
    lg = R.parse_log(log, st["log_count"])
    assert len(lg) == st["finished"]
    d = depths.cpu().numpy()
    assert np.array_equal(d[0], [first])
    tables = batch["table"].cpu().numpy()
    bounds = [n * e // E for e in range(E + 1)]
    for e in range(1, E):
        ts = oracle.table_stats(lg[lg["lineage"] < bounds[e]], tables, 1, w["n_bins"], w["bin_width"])
        ref = oracle.refine_depths(ts, w["n_bins"], w["bin_width"], probs, d[e - 1], gap)
        assert np.allclose(d[e], ref, rtol=0, atol=1e-6), (e, d[e], ref)
    s = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    _say(f"refined depths {np.round(d[:, 0], 1).tolist()} vs oracle "
         f"{np.round(np.array(meta['depths'])[:, 0], 1).tolist()}; KS D={D:.4g} p={p:.3g}")
    assert p > 0.01


def test_in_launch_depths_follow_the_oracle_rule_and_statistics(R, ctx):
    """The same refinement inside one persistent launch (16,384 B at 1 keV, 6 depths, 4 epochs
    of claim positions, 32 lanes per track with the 64-lane tail, one block per CU: 2,048
    segments, so every later epoch starts after thousands of families have finished): every
    table version equals the
    oracle's rule applied to the statistics snapshot it was placed from, starting from the
    first table, to 1e-6 A; each snapshot is exactly a part of the run's final per-table
    statistics (dyadic weights: sums are exact); the ledger is exact; the weighted stopping
    depths match the stored oracle run of the epoch procedure (KS p > 0.01).  The plain form
    is rejected."""
    meta, zo, wo = _load_golden("c0_refined")
    w = WORKLOADS["c0_b1kev"]
    m = meta["workload"]
    n, E, probs, first, gap = 16384, m["n_epochs"], m["probs"], m["first"], m["min_gap"]
    nb, bw = w["n_bins"], w["bin_width"]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    cfg = rcfg(R, n_bins=nb, thresholds=[first], form=R.FORM_PERSISTENT, lanes_per_track=32, waves_per_cu=1)
    shape = R.launch_shape(ctx, batch, cfg)
    _say(f"in-launch refinement shape {shape}")
    assert shape["segments"] <= n // (2 * E)
    snaps = torch.zeros((E, 1, nb + 2), dtype=torch.float64, device="cuda")
    hist, stats, depths, log = R.run_refined(ctx, w["species"], batch, cfg, E, probs, gap, log_cap=1000000,
                                             in_launch=True, snapshots=snaps)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    _say(f"in-launch refinement stats {st}")
    assert st["primaries"] == n and st["error_flags"] == 0
    assert st["w_stopped"] + st["w_backscattered"] + st["w_quarantined"] == n
    assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] == st["w_stopped"]
    lg = R.parse_log(log, st["log_count"])
    assert len(lg) == st["finished"]
    d, S = depths.cpu().numpy(), snaps.cpu().numpy()
    assert np.array_equal(d[0], [first]) and not S[0].any()
    final = oracle.table_stats(lg, batch["table"].cpu().numpy(), 1, nb, bw)
    for e in range(1, E):
        assert S[e, 0, nb + 1] > 0.0, e
        assert np.all(S[e] <= final), e
        ref = oracle.refine_depths(S[e], nb, bw, probs, d[0], gap)
        assert np.allclose(d[e], ref, rtol=0, atol=1e-6), (e, d[e], ref)
    s = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    _say(f"in-launch depths {np.round(d[:, 0], 1).tolist()} from booked weight "
         f"{S[:, 0, nb + 1].tolist()}; KS D={D:.4g} p={p:.3g}")
    assert p > 0.01
    with pytest.raises(R.ReedmdError, match="persistent"):
        R.run_refined(ctx, w["species"], batch, rcfg(R, n_bins=nb, thresholds=[first]), E, probs, gap,
                      in_launch=True)


def test_in_launch_refinement_edge_cases(R, ctx):
    """One epoch in one launch is the plain persistent run (histogram and totals bitwise, the
    caller's table reported); more epochs than primaries run one primary per epoch (exact
    ledger, a table version per epoch); a snapshot tensor of the wrong shape is rejected."""
    w = WORKLOADS["c0_b1kev"]
    first = [10.0, 20.0, 30.0, 40.0]
    probs = [0.5, 0.25, 0.125, 0.0625]
    cfg = rcfg(R, n_bins=w["n_bins"], thresholds=[first], form=R.FORM_PERSISTENT, lanes_per_track=32)
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, 512)
    h1, s1, d1 = R.run_refined(ctx, w["species"], batch, cfg, 1, probs, 1.0, in_launch=True)
    h0, s0, _ = R.run(ctx, w["species"], batch, cfg)
    torch.cuda.synchronize()
    assert torch.equal(h1, h0)
    a, b = R.parse_stats(s1), R.parse_stats(s0)
    for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped", "w_stopped"):
        assert a[k] == b[k], k
    assert np.array_equal(d1.cpu().numpy(), [[first]])
    small = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, 8)
    h, st, d = R.run_refined(ctx, w["species"], small, cfg, 64, probs, 1.0, in_launch=True)
    torch.cuda.synchronize()
    st = R.parse_stats(st)
    assert d.shape == (8, 1, 4) and st["primaries"] == 8
    assert float(h.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
        st["w_quarantined"] == 8.0
    with pytest.raises(ValueError, match="snapshots"):
        R.run_refined(ctx, w["species"], small, cfg, 2, probs, 1.0, in_launch=True,
                      snapshots=torch.zeros((2, 1, 7), dtype=torch.float64, device="cuda"))


def test_in_launch_depths_on_the_mixed_workload_six_tables(R, ctx):
    """In-launch refinement with several tables (16,384 mixed B/P/As primaries at 1-100 keV,
    the six (species, energy decade) tables of 12 depths as the first versions, targets
    10^(-5k/12), 4 epochs, 32 lanes, one workgroup per CU): every version of every table is the
    oracle's rule applied to its snapshot (1e-6 A), each snapshot is bounded by the run's final
    per-table statistics element by element, and the ledger is exact."""
    from tests.workloads import C2_THRESHOLDS
    w = WORKLOADS["c2_mixed"]
    n, E, gap = 16384, 4, 1.0
    nb, bw = w["n_bins"], w["bin_width"]
    probs = [10.0 ** (-5.0 * k / 12.0) for k in range(1, 13)]
    first = [list(t) for t in C2_THRESHOLDS]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    cfg = rcfg(R, n_bins=nb, bin_width=bw, thresholds=first, form=R.FORM_PERSISTENT, lanes_per_track=32,
               waves_per_cu=4)
    shape = R.launch_shape(ctx, batch, cfg)
    assert shape["segments"] <= n // (2 * E)
    snaps = torch.zeros((E, 6, nb + 2), dtype=torch.float64, device="cuda")
    hist, stats, depths, log = R.run_refined(ctx, w["species"], batch, cfg, E, probs, gap, log_cap=1000000,
                                             in_launch=True, snapshots=snaps)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    _say(f"in-launch refinement, six tables: {st}")
    assert st["primaries"] == n and st["error_flags"] == 0
    assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
        st["w_quarantined"] == float(n)
    lg = R.parse_log(log, st["log_count"])
    assert len(lg) == st["finished"]
    d, S = depths.cpu().numpy(), snaps.cpu().numpy()
    assert np.array_equal(d[0], np.array(first)) and not S[0].any()
    final = oracle.table_stats(lg, batch["table"].cpu().numpy(), 6, nb, bw)
    moved = 0
    for e in range(1, E):
        assert np.all(S[e] <= final), e
        # claims run longest-expected first, so a table of short tracks may have booked nothing
        # when the first epochs begin (its depths then stay); some table always has
        assert S[e][:, nb + 1].max() > 0.0, e
        ref = oracle.refine_depths(S[e], nb, bw, probs, d[0], gap)
        assert np.allclose(d[e], ref, rtol=0, atol=1e-6), (e, np.abs(d[e] - ref).max())
        moved += int(np.sum(np.abs(d[e] - d[0]) > 1.0))
    _say(f"six-table versions: {moved} depths moved by more than 1 A; last {np.round(d[-1][:, :3], 1).tolist()}")
    assert moved > 0


def _c1_subset_batches(R, ctx):
    w = WORKLOADS["c1_as10kev"]
    sc = R.SamplerConfig(**w["sampler"])
    return [(R.sample_primaries(ctx, sc, 0, 512, id0=0), 0),
            (R.sample_primaries(ctx, sc, 0, 512, id0=32768), 32768)]


def _run_c1_subset(R, ctx, **kw):
    w = WORKLOADS["c1_as10kev"]
    cfg = rcfg(R, n_bins=w["n_bins"], thresholds=[list(C1_THRESHOLDS)], **kw)
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    logs = []
    for b, id0 in _c1_subset_batches(R, ctx):
        _, _, log, _ = R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, log_cap=40000)
        logs.append(log)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    return hist.cpu().numpy(), st, logs


def test_splitting_run_matches_oracle_and_forms_agree_bitwise(R, ctx):
    """1,024 As at 10 keV with 8 cloning depths: exact weight ledger; plain and persistent
    forms (and a tiny queue that forces the overflow path), at 16, 32 and 64 lanes per track,
    give bitwise-identical histograms and equal totals; every clone key derives from its
    primary's key as the oracle derives it;
    the weighted depth distribution agrees with the stored oracle run (KS p > 0.01)."""
    meta, zo, wo = _load_golden("c1_subset")
    _say("c1 subset plain")
    hp, sp, logs = _run_c1_subset(R, ctx, form=R.FORM_PLAIN)
    _say(f"plain stats {sp}")
    assert sp["primaries"] == 1024
    tot = hp.sum() + sp["w_underflow"] + sp["w_overflow"] + sp["w_backscattered"] + sp["w_quarantined"]
    assert tot == 1024.0
    assert sp["clones"] > 0 and sp["error_flags"] == 0
    _say("c1 subset persistent")
    hq, sq, _ = _run_c1_subset(R, ctx, form=R.FORM_PERSISTENT)
    assert np.array_equal(hp, hq)
    for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped", "n_backscattered"):
        assert sp[k] == sq[k], k
    _say("c1 subset persistent, queue of 2")
    ht, stt, _ = _run_c1_subset(R, ctx, form=R.FORM_PERSISTENT, queue_capacity=2)
    assert np.array_equal(hp, ht)
    assert stt["stack_overflow"] > 0
    for lanes in (16, 32, 64):
        _say(f"c1 subset persistent, {lanes} lanes per track")
        hl, sl, _ = _run_c1_subset(R, ctx, form=R.FORM_PERSISTENT, lanes_per_track=lanes)
        assert np.array_equal(hp, hl), lanes
        for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped", "n_backscattered"):
            assert sp[k] == sl[k], (lanes, k)
    # statistics vs the oracle
    allg = np.concatenate([R.parse_log(l, l.shape[0]) for l in logs])
    allg = allg[allg["status"] != 0]          # unused log rows are all zero
    assert len(allg) == sp["finished"]
    fam = _check_clone_keys(allg)
    assert fam == 1024
    g = allg[allg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(g["z_stop"], g["w"], zo, wo)
    _say(f"c1 KS D={D:.4g} p={p:.3g}; gpu clones {sp['clones']} oracle {meta['stats']['clones']}; "
         f"clone keys checked on {len(allg)} tracks of {fam} families")
    assert p > 0.01


def test_cancel_drains_with_exact_ledger(R, ctx):
    w = WORKLOADS["c1_as10kev"]
    for form in (R.FORM_PLAIN, R.FORM_PERSISTENT):
        b = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, 300)
        cancel = torch.ones(1, dtype=torch.int32, device="cuda")
        h, s, _ = R.run(ctx, w["species"], b, rcfg(R, n_bins=w["n_bins"], thresholds=[list(C1_THRESHOLDS)],
                                                   form=form), cancel=cancel)
        torch.cuda.synchronize()
        st = R.parse_stats(s)
        assert st["n_cancelled"] == 300 and st["w_cancelled"] == 300.0 and float(h.sum()) == 0.0


def test_step_cap_quarantines(R, ctx):
    b = R.sample_primaries(ctx, R.SamplerConfig(), 0, 64)
    h, s, _ = R.run(ctx, ("B",), b, rcfg(R, max_steps=50))
    torch.cuda.synchronize()
    st = R.parse_stats(s)
    assert st["n_stepcap"] + st["n_stopped"] + st["n_backscattered"] == 64
    assert st["n_stepcap"] > 60 and st["w_quarantined"] == st["n_stepcap"]


def test_graph_replay_and_autotune_are_consistent(R, ctx):
    w = WORKLOADS["c0_b1kev"]
    b = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, 512)
    ref, _, _ = R.run(ctx, w["species"], b, rcfg(R, lanes_per_track=64))
    outs = []
    for _ in range(3):
        h, s, _ = R.run(ctx, w["species"], b, rcfg(R, lanes_per_track=64, form=R.FORM_PERSISTENT))
        torch.cuda.synchronize()
        outs.append(h.cpu().numpy())
    for o in outs:
        assert np.array_equal(o, ref.cpu().numpy())
    lanes, waves = R.autotune(ctx, w["species"], b, rcfg(R, form=R.FORM_PERSISTENT), pilot=256)
    assert lanes in (16, 32, 64)
    h, s, _ = R.run(ctx, w["species"], b, rcfg(R, form=R.FORM_PERSISTENT))
    torch.cuda.synchronize()
    assert R.parse_stats(s)["finished"] == 512


def test_graph_cache_keeps_one_pipeline_for_fresh_buffers(R):
    """The persistent pipeline graph is cached per launch shape, not per buffer address:
    50 runs whose batch, histogram and statistics are freshly allocated each time (all kept
    alive, so every call sees new addresses) keep one cached graph and give bitwise-equal
    histograms and equal statistics."""
    w = WORKLOADS["c0_b1kev"]
    c = R.Context()
    try:
        sc = R.SamplerConfig(**w["sampler"])
        cfg = rcfg(R, form=R.FORM_PERSISTENT, lanes_per_track=64, n_bins=w["n_bins"],
                   thresholds=[[20.0, 40.0, 60.0]])
        keep, hists, finished = [], [], set()
        for i in range(50):
            b = R.sample_primaries(c, sc, 0, 128)
            h, st, k = R.run(c, w["species"], b, cfg)
            keep.append((b, h, st, k))
            hists.append(h)
        torch.cuda.synchronize()
        assert len({h.data_ptr() for h in hists}) == 50
        assert c.cached_graphs() == 1
        ref = hists[0].cpu().numpy()
        for (b, h, st, k) in keep:
            assert np.array_equal(h.cpu().numpy(), ref)
            s = R.parse_stats(st)
            finished.add((s["finished"], s["clones"], s["track_steps"]))
            assert s["primaries"] == 128
        assert len(finished) == 1
        # a second launch shape adds a second graph (its larger clone stacks first empty the
        # cache, so the first shape is built again after it)
        R.run(c, w["species"], b, rcfg(R, form=R.FORM_PERSISTENT, lanes_per_track=16, n_bins=w["n_bins"],
                                        thresholds=[[20.0, 40.0, 60.0]]))
        h2, _, _ = R.run(c, w["species"], b, cfg)
        torch.cuda.synchronize()
        assert c.cached_graphs() == 2
        assert np.array_equal(h2.cpu().numpy(), ref)
    finally:
        c.close()


def _run_subset(R, ctx, wname, thresholds, ids, **kw):
    w = WORKLOADS[wname]
    sc = R.SamplerConfig(**w["sampler"])
    cfg = rcfg(R, n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=thresholds, **kw)
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    logs = []
    for id0, id1 in ids:
        b = R.sample_primaries(ctx, sc, 0, id1 - id0, id0=id0)
        _, _, log, _ = R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, log_cap=60000)
        logs.append(log)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    lg = np.concatenate([R.parse_log(l, l.shape[0]) for l in logs])
    lg = lg[lg["status"] != 0]
    return hist.cpu().numpy(), st, lg


@pytest.mark.parametrize("wname,thr_name,golden", [("c2_mixed", "c2", "c2_subset"),
                                                   ("c4_as100kev", "c4", "c4_subset")])
def test_mixed_and_deep_tail_workloads_match_oracle(R, ctx, wname, thr_name, golden):
    """Subsets of the mixed B/P/As 1-100 keV workload (6 cloning tables of 12 depths) and of
    the 100 keV As [001] channeling workload (16 depths to 1e-6): exact weight ledger; the
    persistent form with the autotuned launch shape, and with 16 lanes per track with and
    without the 64-lane tail launch, gives the same histogram and totals bitwise as the plain
    form; the weighted depth distribution agrees with the stored oracle run."""
    from tests.workloads import C2_THRESHOLDS, C4_THRESHOLDS
    thr = C2_THRESHOLDS if thr_name == "c2" else [list(C4_THRESHOLDS)]
    meta, zo, wo = _load_golden(golden)
    ids = meta["workload"]["ids"]
    n = sum(b - a for a, b in ids)
    hp, sp, lp = _run_subset(R, ctx, wname, thr, ids, form=R.FORM_PLAIN, lanes_per_track=64)
    _say(f"{wname} plain {sp}")
    tot = hp.sum() + sp["w_underflow"] + sp["w_overflow"] + sp["w_backscattered"] + sp["w_quarantined"]
    assert tot == float(n) and sp["error_flags"] == 0
    w = WORKLOADS[wname]
    sc = R.SamplerConfig(**w["sampler"])
    b = R.sample_primaries(ctx, sc, 0, ids[0][1] - ids[0][0], id0=ids[0][0])
    lanes, waves = R.autotune(ctx, w["species"], b, rcfg(R, n_bins=w["n_bins"], bin_width=w["bin_width"],
                                                         thresholds=thr, form=R.FORM_PERSISTENT),
                              pilot=min(64, n))
    _say(f"autotuned lanes {lanes} waves/CU {waves}")
    hq, sq, lq = _run_subset(R, ctx, wname, thr, ids, form=R.FORM_PERSISTENT, lanes_per_track=lanes,
                             waves_per_cu=waves)
    assert np.array_equal(hp, hq)
    assert sp["finished"] == sq["finished"] and sp["track_steps"] == sq["track_steps"]
    # 16 lanes with and without the 64-lane tail launch: the handed-off tracks continue
    # bit for bit, so histograms and totals are equal
    hh, sh, _ = _run_subset(R, ctx, wname, thr, ids, form=R.FORM_PERSISTENT, lanes_per_track=16)
    hn, sn, _ = _run_subset(R, ctx, wname, thr, ids, form=R.FORM_PERSISTENT, lanes_per_track=16, no_tail_handoff=1)
    _say(f"{wname}: tracks handed to the 64-lane tail launch {sh['handed_off']} (off: {sn['handed_off']})")
    assert sh["handed_off"] > 0 and sn["handed_off"] == 0
    assert np.array_equal(hp, hh) and np.array_equal(hp, hn)
    for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped", "n_backscattered", "n_stepcap"):
        assert sp[k] == sh[k] == sn[k], k
    s = lp[lp["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    _say(f"{wname} KS D={D:.4g} p={p:.3g}; gpu tracks {sp['finished']} oracle {meta['stats']['finished']}")
    assert p > 0.01

"""GPU parity of the fluorite (UO2) target, the recoil start and the radial range (through the
C ABI) against the FP64 oracle: starting domains and forces, single and twenty steps at the
FP64 tolerances (1e-10 per step, 1e-8 over twenty), the two lane layouts against each other,
the FP32 pair term at 1e-5, and the 85 keV U recoil subset with cloning against the stored
oracle run (weighted KS p > 0.01, exact ledger, plain and persistent forms bitwise equal).
"""
import gzip
import json
import os
import sys

import numpy as np
import pytest

import oracle
from tests import physref
from tests.workloads import C5_THRESHOLDS, UO2, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NS = oracle.NSLOT_FLUORITE
W5 = WORKLOADS["c5_u85kev_uo2"]
SPECIES = ("U", "B")


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
    c = R.Context(structure=R.FLUORITE, **UO2)
    yield c
    c.close()


def ocfg(**kw):
    d = dict(UO2)
    d.update(structure=oracle.FLUORITE, species=SPECIES, range_mode=oracle.RANGE_RADIAL, vacancy=1)
    d.update(kw)
    return oracle.Config(**d)


def rcfg(R, **kw):
    kw.setdefault("range_mode", R.RANGE_RADIAL)
    kw.setdefault("vacancy", 1)
    return R.RunConfig(**kw)


def _prims(n, seed=3):
    """Recoils on the cation site of cell (0, 0, 40) in random directions, U and B, 2-85 keV;
    every third entry moved off the site (no vacancy is then next to it)."""
    sc = oracle.SamplerCfg(choice=(0, 1), E_min=2000.0, E_max=85000.0, dir_mode=oracle.DIR_ISOTROPIC,
                           start_mode=oracle.START_SITE, a=UO2["a"], z_start=40 * UO2["a"])
    pr = oracle.sample_primaries(sc, seed, n)
    pr["pos"][0, 1::3] += 1.3
    pr["pos"][1, 1::3] += 0.4
    return pr


def assert_records_close(got, ref, rtol=1e-10, what=""):
    """Integers and the header's vacancy and start point exactly, floats to rtol relative to
    the larger of the value and 1e-9 times the field's largest magnitude; the ion force
    relative to the largest pair force."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    gi, ri = got.view(np.int64), ref.view(np.int64)
    assert np.array_equal(gi[12:22], ri[12:22]), (what, gi[12:22], ri[12:22])
    assert np.array_equal(gi[25:29], ri[25:29]), (what, "vacancy", gi[25:29], ri[25:29])
    assert np.array_equal(got[29:32], ref[29:32]), (what, "start point")
    st = oracle.unpack_record(ref)
    ex = oracle.slot_exists(st["center"], oracle.FLUORITE, st["vac_cell"], st["vac_basis"])

    def cmp(a, b, name):
        scale = np.maximum(np.abs(b), 1e-9 * max(np.abs(b).max(), 1e-300))
        err = np.abs(a - b) / scale
        assert err.max() <= rtol, (what, name, float(err.max()), int(np.argmax(err)))

    cmp(got[0:3], ref[0:3], "x")
    cmp(got[3:6], ref[3:6], "v")
    fb = ref[32 + 6 * NS: 32 + 9 * NS].reshape(3, NS)[:, ex]
    fscale = max(np.abs(fb).max(), np.abs(ref[6:9]).max(), 1e-300)
    assert np.abs(got[6:9] - ref[6:9]).max() <= rtol * fscale, (what, "F", got[6:9], ref[6:9])
    assert abs(got[9] - ref[9]) <= rtol * abs(ref[9]) + 1e-300, (what, "rho")
    assert got[10] == ref[10]
    A = got[32:].reshape(9, NS)
    B = ref[32:].reshape(9, NS)
    assert not A[:, ~ex].any(), (what, "empty slots must hold zeros")
    for f, name in ((slice(0, 3), "ax"), (slice(3, 6), "av"), (slice(6, 9), "af")):
        cmp(A[f][:, ex].ravel(), B[f][:, ex].ravel(), name)
    return ex


@pytest.mark.parametrize("lanes", [64, 32])
def test_fluorite_initial_domain_and_forces_match_oracle(R, ctx, lanes):
    n = 36
    pr = _prims(n)
    got = R.track_init(ctx, SPECIES, R.batch_from_numpy(pr), rcfg(R, lanes_per_track=lanes)).cpu().numpy()
    assert got.shape[1] == oracle.RECORD_WORDS_FLUORITE
    c = ocfg()
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        ex = assert_records_close(got[i], t.record(), what=f"init {i} lanes {lanes}")
        assert ex.sum() == 323      # the vacant site of every recoil is inside its first domain


def test_fluorite_lanes_16_is_rejected(R, ctx):
    pr = _prims(4)
    with pytest.raises(R.ReedmdError, match="32 or 64"):
        R.track_init(ctx, SPECIES, R.batch_from_numpy(pr), rcfg(R, lanes_per_track=16))


def _oracle_states(n, seed=4, max_adv=3000, near_shift=False):
    pr = _prims(n, seed)
    c = ocfg()
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        t.advance(int(rng.integers(0, max_adv)), events=True)
        if near_shift:
            c0 = t.state()["center"].copy()
            for _ in range(5000):
                prev = t.record()
                t.step()
                if (t.state()["center"] != c0).any():
                    t = oracle.Track.from_record(c, prev)
                    break
        recs.append(t.record())
    return c, np.array(recs)


@pytest.mark.parametrize("near_shift", [False, True])
def test_fluorite_one_step_matches_oracle(R, ctx, near_shift):
    c, recs = _oracle_states(30, seed=7 + int(near_shift), near_shift=near_shift)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES, dev, rcfg(R, lanes_per_track=64), nsteps=1)
    got = dev.cpu().numpy()
    shifted = 0
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.step()
        ref = t.record()
        shifted += int((ref.view(np.int64)[12:15] != recs[i].view(np.int64)[12:15]).any())
        assert_records_close(got[i], ref, what=f"step {i}")
    if near_shift:
        assert shifted >= 0.8 * len(recs)


def test_fluorite_twenty_steps_and_lane_layouts(R, ctx):
    c, recs = _oracle_states(20, seed=12)
    a = torch.as_tensor(recs.copy(), device="cuda")
    b = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES, a, rcfg(R, lanes_per_track=64), nsteps=20)
    R.debug_step(ctx, SPECIES, b, rcfg(R, lanes_per_track=32), nsteps=20)
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.advance(20, events=False)
        assert_records_close(ga[i], t.record(), rtol=1e-8, what=f"20 steps {i}")
        assert_records_close(gb[i], ga[i], rtol=1e-11, what=f"lanes 32 vs 64 {i}")


def test_fluorite_fp32_pair_term_one_step(R, ctx):
    c, recs = _oracle_states(24, seed=15)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES, dev, rcfg(R, lanes_per_track=32, force_precision=R.FORCE_FP32), nsteps=1)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.step()
        assert_records_close(got[i], t.record(), rtol=1e-5, what=f"fp32 step {i}")


def test_recoil_sampler_matches_oracle(R, ctx):
    n = 4000
    ref = oracle.sample_primaries(oracle.SamplerCfg(**W5["sampler"]), 9, n, id0=3)
    got = R.sample_primaries(ctx, R.SamplerConfig(**W5["sampler"]), 9, n, id0=3)
    torch.cuda.synchronize()
    assert np.array_equal(got["key"].cpu().numpy().view(np.uint64), ref["key"])
    assert np.array_equal(got["pos"].cpu().numpy(), ref["pos"])
    assert np.allclose(got["dir"].cpu().numpy(), ref["dir"], rtol=0, atol=2e-15)


def _load_golden(name):
    meta = json.load(open(os.path.join(HERE, "golden", name + ".json")))
    zw = np.loadtxt(gzip.open(os.path.join(HERE, "golden", name + "_stopped.txt.gz"), "rt"))
    return meta, zw[:, 0], zw[:, 1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_u_recoil_subset_matches_oracle(R, ctx, precision):
    """256 U recoils at 85 keV in UO2 with 8 radial cloning distances: exact weight ledger;
    plain and persistent forms give bitwise-identical histograms; the weighted distribution
    of the stopping distance agrees with the stored FP64 oracle run (KS p > 0.01), for the
    FP64 path and for the FP32 pair term."""
    meta, zo, wo = _load_golden("c5_subset")
    batch = R.sample_primaries(ctx, R.SamplerConfig(**W5["sampler"]), 0, 256)
    fp = R.FORCE_FP32 if precision == "fp32" else R.FORCE_FP64
    out = {}
    for form in (R.FORM_PLAIN, R.FORM_PERSISTENT):
        cfg = rcfg(R, n_bins=W5["n_bins"], bin_width=W5["bin_width"], thresholds=[list(C5_THRESHOLDS)],
                   form=form, force_precision=fp)
        hist, stats, log, _ = R.run(ctx, W5["species"], batch, cfg, log_cap=20000)
        torch.cuda.synchronize()
        st = R.parse_stats(stats)
        _say(f"c5 {precision} form {form} stats {st}")
        assert st["primaries"] == 256 and st["error_flags"] == 0
        tot = float(hist.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + st["w_quarantined"]
        assert tot == 256.0
        out[form] = (hist.cpu().numpy(), st, R.parse_log(log, st["log_count"]))
    hp, sp, lg = out[R.FORM_PLAIN]
    hq, sq, _ = out[R.FORM_PERSISTENT]
    assert np.array_equal(hp, hq)
    for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped"):
        assert sp[k] == sq[k], k
    s = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    _say(f"c5 {precision} KS D={D:.4g} p={p:.3g}; gpu clones {sp['clones']} oracle {meta['stats']['clones']}")
    assert p > 0.01


def test_u_recoil_adaptive_distances_follow_the_oracle_rule(R, ctx):
    """Eight cloning distances re-placed between 4 epochs (512 U recoils at 85 keV, survival
    2^-k, from a deliberately short first table; the setting of Sec. 4): every table the GPU ran
    with equals the oracle's rule applied to the GPU's own tracks of the earlier epochs, to 1e-6
    A; the ledger is exact; the weighted stopping distances match the stored oracle run of the
    same procedure (KS p > 0.01)."""
    meta, zo, wo = _load_golden("c5_refined")
    m = meta["workload"]
    n, E, probs, first, gap = m["n"], m["n_epochs"], m["probs"], m["first"], m["min_gap"]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**W5["sampler"]), 0, n)
    cfg = rcfg(R, n_bins=W5["n_bins"], bin_width=W5["bin_width"], thresholds=[first], form=R.FORM_PERSISTENT)
    hist, stats, depths, log = R.run_refined(ctx, W5["species"], batch, cfg, E, probs, gap, log_cap=200000)
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
        ts = oracle.table_stats(lg[lg["lineage"] < bounds[e]], tables, 1, W5["n_bins"], W5["bin_width"])
        ref = oracle.refine_depths(ts, W5["n_bins"], W5["bin_width"], probs, d[e - 1], gap)
        assert np.allclose(d[e], ref, rtol=0, atol=1e-6), (e, d[e], ref)
    s = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(s["z_stop"], s["w"], zo, wo)
    _say(f"c5 refined distances {np.round(d[:, 0], 1).tolist()} vs oracle "
         f"{np.round(np.array(meta['depths'])[:, 0], 1).tolist()}; KS D={D:.4g} p={p:.3g}")
    assert p > 0.01

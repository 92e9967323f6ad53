"""The Firsov + Brandt-Kitagawa stopping (paper Sec. 2, "Third") in the kernels, through the C
ABI: starting records and steps against the oracle's same model at 1e-10 (diamond at 64, 32
and 16 lanes, fluorite UO2 at 64 and 32), bitwise agreement of the lane layouts, the argument
errors of the unsupported combinations, and a whole run of 32,768 B at 1 keV against the stored
oracle run (weighted KS p > 0.01, mean and standard deviation within 1 % or three standard
errors of the difference)."""
import gzip
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from tests import physref
from tests import test_gpu_fluorite as FL
from tests.test_gpu_parity import SPECIES3, _prims, assert_records_close
from tests.workloads import UO2, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
N_E = 32.0 / 5.431 ** 3     # silicon's valence electrons per A^3


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


@pytest.fixture(scope="module", params=[N_E, 0.0], ids=["fk+bk", "fk"])
def model(R, request):
    n_e = request.param
    c = R.Context(stop_mode=R.STOP_FKBK, n_e=n_e)
    yield c, oracle.Config(species=SPECIES3, stop_mode=oracle.STOP_FKBK, n_e=n_e)
    c.close()


@pytest.mark.parametrize("lanes", [64, 32, 16])
def test_fkbk_initial_records_match_oracle(R, model, lanes):
    ctx, oc = model
    n = 36
    pr = _prims(n, seed=61)
    pr["pos"][2, ::3] = 31.7 + 9.0 * np.arange(len(pr["pos"][2, ::3]))
    got = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr), R.RunConfig(lanes_per_track=lanes)).cpu().numpy()
    for i in range(n):
        t = oracle.Track.start(oc, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        ref = t.record()
        assert_records_close(got[i], ref, what=f"init {i} lanes {lanes}")
    # the stored stopping weight is the Firsov sum, not the exponential density
    assert abs(ref[9] - oracle.Track.start(oracle.Config(species=SPECIES3), int(pr["species"][-1]),
                                           float(pr["E0"][-1]), pr["pos"][:, -1], pr["dir"][:, -1],
                                           int(pr["key"][-1])).record()[9]) > 1e-3 * abs(ref[9])


def _states(oc, n, seed, max_adv=2500):
    pr = _prims(n, seed)
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n):
        t = oracle.Track.start(oc, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        t.advance(int(rng.integers(0, max_adv)), events=True)
        recs.append(t.record())
    return np.array(recs)


def test_fkbk_steps_match_oracle(R, model):
    """One step at 1e-10 (64 lanes), twenty steps at 1e-8 (16 lanes)."""
    ctx, oc = model
    recs = _states(oc, 32, seed=71)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, R.RunConfig(lanes_per_track=64), nsteps=1)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(oc, recs[i])
        t.step()
        assert_records_close(got[i], t.record(), what=f"step {i}")
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, R.RunConfig(lanes_per_track=16), nsteps=20)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(oc, recs[i])
        t.advance(20, events=False)
        assert_records_close(got[i], t.record(), rtol=1e-8, what=f"20 steps {i}")


@pytest.mark.parametrize("lanes", [32, 16])
def test_fkbk_lane_layouts_agree_bitwise(R, model, lanes):
    ctx, oc = model
    recs = _states(oc, 16, seed=81)
    a = torch.as_tensor(recs.copy(), device="cuda")
    b = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, a, R.RunConfig(lanes_per_track=64), nsteps=5)
    R.debug_step(ctx, SPECIES3, b, R.RunConfig(lanes_per_track=lanes), nsteps=5)
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    for i in range(len(recs)):
        assert np.array_equal(gb[i].view(np.int64), ga[i].view(np.int64)), f"lanes {lanes} record {i}"


@pytest.mark.parametrize("lanes", [64, 32])
def test_fkbk_fluorite_records_and_steps_match_oracle(R, lanes):
    """U and B recoils in UO2 (cation and anion constants of Firsov's kernel per target atom)."""
    ctx = R.Context(structure=R.FLUORITE, stop_mode=R.STOP_FKBK, n_e=0.05, **UO2)
    try:
        oc = FL.ocfg(stop_mode=oracle.STOP_FKBK, n_e=0.05)
        pr = FL._prims(24, seed=91)
        got = R.track_init(ctx, FL.SPECIES, R.batch_from_numpy(pr), FL.rcfg(R, lanes_per_track=lanes)).cpu().numpy()
        recs = []
        for i in range(len(got)):
            t = oracle.Track.start(oc, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                                   pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
            FL.assert_records_close(got[i], t.record(), what=f"fluorite init {i} lanes {lanes}")
            t.advance(300 + 37 * i, events=True)
            recs.append(t.record())
        recs = np.array(recs)
        dev = torch.as_tensor(recs.copy(), device="cuda")
        R.debug_step(ctx, FL.SPECIES, dev, FL.rcfg(R, lanes_per_track=lanes), nsteps=1)
        got = dev.cpu().numpy()
        for i in range(len(recs)):
            t = oracle.Track.from_record(oc, recs[i])
            t.step()
            FL.assert_records_close(got[i], t.record(), what=f"fluorite step {i} lanes {lanes}")
    finally:
        ctx.close()


def test_fkbk_unsupported_combinations(R):
    ctx = R.Context(stop_mode=R.STOP_FKBK, n_e=N_E)
    try:
        b = R.batch_from_numpy(_prims(4, seed=3))
        with pytest.raises(R.ReedmdError, match="FP64"):
            R.track_init(ctx, SPECIES3, b, R.RunConfig(force_precision=R.FORCE_FP32))
        with pytest.raises(R.ReedmdError, match="27 cells"):
            R.run(ctx, SPECIES3, b, R.RunConfig(r_cut=5.0))
        with pytest.raises(R.ReedmdError, match="OFF, UNIFORM and LOCAL"):
            R.grad(ctx, ("B",), b, R.RunConfig(), 1.0, 1.0)
    finally:
        ctx.close()
    with pytest.raises(R.ReedmdError, match="n_e"):
        R.Context(stop_mode=R.STOP_FKBK, n_e=-1.0)


def test_fkbk_whole_run_matches_stored_oracle_run(R):
    """32,768 B at 1 keV (7 degree tilt) with the Firsov + Brandt-Kitagawa stopping, plain
    form: exact ledger; weighted KS p > 0.01, mean and std of the stopping depth within 1 %
    where three standard errors of the difference fit in 1 %, else within three."""
    meta = json.load(open(os.path.join(GOLDEN, "c0_fkbk.json")))
    zw = np.loadtxt(gzip.open(os.path.join(GOLDEN, "c0_fkbk_stopped.txt.gz"), "rt"))
    zo, wo = zw[:, 0], zw[:, 1]
    w = WORKLOADS["c0_b1kev"]
    n = meta["workload"]["n"]
    ctx = R.Context(stop_mode=R.STOP_FKBK, n_e=meta["workload"]["n_e"])
    try:
        batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
        hist, stats, log, _ = R.run(ctx, w["species"], batch, R.RunConfig(n_bins=w["n_bins"]), log_cap=n + 16)
        torch.cuda.synchronize()
        st = R.parse_stats(stats)
        _say(f"c0 fkbk gpu {st}")
        assert st["primaries"] == n and st["finished"] == n and st["error_flags"] == 0
        assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
            st["w_quarantined"] == float(n)
        lg = R.parse_log(log, st["log_count"])
        g = lg[lg["status"] == R.STOPPED]
        D, p = physref.weighted_ks(g["z_stop"], g["w"], zo, wo)
        mg = physref.family_moments(g["z_stop"], g["w"], g["lineage"])
        mo = physref.family_moments(zo, wo, np.arange(len(zo)))
        _say(f"c0 fkbk KS D={D:.4g} p={p:.3g}; mean gpu {mg[0]:.3f} oracle {mo[0]:.3f}; std {mg[1]:.3f} vs {mo[1]:.3f}")
        assert p > 0.01
        for k in (0, 1):
            rel = abs(mg[k] - mo[k]) / mo[k]
            se = math.hypot(mg[2 + k], mo[2 + k]) / mo[k]
            assert rel <= (0.01 if 3.0 * se <= 0.01 else 3.0 * se), (k, rel, se)
    finally:
        ctx.close()

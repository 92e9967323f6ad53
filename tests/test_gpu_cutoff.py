"""Interaction cut-off (a smaller interaction set than the 27 cells of Sec. 2) through the
C ABI: per-step parity with the oracle run at the same cut-off, bitwise agreement of the lane
layouts, the gate of each candidate set against the stored 27-cell oracle runs (weighted KS
p > 0.01, moments within 1 % or three standard errors of the difference), and the
interaction-set autotuner."""
import gzip
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
from tests import physref
from tests.test_gpu_parity import SPECIES3, _prims, assert_records_close
from tests.workloads import C1_THRESHOLDS, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _states(n, r_cut, seed, max_adv=2500):
    """Oracle records of tracks advanced a random number of steps at the given cut-off."""
    pr = _prims(n, seed)
    c = oracle.Config(species=SPECIES3, r_cut=r_cut)
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        t.advance(int(rng.integers(0, max_adv)), events=True)
        recs.append(t.record())
    return c, np.array(recs)


@pytest.mark.parametrize("r_cut", [3.0, 5.0])
@pytest.mark.parametrize("lanes", [64, 32, 16])
def test_cutoff_initial_domain_and_forces_match_oracle(R, ctx, lanes, r_cut):
    n = 40
    pr = _prims(n, seed=21)
    pr["pos"][2, ::3] = 29.1 + 13.0 * np.arange(len(pr["pos"][2, ::3]))
    got = R.track_init(ctx, SPECIES3, R.batch_from_numpy(pr),
                       R.RunConfig(lanes_per_track=lanes, r_cut=r_cut)).cpu().numpy()
    c = oracle.Config(species=SPECIES3, r_cut=r_cut)
    pushed = 0
    for i in range(n):
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["E0"][i]), pr["pos"][:, i],
                               pr["dir"][:, i], int(pr["key"][i]), int(pr["table"][i]), i)
        ref = t.record()
        assert_records_close(got[i], ref, what=f"init {i} lanes {lanes} r_cut {r_cut}")
        af = ref[32 + 6 * 216: 32 + 9 * 216].reshape(3, 216)
        pushed += int((np.abs(af).sum(axis=0) > 0).sum())
    # the cut-off removes most atoms from the set (about 45 of 216 within 6 A)
    assert 0 < pushed < 0.4 * 216 * n


@pytest.mark.parametrize("r_cut", [5.0, 6.0])
def test_cutoff_steps_match_oracle(R, ctx, r_cut):
    """One step at 1e-10 and twenty steps at 1e-8, tracks that have recoiled atoms."""
    c, recs = _states(32, r_cut, seed=31)
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, R.RunConfig(lanes_per_track=64, r_cut=r_cut), nsteps=1)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.step()
        assert_records_close(got[i], t.record(), what=f"step {i} r_cut {r_cut}")
    dev = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, dev, R.RunConfig(lanes_per_track=16, r_cut=r_cut), nsteps=20)
    got = dev.cpu().numpy()
    for i in range(len(recs)):
        t = oracle.Track.from_record(c, recs[i])
        t.advance(20, events=False)
        assert_records_close(got[i], t.record(), rtol=1e-8, what=f"20 steps {i} r_cut {r_cut}")


def test_cutoff_beyond_the_domain_matches_the_27_cells(R, ctx):
    """A cut-off longer than any ion-atom distance in the domain keeps every atom: the
    compacted pass then agrees with the 27-cell pass (the same terms, summed in another
    grouping when slots are empty) to 1e-11 over ten steps."""
    c, recs = _states(16, 0.0, seed=41)
    a = torch.as_tensor(recs.copy(), device="cuda")
    b = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, a, R.RunConfig(lanes_per_track=32), nsteps=10)
    R.debug_step(ctx, SPECIES3, b, R.RunConfig(lanes_per_track=32, r_cut=100.0), nsteps=10)
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    for i in range(len(recs)):
        assert_records_close(gb[i], ga[i], rtol=1e-11, what=f"r_cut 100 vs 27 cells {i}")


@pytest.mark.parametrize("lanes", [32, 16])
def test_cutoff_lane_layouts_agree_bitwise(R, ctx, lanes):
    """The compacted list is summed in the same fixed grouping for every lane layout."""
    c, recs = _states(16, 5.0, seed=51)
    a = torch.as_tensor(recs.copy(), device="cuda")
    b = torch.as_tensor(recs.copy(), device="cuda")
    R.debug_step(ctx, SPECIES3, a, R.RunConfig(lanes_per_track=64, r_cut=5.0), nsteps=5)
    R.debug_step(ctx, SPECIES3, b, R.RunConfig(lanes_per_track=lanes, r_cut=5.0), nsteps=5)
    ga, gb = a.cpu().numpy(), b.cpu().numpy()
    for i in range(len(recs)):
        assert np.array_equal(gb[i].view(np.int64), ga[i].view(np.int64)), f"lanes {lanes} record {i}"


def test_cutoff_argument_errors(R, ctx):
    pr = _prims(4, seed=3)
    b = R.batch_from_numpy(pr)
    with pytest.raises(R.ReedmdError, match="FP64"):
        R.track_init(ctx, SPECIES3, b, R.RunConfig(r_cut=5.0, force_precision=R.FORCE_FP32))
    with pytest.raises(R.ReedmdError, match="resolved by the run"):
        R.track_init(ctx, SPECIES3, b, R.RunConfig(r_cut=-1.0))
    with pytest.raises(R.ReedmdError, match="finite"):
        R.run(ctx, SPECIES3, b, R.RunConfig(r_cut=float("nan")))
    with pytest.raises(R.ReedmdError, match="27-cell"):
        R.grad(ctx, ("B",), b, R.RunConfig(r_cut=5.0), 1.0, 1.0)
    with pytest.raises(R.ReedmdError, match="n_candidates"):
        R.autotune_domain(ctx, SPECIES3, b, R.RunConfig(), candidates=())
    with pytest.raises(R.ReedmdError, match="candidates"):
        R.autotune_domain(ctx, SPECIES3, b, R.RunConfig(), candidates=(0.0, -5.0))


def _load(name):
    meta = json.load(open(os.path.join(GOLDEN, name + ".json")))
    zwl = np.loadtxt(gzip.open(os.path.join(GOLDEN, name + "_stopped.txt.gz"), "rt"))
    if zwl.shape[1] < 3:
        zwl = np.column_stack([zwl, np.arange(len(zwl))])
    return meta, zwl[:, 0], zwl[:, 1], zwl[:, 2].astype(np.int64)


def _gate(R, tag, lg, zo, wo, lo):
    """Weighted KS p > 0.01; mean and std within 1 % where three standard errors of the
    difference fit in 1 %, else within three standard errors (family-grouped)."""
    g = lg[lg["status"] == R.STOPPED]
    D, p = physref.weighted_ks(g["z_stop"], g["w"], zo, wo)
    mg = physref.family_moments(g["z_stop"], g["w"], g["lineage"])
    mo = physref.family_moments(zo, wo, lo)
    _say(f"{tag}: KS D={D:.4g} p={p:.3g}")
    assert p > 0.01, (tag, p)
    for k, name in ((0, "mean"), (1, "std")):
        rel = abs(mg[k] - mo[k]) / mo[k]
        se = math.hypot(mg[2 + k], mo[2 + k]) / mo[k]
        bound = 0.01 if 3.0 * se <= 0.01 else 3.0 * se
        _say(f"{tag}: {name} gpu {mg[k]:.3f} oracle {mo[k]:.3f} A, difference {100 * rel:.3f} % "
             f"(SE {100 * se:.3f} %, bound {100 * bound:.2f} %)")
        assert rel <= bound, (tag, name, rel, bound)


@pytest.mark.parametrize("r_cut", [5.0, 6.0])
def test_cutoff_gate_on_1kev_b_against_27_cell_oracle(R, ctx, r_cut):
    """65,536 B at 1 keV (7 degree tilt), no cloning, against the stored 27-cell oracle run."""
    meta, zo, wo, lo = _load("c0_accept")
    w = WORKLOADS["c0_b1kev"]
    n = meta["workload"]["n"]
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    hist, stats, log, _ = R.run(ctx, w["species"], batch, R.RunConfig(n_bins=w["n_bins"], r_cut=r_cut),
                                log_cap=n + 16)
    hist0, stats0, _ = R.run(ctx, w["species"], batch, R.RunConfig(n_bins=w["n_bins"]))
    torch.cuda.synchronize()
    st, st0 = R.parse_stats(stats), R.parse_stats(stats0)
    assert st["primaries"] == n and st["finished"] == n and st["error_flags"] == 0
    assert float(hist.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
        st["w_quarantined"] == float(n)
    ratio = st["pair_evals"] / st["track_steps"]
    _say(f"c0 r_cut {r_cut}: {ratio:.1f} pair terms per step (27 cells: "
         f"{st0['pair_evals'] / st0['track_steps']:.1f})")
    assert ratio < 0.5 * st0["pair_evals"] / st0["track_steps"]
    lg = R.parse_log(log, st["log_count"])
    lg = lg.copy()
    _gate(R, f"c0 r_cut {r_cut}", lg, zo, wo, np.arange(len(zo)) if lo is None else lo)


@pytest.mark.parametrize("r_cut", [5.0, 6.0])
def test_cutoff_gate_on_10kev_as_with_cloning_against_27_cell_oracle(R, ctx, r_cut):
    """8,192 As at 10 keV (half in the [110] channel cone) with 8 cloning depths, persistent
    form, against the stored 27-cell oracle run; exact ledger."""
    meta, zo, wo, lo = _load("c1_accept")
    w = WORKLOADS["c1_as10kev"]
    ids = meta["workload"]["ids"]
    n = sum(b - a for a, b in ids)
    sc = R.SamplerConfig(**w["sampler"])
    cfg = R.RunConfig(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=[list(C1_THRESHOLDS)],
                      max_steps=meta["workload"]["max_steps"], form=R.FORM_PERSISTENT, r_cut=r_cut)
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    logs = []
    for a, b in ids:
        bt = R.sample_primaries(ctx, sc, 0, b - a, id0=a)
        _, _, log, _ = R.run(ctx, w["species"], bt, cfg, hist=hist, stats=stats, id0=a, log_cap=40 * (b - a))
        logs.append(log)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    _say(f"c1 r_cut {r_cut}: {st}")
    tot = float(hist.sum().item()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
        st["w_quarantined"] + st["w_cancelled"]
    assert tot == float(n) and st["primaries"] == n and st["error_flags"] == 0
    lg = np.concatenate([R.parse_log(l, l.shape[0]) for l in logs])
    lg = lg[lg["status"] != 0]
    assert len(lg) == st["finished"]
    _gate(R, f"c1 r_cut {r_cut}", lg, zo, wo, lo)


def test_domain_autotuner_gates_times_and_records(R, ctx):
    """Pilot of 4,096 B at 1 keV: the 27 cells always pass; cut-offs of 5 and 6 A pass the
    gate and run fewer pair terms; the recorded choice is the one a run with r_cut < 0 uses
    (per-track results equal to a run with that cut-off given explicitly)."""
    w = WORKLOADS["c0_b1kev"]
    n = 8192
    batch = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
    base = dict(n_bins=w["n_bins"])
    best, rows = R.autotune_domain(ctx, w["species"], batch, R.RunConfig(**base), candidates=(0.0, 5.0, 6.0),
                                   pilot=4096)
    for r in rows:
        _say(f"candidate r_cut {r[0]}: {r[1]:.2f} ms, KS p {r[2]:.3g}, mean {100 * r[3]:.3f} %, "
             f"std {100 * r[4]:.3f} %, passed {r[5]}")
    assert rows[0][5] and rows[0][2] == 1.0
    assert all(r[1] > 0 for r in rows)
    passing = [r for r in rows if r[5]]
    assert best == min(passing, key=lambda r: r[1])[0]
    assert rows[1][5] and rows[2][5]
    logs = []
    for rc in (-1.0, best):
        _, st, log, _ = R.run(ctx, w["species"], batch, R.RunConfig(r_cut=rc, **base), log_cap=n + 16)
        torch.cuda.synchronize()
        lg = R.parse_log(log, R.parse_stats(st)["log_count"])
        logs.append(np.sort(lg, order="lineage"))
    assert np.array_equal(logs[0]["z_stop"], logs[1]["z_stop"])
    assert np.array_equal(logs[0]["steps"], logs[1]["steps"])

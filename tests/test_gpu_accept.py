"""Statistical parity of whole runs at the acceptance sizes, through the C ABI.

Stored oracle runs (tests/golden/make_golden.py c1big / c2big / c4big; oracle only):
8,192 As at 10 keV (ids 0..4095 in the [110] channel cone, 32768..36863 at 7 degree tilt),
16,384 primaries of the mixed B/P/As 1-100 keV workload, and 1,024 As at 100 keV along
[001] with 16 cloning depths to 1e-6.  The GPU runs the same primaries (same ids and
crystal keys) in the persistent form with the launch shape the autotuner picks.  Whole
trajectories are chaotic, so the comparison is statistical: weighted two-sample KS
p > 0.01 on the stopping depths, and the weighted mean and standard deviation of the
depth within 1 % where the standard error of their difference allows a 3-sigma test at
1 % (otherwise within 3 standard errors, which are printed); plus the exact weight
ledger and the clone-key derivation of every finished track.
"""
import gzip
import json
import math
import os
import sys

import numpy as np
import pytest

from tests import physref
from tests.clone_keys import check_clone_keys as _check_clone_keys
from tests.workloads import C1_THRESHOLDS, C2_THRESHOLDS, C4_THRESHOLDS, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
THR = {"c1": [list(C1_THRESHOLDS)], "c2": [list(t) for t in C2_THRESHOLDS], "c4": [list(C4_THRESHOLDS)]}


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


def _load(name):
    meta = json.load(open(os.path.join(GOLDEN, name + ".json")))
    zwl = np.loadtxt(gzip.open(os.path.join(GOLDEN, name + "_stopped.txt.gz"), "rt"))
    return meta, zwl[:, 0], zwl[:, 1], zwl[:, 2].astype(np.int64)


@pytest.mark.parametrize("golden,wname,thr", [("c1_accept", "c1_as10kev", "c1"),
                                              ("c2_accept", "c2_mixed", "c2"),
                                              ("c4_accept", "c4_as100kev", "c4")])
def test_acceptance_subset_matches_oracle(R, golden, wname, thr):
    meta, zo, wo, lo = _load(golden)
    w = WORKLOADS[wname]
    ids = meta["workload"]["ids"]
    n = sum(b - a for a, b in ids)
    ctx = R.Context()
    try:
        sc = R.SamplerConfig(**w["sampler"])
        base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=THR[thr],
                    max_steps=meta["workload"]["max_steps"], form=R.FORM_PERSISTENT)
        batches = [(R.sample_primaries(ctx, sc, 0, b - a, id0=a), a) for a, b in ids]
        lanes, waves = R.autotune(ctx, w["species"], batches[0][0], R.RunConfig(**base),
                                  pilot=int(batches[0][0]["energy"].shape[0]))
        cfg = R.RunConfig(lanes_per_track=lanes, waves_per_cu=waves, **base)
        _say(f"{golden}: {n} primaries, autotuned {lanes} lanes, {waves} waves/CU")
        hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
        stats = R.new_stats()
        logs = []
        for b, id0 in batches:
            cap = 40 * int(b["energy"].shape[0])
            _, _, log, _ = R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, log_cap=cap)
            logs.append(log)
        torch.cuda.synchronize()
        st = R.parse_stats(stats)
        lg = np.concatenate([R.parse_log(l, l.shape[0]) for l in logs])
        lg = lg[lg["status"] != 0]
        _say(f"{golden}: gpu {st}")
        tot = float(hist.sum().item()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
            st["w_quarantined"] + st["w_cancelled"]
        assert tot == float(n) and st["primaries"] == n and st["error_flags"] == 0
        assert len(lg) == st["finished"]
        fam = _check_clone_keys(lg)
        assert fam == n
        g = lg[lg["status"] == R.STOPPED]
        D, p = physref.weighted_ks(g["z_stop"], g["w"], zo, wo)
        mg = physref.family_moments(g["z_stop"], g["w"], g["lineage"])
        mo = physref.family_moments(zo, wo, lo)
        os_ = meta["stats"]
        _say(f"{golden}: KS D={D:.4g} p={p:.3g}; tracks gpu {st['finished']} oracle {os_['finished']}; "
             f"step-capped gpu {st['n_stepcap']} oracle {os_['n_stepcap']}")
        assert p > 0.01
        for k, name in ((0, "mean"), (1, "std")):
            rel = abs(mg[k] - mo[k]) / mo[k]
            se = math.hypot(mg[2 + k], mo[2 + k]) / mo[k]
            bound = 0.01 if 3.0 * se <= 0.01 else 3.0 * se
            _say(f"{golden}: {name} gpu {mg[k]:.2f} +- {mg[2 + k]:.2f} A, oracle {mo[k]:.2f} +- {mo[2 + k]:.2f} A, "
                 f"difference {100 * rel:.3f} % (SE of the difference {100 * se:.3f} %, bound {100 * bound:.2f} %)")
            assert rel <= bound, (name, rel, bound)
    finally:
        ctx.close()

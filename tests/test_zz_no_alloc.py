"""The allocation-free entry point (reedmd_run_noalloc, through the C ABI) against the
plain form of reedmd_run: two calls in a row, the second with a smaller batch, give
bitwise-equal histograms and equal totals (the results do not depend on the number of track
segments, which the allocation-free run cuts to its scratch array).  Oversized requests are
rejected with an error and the persistent form is refused."""
import sys

import numpy as np
import pytest

from tests.workloads import C1_THRESHOLDS, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _compare(R, ctx, n, id0):
    w = WORKLOADS["c1_as10kev"]
    sc = R.SamplerConfig(**w["sampler"])
    b = R.sample_primaries(ctx, sc, 0, n, id0=id0)
    ref_cfg = R.RunConfig(form=R.FORM_PLAIN, lanes_per_track=64, n_bins=w["n_bins"], thresholds=[list(C1_THRESHOLDS)])
    h_ref, s_ref, _ = R.run(ctx, w["species"], b, ref_cfg, id0=id0)
    thr = torch.tensor([list(C1_THRESHOLDS)], dtype=torch.float64, device="cuda")
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    torch.cuda.synchronize()
    cfg = R.RunConfig(form=R.FORM_PLAIN, lanes_per_track=64, n_bins=w["n_bins"])
    R.run_noalloc(ctx, w["species"], b, cfg, hist, stats, thresholds=thr, id0=id0)
    torch.cuda.synchronize()
    a, r = R.parse_stats(stats), R.parse_stats(s_ref)
    _say(f"n={n}: no-alloc {a['finished']} tracks, {a['clones']} clones; reference {r['finished']}, {r['clones']}")
    assert np.array_equal(hist.cpu().numpy(), h_ref.cpu().numpy())
    for k in ("primaries", "finished", "clones", "track_steps", "pair_evals", "n_stopped", "n_backscattered",
              "n_stepcap", "w_stopped", "w_backscattered", "w_overflow", "w_underflow", "error_flags"):
        assert a[k] == r[k], (n, k, a[k], r[k])
    # sums of weight x depth are floating-point atomics in whatever order the tracks finish
    for k in ("sum_wz", "sum_wz2"):
        assert abs(a[k] - r[k]) <= 1e-12 * abs(r[k]), (n, k, a[k], r[k])
    assert a["primaries"] == n


def test_noalloc_run_equals_plain_run_twice(R):
    ctx = R.Context()
    try:
        # 1,024 As primaries with 8 cloning depths: 1,024 segments of clone stacks would need
        # 146 MiB, so the allocation-free run cuts them to what fits its 128 MiB array
        _compare(R, ctx, 1024, 0)
        # a second call on the same array, smaller, from the tilted half of the workload
        _compare(R, ctx, 300, 40000)
    finally:
        ctx.close()


def test_noalloc_rejects_what_it_cannot_do(R):
    ctx = R.Context()
    try:
        w = WORKLOADS["c1_as10kev"]
        b = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, 16)
        hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
        stats = R.new_stats()
        with pytest.raises(R.ReedmdError):
            R.run_noalloc(ctx, w["species"], b, R.RunConfig(form=R.FORM_PERSISTENT, n_bins=w["n_bins"]), hist, stats)
        # a batch whose claim order alone (4 bytes per primary) exceeds the 128 MiB array is
        # refused before anything is launched (the batch arrays are never read)
        big = R.empty_batch(34_000_000)
        with pytest.raises(R.ReedmdError):
            R.run_noalloc(ctx, w["species"], big, R.RunConfig(form=R.FORM_PLAIN, n_bins=w["n_bins"]), hist, stats)
        del big
        torch.cuda.synchronize()
        assert R.parse_stats(stats)["primaries"] == 0
    finally:
        ctx.close()

"""Parity at the benchmark's full size and launch configuration (65,536 As primaries at 10 keV,
8 cloning depths, persistent form, 16 lanes per track, the occupancy-sized grid): sampled
starting records and single steps against the oracle one by one (1e-10), and for the whole run
the properties that hold at any size: exact weight ledger, every finished track's weight is
exactly 2^-k for its k crossed depths, the histogram equals the binned track log bit for bit,
finished = primaries + clones, and the moment sums match the log.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.workloads import C1_THRESHOLDS, WORKLOADS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = WORKLOADS["c1_as10kev"]
N = W["n"]


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


def _sampler():
    return dict(W["sampler"], n_cone=N // 2)


def _close(a, b, rtol):
    scale = np.maximum(np.abs(b), 1e-9 * max(np.abs(b).max(), 1e-300))
    return float((np.abs(a - b) / scale).max()) <= rtol


def test_full_size_sampled_records_and_steps_match_oracle(R, ctx):
    batch = R.sample_primaries(ctx, R.SamplerConfig(**_sampler()), 0, N)
    cfg = R.RunConfig(lanes_per_track=16)
    rec = R.track_init(ctx, W["species"], batch, cfg)
    init = rec.cpu().numpy()
    R.debug_step(ctx, W["species"], rec, cfg, nsteps=1)
    torch.cuda.synchronize()
    stepped = rec.cpu().numpy()
    pr = {k: v.cpu().numpy() for k, v in batch.items()}
    c = oracle.Config(species=W["species"])
    idx = np.unique(np.concatenate([np.linspace(0, N - 1, 48).astype(int), [N // 2 - 1, N // 2, N - 1]]))
    for i in idx:
        t = oracle.Track.start(c, int(pr["species"][i]), float(pr["energy"][i]), pr["pos"][:, i], pr["dir"][:, i],
                               int(pr["key"][i].astype(np.uint64)), int(pr["table"][i]), int(i))
        r0 = t.record()
        t.step()
        r1 = t.record()
        for got, ref, what in ((init[i], r0, "init"), (stepped[i], r1, "step")):
            assert np.array_equal(got.view(np.int64)[12:22], ref.view(np.int64)[12:22]), (what, i)
            ex = oracle.slot_exists(ref.view(np.int64)[12:15])
            assert _close(got[0:6], ref[0:6], 1e-10), (what, i)
            A = got[32:].reshape(9, 216)[:, ex]
            B = ref[32:].reshape(9, 216)[:, ex]
            assert _close(A[0:6].ravel(), B[0:6].ravel(), 1e-10), (what, i, "atoms")
            fs = max(np.abs(B[6:9]).max(), np.abs(ref[6:9]).max())
            assert np.abs(got[6:9] - ref[6:9]).max() <= 1e-10 * fs, (what, i, "F")
    _say(f"full size: {len(idx)} sampled records and steps of {N} match the oracle")


def test_full_size_run_invariants_in_the_bench_configuration(R, ctx):
    batch = R.sample_primaries(ctx, R.SamplerConfig(**_sampler()), 0, N)
    cfg = R.RunConfig(form=R.FORM_PERSISTENT, lanes_per_track=16, thresholds=[list(C1_THRESHOLDS)],
                      n_bins=W["n_bins"], bin_width=W["bin_width"])
    shape = R.launch_shape(ctx, batch, cfg)
    assert shape["lanes"] == 16 and shape["blocks"] >= 256
    cap = 40 * N
    hist, stats, log, _ = R.run(ctx, W["species"], batch, cfg, log_cap=cap)
    torch.cuda.synchronize()
    st = R.parse_stats(stats)
    _say(f"full size run {shape}: {st}")
    assert st["primaries"] == N and st["error_flags"] == 0 and st["log_count"] <= cap
    assert st["finished"] == N + st["clones"]
    lg = R.parse_log(log, st["log_count"])
    assert len(lg) == st["finished"]
    # every primary's family is present and weights are exact powers of two
    assert np.array_equal(np.unique(lg["lineage"]), np.arange(N))
    assert np.array_equal(lg["w"], np.ldexp(1.0, -lg["next_k"].astype(np.int64)))
    # exact ledger
    tot = float(hist.sum()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + st["w_quarantined"]
    assert tot == float(N)
    wsum = np.zeros(N)
    np.add.at(wsum, lg["lineage"], lg["w"])
    assert np.all(wsum == 1.0)
    # the histogram is the binned log, bit for bit (sums of powers of two)
    s = lg[lg["status"] == R.STOPPED]
    fb = np.floor(s["z_stop"] / W["bin_width"])
    inb = (fb >= 0) & (fb < W["n_bins"])
    ref = np.zeros(W["n_bins"])
    np.add.at(ref, fb[inb].astype(np.int64), s["w"][inb])
    assert np.array_equal(hist.cpu().numpy(), ref)
    assert st["w_overflow"] == float(s["w"][fb >= W["n_bins"]].sum())
    m1 = float((s["w"] * s["z_stop"]).sum())
    assert abs(st["sum_wz"] - m1) <= 1e-9 * abs(m1)
    # crossed depths: a track that stops beyond depth j was beyond it at the end of an earlier
    # step (a step moves it far less than the spacing of the depths) unless j was passed in
    # its last step, where the stop is booked before any cloning
    thr = np.array(C1_THRESHOLDS)
    k_below = np.searchsorted(thr, s["z_stop"], side="right")
    assert np.all(s["next_k"] >= k_below - 1)
    assert np.all(s["next_k"] <= len(thr))
    _say(f"full size: {st['finished']} tracks, {st['clones']} clones, exact ledger and histogram")

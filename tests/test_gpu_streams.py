"""The binding on a caller's stream that is not the current one: every output (batch arrays,
histogram, statistics) is allocated and cleared on the stream the work is launched on, so a
run there equals the same run on the current stream bit for bit, even while the current
stream is still busy with earlier work."""
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


@pytest.fixture(scope="module")
def ctx(R):
    c = R.Context()
    yield c
    c.close()


def test_side_stream_run_equals_current_stream_run(R, ctx):
    w = WORKLOADS["c1_as10kev"]
    n = 1024
    sc = R.SamplerConfig(**dict(w["sampler"], n_cone=n // 2))
    cfg = R.RunConfig(form=R.FORM_PERSISTENT, thresholds=[list(C1_THRESHOLDS)], n_bins=w["n_bins"],
                      bin_width=w["bin_width"])
    _say("current stream")
    b0 = R.sample_primaries(ctx, sc, 0, n)
    h0, s0, _ = R.run(ctx, w["species"], b0, cfg)
    torch.cuda.synchronize()
    _say("side stream, current stream busy")
    side = torch.cuda.Stream()
    busy = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    for _ in range(8):
        busy.fill_(1.0)          # queued on the current stream ahead of anything ordered there
    b1 = R.sample_primaries(ctx, sc, 0, n, stream=side)
    h1, s1, _ = R.run(ctx, w["species"], b1, cfg, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    for k in b0:
        assert torch.equal(b0[k], b1[k]), k
    st0, st1 = R.parse_stats(s0), R.parse_stats(s1)
    _say(f"stats {st1}")
    assert st1["primaries"] == n and st1["error_flags"] == 0
    assert torch.equal(h0, h1)
    for k in ("finished", "clones", "track_steps", "pair_evals", "n_stopped", "n_backscattered",
              "w_underflow", "w_overflow", "w_backscattered", "w_quarantined"):
        assert st0[k] == st1[k], k
    assert float(h1.sum()) + st1["w_underflow"] + st1["w_overflow"] + st1["w_backscattered"] == float(n)
    del busy

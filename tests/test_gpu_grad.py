"""GPU adjoint gradient of the mean projected range vs the oracle's forward-mode
derivative and central finite differences (through the C ABI)."""
import math
import sys

import numpy as np
import pytest

import oracle

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


def _batch(n, species_idx, E, seed, tilt=math.radians(7.0)):
    return oracle.sample_primaries(oracle.SamplerCfg(choice=(species_idx,), E_min=E, E_max=E, tilt=tilt), seed, n)


def test_adjoint_matches_oracle_forward_mode(R, ctx):
    """Per track, on short tracks (hundreds to a few thousand steps, so several 64-step
    segments): the reverse-mode derivative equals the oracle's forward-mode derivative of
    the same discrete map.  Both are pathwise derivatives of chaotic trajectories computed on
    slightly differently rounded paths, so tracks are compared where the two stopping depths
    agree to 1e-9 (the paths have not separated), at 1e-6 relative."""
    species = ("B", "P", "As")
    pr = _batch(48, 0, 300.0, 21)
    b = R.batch_from_numpy(pr)
    cfg = R.RunConfig(max_steps=20000)
    g = R.grad(ctx, species, b, cfg, 1.0, 1.0, per_track=True)
    tr = g["tracks"].cpu().numpy()
    oc = oracle.Config(species=species)
    checked = 0
    for i in range(len(tr)):
        st, z, dk, ds, n = oracle.grad_track(oc, 0, pr["E0"][i], pr["pos"][:, i], pr["dir"][:, i],
                                             int(pr["key"][i]), max_steps=20000)
        assert int(tr[i, 3]) == st
        if st != oracle.STOPPED:
            continue
        if abs(tr[i, 0] - z) > 1e-9 * abs(z):
            continue
        checked += 1
        assert int(tr[i, 4]) == n
        for gv, ov, name in ((tr[i, 1], dk, "dk"), (tr[i, 2], ds, "ds")):
            assert abs(gv - ov) <= 1e-6 * max(abs(ov), 1e-3 * abs(z)), (i, name, gv, ov, n)
    _say(f"compared {checked} tracks")
    assert checked >= 24


def test_adjoint_short_tracks_under_a_small_step_cap(R, ctx):
    """40 eV B (99-300 steps) under max_steps = 200: a few 64-step segments, a last segment
    of any length, small checkpoint and drop-log capacities, and tracks ending as capped or
    backscattered.  Status and step count equal the oracle's for every track; stopped tracks
    have the oracle's forward-mode derivatives (1e-6), capped ones are excluded from the mean."""
    species = ("B",)
    pr = _batch(64, 0, 40.0, 9)
    b = R.batch_from_numpy(pr)
    cfg = R.RunConfig(max_steps=200)
    g = R.grad(ctx, species, b, cfg, 1.0, 1.0, per_track=True)
    tr = g["tracks"].cpu().numpy()
    oc = oracle.Config(species=species)
    seen = {oracle.STOPPED: 0, oracle.STEPCAP: 0}
    checked = 0
    for i in range(len(tr)):
        st, z, dk, ds, n = oracle.grad_track(oc, 0, pr["E0"][i], pr["pos"][:, i], pr["dir"][:, i],
                                             int(pr["key"][i]), max_steps=200)
        assert int(tr[i, 3]) == st, i
        assert int(tr[i, 4]) == n, i
        if st in seen:
            seen[st] += 1
        if st != oracle.STOPPED:
            assert tr[i, 1] == 0.0 and tr[i, 2] == 0.0
            continue
        if abs(tr[i, 0] - z) > 1e-9 * abs(z):
            continue
        checked += 1
        for gv, ov, name in ((tr[i, 1], dk, "dk"), (tr[i, 2], ds, "ds")):
            assert abs(gv - ov) <= 1e-6 * max(abs(ov), 1e-3 * abs(z)), (i, name, gv, ov, n)
    _say(f"stopped {seen[oracle.STOPPED]}, capped {seen[oracle.STEPCAP]}, compared {checked}")
    assert seen[oracle.STOPPED] >= 8 and seen[oracle.STEPCAP] >= 8 and checked >= 8
    assert g["count"] == seen[oracle.STOPPED]


def test_adjoint_matches_oracle_forward_mode_on_5kev_p(R, ctx):
    """The adjoint workload's species and energy (P at 5 keV, 7 degree tilt), with the tracks
    ended early by a raised stopping energy (3 keV, a few hundred steps: several 64-step
    segments, domain moves and hard collisions): per track the reverse-mode derivatives equal
    the oracle's forward-mode ones to 1e-6 where the two paths have not separated (stopping
    depths equal to 1e-9)."""
    species = ("P",)
    pr = _batch(64, 0, 5000.0, 0)
    b = R.batch_from_numpy(pr)
    cfg = R.RunConfig(max_steps=20000, E_stop=3000.0)
    g = R.grad(ctx, species, b, cfg, 1.0, 1.0, per_track=True)
    tr = g["tracks"].cpu().numpy()
    oc = oracle.Config(species=species, E_stop=3000.0)
    checked, steps = 0, []
    for i in range(len(tr)):
        st, z, dk, ds, n = oracle.grad_track(oc, 0, pr["E0"][i], pr["pos"][:, i], pr["dir"][:, i],
                                             int(pr["key"][i]), max_steps=20000)
        assert int(tr[i, 3]) == st
        if st != oracle.STOPPED or abs(tr[i, 0] - z) > 1e-9 * abs(z):
            continue
        checked += 1
        steps.append(n)
        assert int(tr[i, 4]) == n
        for gv, ov, name in ((tr[i, 1], dk, "dk"), (tr[i, 2], ds, "ds")):
            assert abs(gv - ov) <= 1e-6 * max(abs(ov), 1e-3 * abs(z)), (i, name, gv, ov, n)
    _say(f"5 keV P to 3 keV: compared {checked} of {len(tr)} tracks, {min(steps)}-{max(steps)} steps")
    assert checked >= 32


def _per_track_fd(R, ctx, species, b, cfg, which, h, k=1.0, s=1.0):
    """Central difference of every track's stopping depth on the same seeded crystal, and the
    tracks that stop in both runs."""
    up, dn = dict(k=k, s=s), dict(k=k, s=s)
    up[which] += h
    dn[which] -= h
    zu = R.grad(ctx, species, b, cfg, up["k"], up["s"], per_track=True)["tracks"].cpu().numpy()
    zd = R.grad(ctx, species, b, cfg, dn["k"], dn["s"], per_track=True)["tracks"].cpu().numpy()
    ok = (zu[:, 3] == R.STOPPED) & (zd[:, 3] == R.STOPPED)
    return (zu[:, 0] - zd[:, 0]) / (2 * h), ok


def _fd_check(R, ctx, species, pr, cfg, min_linear, h1=1e-7, h2=1e-8, lin_tol=1e-4):
    """Per-track pathwise derivatives against central differences.  A track counts as linear
    when its central differences at h1 and h2 agree to lin_tol (relative); on linear tracks
    the adjoint must agree with the h1 difference to 1e-3 per track and to 1e-4 on their mean,
    and at least min_linear[k or s] tracks must be linear.  The h = 1e-4 difference is
    reported beside it, with the all-track mean of the adjoint and its standard error."""
    b = R.batch_from_numpy(pr)
    g = R.grad(ctx, species, b, cfg, 1.0, 1.0, per_track=True)
    tr = g["tracks"].cpu().numpy()
    stopped = tr[:, 3] == R.STOPPED
    report = {}
    for col, which in ((1, "k"), (2, "s")):
        f1, ok1 = _per_track_fd(R, ctx, species, b, cfg, which, h1)
        f2, ok2 = _per_track_fd(R, ctx, species, b, cfg, which, h2)
        f4, ok4 = _per_track_fd(R, ctx, species, b, cfg, which, 1e-4)
        ok = stopped & ok1 & ok2
        lin = ok & (np.abs(f1 - f2) <= lin_tol * np.maximum(np.maximum(np.abs(f1), np.abs(f2)), 1e-3))
        adj = tr[:, col]
        allm = adj[stopped].mean()
        alls = adj[stopped].std(ddof=1) / math.sqrt(max(stopped.sum(), 2))
        msg = (f"d/d{which}: {lin.sum()} of {ok.sum()} stopped tracks linear at h = {h1:g} / {h2:g}; "
               f"all-track adjoint mean {allm:.6g} +- {alls:.3g}")
        report[which] = dict(linear=int(lin.sum()), stopped=int(ok.sum()))
        if lin.any():
            rel = np.abs(adj[lin] - f1[lin]) / np.maximum(np.abs(f1[lin]), 1e-3)
            # per-track derivatives have both signs: the mean is compared on the scale of the
            # mean magnitude
            mean_rel = abs(adj[lin].mean() - f1[lin].mean()) / max(np.abs(f1[lin]).mean(), 1e-3)
            l4 = lin & ok4
            rel4 = np.abs(adj[l4] - f4[l4]) / np.maximum(np.abs(f4[l4]), 1e-3)
            msg += (f"; on linear tracks per-track worst {rel.max():.3g}, mean adjoint {adj[lin].mean():.8g} vs "
                    f"FD {f1[lin].mean():.8g} (relative {mean_rel:.3g}); at h = 1e-4 {int((rel4 <= 1e-4).sum())} "
                    f"of them agree to 1e-4 (median {np.median(rel4):.3g})")
            report[which].update(worst=float(rel.max()), mean_rel=float(mean_rel))
        _say(msg)
        assert lin.sum() >= min_linear[which], (which, int(lin.sum()))
        if lin.any():
            assert (rel <= 1e-3).all(), (which, rel.max())
            assert mean_rel <= 1e-4, (which, mean_rel)
    return report


def test_adjoint_matches_central_differences_on_linear_tracks(R, ctx):
    """Pathwise derivatives of chaotic tracks match finite differences where a track is in its
    linear regime.  Tracks are classified by central differences at h = 1e-7 and 1e-8 on the
    same seeded crystal (agreement to 1e-4); on linear tracks the adjoint agrees with the
    h = 1e-7 difference to 1e-3 per track and to 1e-4 on the mean.  Short 300 eV B tracks, and
    the adjoint workload itself (P at 5 keV, ~2,500-3,500 steps with many hard collisions),
    each with a required minimum of linear tracks for both derivatives."""
    _fd_check(R, ctx, ("B",), _batch(128, 0, 300.0, 5), R.RunConfig(max_steps=16384), dict(k=32, s=8))
    _fd_check(R, ctx, ("P",), _batch(256, 0, 5000.0, 0), R.RunConfig(max_steps=16384), dict(k=1, s=1))


def test_autograd_function_returns_the_adjoint(R, ctx):
    species = ("P",)
    pr = _batch(32, 0, 5000.0, 3)
    b = R.batch_from_numpy(pr)
    cfg = R.RunConfig(max_steps=16384)
    k = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    rng = R.ReedMDRange.apply(k, s, ctx, species, b, cfg)
    (3.0 * rng).backward()
    ref = R.grad(ctx, species, b, cfg, 1.0, 1.0)
    assert float(rng.detach()) == ref["mean"]
    assert float(k.grad) == 3.0 * ref["dk"] and float(s.grad) == 3.0 * ref["ds"]
    assert ref["count"] > 0


def test_grad_rejects_cloning(R, ctx):
    b = R.batch_from_numpy(_batch(4, 0, 1000.0, 1))
    with pytest.raises(R.ReedmdError):
        R.grad(ctx, ("B",), b, R.RunConfig(thresholds=[[20.0]]), 1.0, 1.0)

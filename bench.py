"""Throughput benchmark of the REED-MD hot path on one MI355X.

Headline workload: the uneven batch, 1,048,576 primaries with species uniform over B, P and
As and energies log-uniform in 1-100 keV into diamond Si at 7 degree tilt, 6 cloning-depth
tables (species x energy decade) of 12 depths each, run by the persistent kernel with its
device work queue, kept as a HIP graph, in the launch shape the autotuner picks.  One step =
sample the next 1/K of the primaries on the device (K = --steps) and run each of them with
all of its clones to termination (domain following, ZBL forces, local stopping, adaptive
velocity Verlet, cloning, weighted histogram); the K timed steps together run the whole
workload, warm-up steps use primaries from a disjoint id range.  Prints one JSON line:
ion-atom force evaluations per second (value), tracks per second, the FP64 VALU roofline
fraction of the track kernel, the FP64 CPU oracle on a bounded sample of the same workload,
and beside them the 10 keV As workload with its profile accuracy, the FP32 pair-term
variant, the 85 keV U recoils in fluorite UO2 and the adjoint gradient.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP64 operations per ion-atom pair evaluation (exp, sqrt and division counted
# as one each): separation 3, r^2 5, sqrt 1, 1/r 1, r/a 1, four exponents and their
# arguments 8, phi 7, phi' 7, V'(r) 5, coefficient 1, pair force 3, ion force sum 3,
# density weight 3 and sum 1, atom half kicks 12, atom drift 6.
FLOP_PER_PAIR = 67
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 128 FP64 FLOP/clk/CU
FP32_VECTOR_PEAK_TFLOPS = 157.3  # 256 CU x 2.4 GHz x 256 FP32 FLOP/clk/CU
# With the FP32 pair term, 38 of the 67 move to FP32 (r^2 5, sqrt 1, 1/r 1, r/a 1, the
# exponents 8, phi 7, phi' 7, V'(r) 5, coefficient 1, density-weight exponent 2); the
# separation, force components and sums, density sum, kicks and drifts (29) stay FP64.
FLOP_PER_PAIR_F32_PART = 38

# HBM bytes per step (the step's main and tail launches of the track kernel) measured with
# rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (separate runs, mean of the 20 timed steps),
# scaled by the same counters on a 1 GiB copy (FETCH x 2.000, WRITE x 1.000); reported only
# while the track kernel's device sources (track_kernels.hpp, device_physics.hpp) and the
# launch match the ones the counters were taken on.
MEASURED_TRAFFIC = {
    "sources_sha256_prefix": "6a011c2e0fe498bd",
    "workload": "c2", "form": "persistent", "lanes": 32, "blocks": 256, "primaries": 1048576, "slice": 52429,
    "fetch_bytes": 1746539.2 * 1024 * 2.000,
    "write_bytes": 3711666.3 * 1024 * 1.000,
}


def kernel_sources_hash():
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_0810_4737_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.path.join(here, x) for x in ("device_physics.hpp", "track_kernels.hpp")):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["c1", "c2", "c4"], default="c2",
                    help="c2: mixed B/P/As 1-100 keV, 1,048,576 primaries (default, the benchmark line); "
                         "c1: 10 keV As, 65,536 primaries; c4: 100 keV As [001] channeling, 262,144 primaries")
    ap.add_argument("--n", type=int, default=0, help="primaries of the workload (default: its full size)")
    ap.add_argument("--whole", action="store_true",
                    help="every step runs the whole workload (default for c1) instead of the next 1/steps of it")
    ap.add_argument("--form", choices=["auto", "plain", "persistent"], default="persistent")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--waves", type=int, default=0, help="resident waves per CU with --lanes (0: by occupancy)")
    ap.add_argument("--queue", type=int, default=0, help="clone-queue capacity in records (0: library default)")
    ap.add_argument("--refine-epochs", type=int, default=8,
                    help="also time the 10 keV As workload with the cloning depths re-placed over this many "
                         "epochs (targets 2^-k, first table the stored depths), once with one launch per "
                         "epoch and once with every epoch inside one persistent launch; reported apart "
                         "(0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-c1", action="store_true", help="skip the 10 keV As leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient / forward time ratio")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 pair-term variant leg")
    ap.add_argument("--no-uo2", action="store_true", help="skip the 85 keV U recoil in UO2 leg")
    ap.add_argument("--no-domain", action="store_true", help="skip the interaction-set (cut-off) autotuner leg")
    ap.add_argument("--no-c4", action="store_true", help="skip the 100 keV As deep-tail accuracy leg")
    ap.add_argument("--no-fkbk", action="store_true", help="skip the Firsov + Brandt-Kitagawa stopping leg")
    ap.add_argument("--uo2-n", type=int, default=0, help="primaries of the UO2 leg (default: the workload's 5,120)")
    ap.add_argument("--grid-share", choices=["half", "full"], default="half",
                    help="with several streams and no --waves: each step's persistent grid takes half of the "
                         "resident workgroups (half) or all of them (full)")
    ap.add_argument("--streams", type=int, default=3,
                    help="sliced workloads: steps go round-robin to this many streams, each with its own "
                         "context, with no host synchronisation between them (1: one stream, one step at a time)")
    ap.add_argument("--pipelined", type=int, default=0,
                    help="also time this many 10 keV As batches back to back on two streams and contexts")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    return ap.parse_args()


WORKLOAD_NAMES = {"c1": "c1_as10kev", "c2": "c2_mixed", "c4": "c4_as100kev"}


def workload_setup(R, key, n):
    """(workload dict, sampler, depth tables, tail depth) of a benchmark workload."""
    from tests.workloads import C1_THRESHOLDS, C2_THRESHOLDS, C4_THRESHOLDS, WORKLOADS
    w = WORKLOADS[WORKLOAD_NAMES[key]]
    if key == "c1":
        return w, R.SamplerConfig(**dict(w["sampler"], n_cone=n // 2)), [list(C1_THRESHOLDS)], C1_THRESHOLDS[6]
    if key == "c2":
        return w, R.SamplerConfig(**w["sampler"]), [list(t) for t in C2_THRESHOLDS], 2000.0
    return w, R.SamplerConfig(**w["sampler"]), [list(C4_THRESHOLDS)], 4000.0


def cpu_baseline(key, target_seconds):
    """The FP64 oracle on the host cores, on the first primaries of the same workload (for the
    10 keV As workload the first ids of both halves), run in chunks of one primary per core
    until the time box is used."""
    import numpy as np

    import oracle
    from tests.workloads import C1_THRESHOLDS, C2_THRESHOLDS, C4_THRESHOLDS, WORKLOADS
    w = WORKLOADS[WORKLOAD_NAMES[key]]
    thr = {"c1": [list(C1_THRESHOLDS)], "c2": [list(t) for t in C2_THRESHOLDS], "c4": [list(C4_THRESHOLDS)]}[key]
    sc = oracle.SamplerCfg(**w["sampler"])
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=thr,
                        max_steps=2_000_000)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    total_pairs, total_tracks, total_prim, t_all = 0, 0, 0, 0.0
    offset = 0
    half = w["n"] // 2
    while t_all < target_seconds and offset < 4096:
        if key == "c1":
            k = max(1, cores // 2)
            a = oracle.sample_primaries(sc, 0, k, id0=offset)
            b = oracle.sample_primaries(sc, 0, k, id0=half + offset)
            prim = {q: np.concatenate([a[q], b[q]], axis=-1) for q in a}
            lin = np.concatenate([offset + np.arange(k), half + offset + np.arange(k)]).astype(np.int64)
        else:
            k = cores
            prim = oracle.sample_primaries(sc, 0, k, id0=offset)
            lin = (offset + np.arange(k)).astype(np.int64)
        t0 = time.perf_counter()
        r = oracle.run(cfg, prim, nthreads=cores, lineage=lin)
        t_all += time.perf_counter() - t0
        total_pairs += r["stats"]["pair_evals"]
        total_tracks += r["stats"]["finished"]
        total_prim += len(lin)
        offset += k
        progress(f"oracle chunk of {len(lin)} primaries: {r['stats']['pair_evals']} pairs, {t_all:.1f} s so far")
    ids = (f"ids 0..{offset - 1} and {half}..{half + offset - 1}" if key == "c1" else f"ids 0..{offset - 1}")
    return dict(value=total_pairs / t_all, unit="force evals/s", cores=cores, kind="oracle",
                sample=f"{total_prim} primaries of the same workload ({ids}, all clones), {t_all:.1f} s wall, "
                       f"{total_tracks / t_all:.1f} tracks/s")


def profile_accuracy(R, torch, np, ctx, w, sampler, n, cfg, reed_log, t_reed, tail_depth):
    """Accuracy per unit time of the deep tail, REED against no splitting.  The same primaries
    run once without cloning; the depth D where their survival is 1e-3 (the 0.1 % deepest
    stop) is the probe.  For both runs the probability of stopping beyond D (and beyond the
    7th cloning depth) is estimated with its relative standard error from 32 independent
    sub-batches (primary id mod 32, batch means), and the figure of merit 1 / (T s^2) uses the
    launch's wall time T.  REED's estimate is the weighted sum over every track of the family."""
    import dataclasses
    ns_cfg = dataclasses.replace(cfg, thresholds=None)
    b = R.sample_primaries(ctx, sampler, 0, n)
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, log, _ = R.run(ctx, w["species"], b, ns_cfg, hist=hist, stats=stats, log_cap=n + 16)
    torch.cuda.synchronize()
    t_ns = time.perf_counter() - t0
    st = R.parse_stats(stats)
    ns_log = R.parse_log(log, st["log_count"])
    zs = np.sort(ns_log["z_stop"][ns_log["status"] == R.STOPPED])
    D = float(zs[min(len(zs) - 1, int(round(len(zs) * (1.0 - 1e-3))))]) if len(zs) else tail_depth

    def estimate(lg, depth):
        deep = (lg["status"] == R.STOPPED) & (lg["z_stop"] >= depth)
        per = np.zeros(n)
        np.add.at(per, lg["lineage"][deep], lg["w"][deep])
        bm = np.array([per[k::32].mean() for k in range(32)])
        p = per.mean()
        rel = bm.std(ddof=1) / math.sqrt(32) / p if p > 0 else float("nan")
        return p, rel

    out = {}
    for name, depth in (("survival_1e-3", D), ("depth_7", tail_depth)):
        pr, rr = estimate(reed_log, depth)
        pn, rn = estimate(ns_log, depth)
        fr = 1.0 / (t_reed * rr * rr) if rr > 0 else None
        fn = 1.0 / (t_ns * rn * rn) if rn > 0 else None
        out[name] = dict(depth_A=depth, reed_probability=pr, reed_rel_err=rr, reed_fom_per_s=fr,
                         nosplit_probability=pn, nosplit_rel_err=rn, nosplit_fom_per_s=fn,
                         fom_ratio=(fr / fn) if (fr and fn) else None)
    out["reed_s"] = t_reed
    out["nosplit_s"] = t_ns
    out["method"] = "32 sub-batches (primary id mod 32), batch means; FOM = 1/(T s^2) with the launch wall time"
    return out


def c4_leg(R, torch, np, n=262144):
    """The deep-tail workload: 262,144 As at 100 keV exactly along [001] with 16 cloning depths
    down to 1e-6, persistent form, autotuned; one REED run and one run of the same primaries
    without cloning, both with every finished track logged.  Probes: the depths where REED's
    weighted survival is 1e-4 and 1e-5; at each, the probability of stopping beyond it with its
    relative standard error from 32 sub-batches (primary id mod 32) and the figure of merit
    1 / (T s^2) of both runs (T the run's wall time)."""
    ctx = R.Context()
    w, sampler, thr, _ = workload_setup(R, "c4", n)
    base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], form=R.FORM_PERSISTENT)
    batch = R.sample_primaries(ctx, sampler, 0, n)
    lanes, waves = R.autotune(ctx, w["species"], batch, R.RunConfig(thresholds=thr, **base), pilot=min(n, 65536))
    runs = {}
    for name, t in (("reed", thr), ("nosplit", None)):
        cfg = R.RunConfig(thresholds=t, lanes_per_track=lanes, waves_per_cu=waves, **base)
        cap = 8 * n if t is not None else n + 16
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, log, _ = R.run(ctx, w["species"], batch, cfg, log_cap=cap)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = R.parse_stats(st)
        assert s["log_count"] <= cap, ("track log too small", s["log_count"], cap)
        lg = R.parse_log(log, s["log_count"])
        runs[name] = (lg, dt, s)
        progress(f"c4 {name}: {dt:.1f} s, {s['finished']} tracks, {s['pair_evals'] / dt:.4g} force evals/s")
    reed = runs["reed"][0]
    st_ = reed[reed["status"] == R.STOPPED]
    order = np.argsort(st_["z_stop"])[::-1]
    surv = np.cumsum(st_["w"][order]) / n          # weighted survival beyond each stopping depth

    def probe(p):
        k = int(np.searchsorted(surv, p))
        return float(st_["z_stop"][order][min(k, len(order) - 1)])

    def estimate(lg, depth):
        deep = (lg["status"] == R.STOPPED) & (lg["z_stop"] >= depth)
        per = np.zeros(n)
        np.add.at(per, lg["lineage"][deep], lg["w"][deep])
        bm = np.array([per[k::32].mean() for k in range(32)])
        pr = per.mean()
        rel = bm.std(ddof=1) / math.sqrt(32) / pr if pr > 0 else float("nan")
        return pr, rel, int(deep.sum())

    out = dict(workload="262,144 As at 100 keV along [001] into Si; 16 cloning depths to 1e-6; 5 A bins",
               primaries=n, lanes_per_track=lanes, reed_s=runs["reed"][1], nosplit_s=runs["nosplit"][1],
               reed_tracks=runs["reed"][2]["finished"], reed_force_evals_per_s=runs["reed"][2]["pair_evals"] / runs["reed"][1],
               nosplit_force_evals_per_s=runs["nosplit"][2]["pair_evals"] / runs["nosplit"][1],
               method="32 sub-batches (primary id mod 32), batch means; FOM = 1/(T s^2) with the run's wall time; "
                      "probe depths where REED's weighted survival is 1e-4 and 1e-5")
    for name, p in (("survival_1e-4", 1e-4), ("survival_1e-5", 1e-5)):
        D = probe(p)
        pr, rr, nr = estimate(reed, D)
        pn, rn, nn = estimate(runs["nosplit"][0], D)
        fr = 1.0 / (runs["reed"][1] * rr * rr) if rr > 0 else None
        fn = 1.0 / (runs["nosplit"][1] * rn * rn) if (rn > 0 and rn == rn) else None
        out[name] = dict(depth_A=D, reed_probability=pr, reed_rel_err=rr, reed_tracks_beyond=nr, reed_fom_per_s=fr,
                         nosplit_probability=pn, nosplit_rel_err=rn, nosplit_tracks_beyond=nn, nosplit_fom_per_s=fn,
                         fom_ratio=(fr / fn) if (fr and fn) else None)
    ctx.close()
    return out


def pipelined_leg(R, torch, w, sampler, n, cfg, k_steps, species):
    """Batches back to back on two streams, each with its own context (clone queue, stacks,
    graphs), histogram and statistics, with no host synchronisation between them: the next
    batch's workgroups start on the compute units that the previous batch's tail leaves
    idle.  The ledger of each context's accumulated batches is checked afterwards."""
    ctxs = [R.Context(), R.Context()]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    hists = [torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda") for _ in range(2)]
    stats = [R.new_stats() for _ in range(2)]
    # one warm batch per context allocates its scratch and builds its graph; every batch is
    # allocated (zero-filled), sampled and run with its own stream current, so the three are
    # ordered on that stream
    for j in range(2):
        with torch.cuda.stream(streams[j]):
            b = R.sample_primaries(ctxs[j], sampler, 0, n, stream=streams[j])
            R.run(ctxs[j], species, b, cfg, hist=hists[j], stats=stats[j], stream=streams[j])
    torch.cuda.synchronize()
    for j in range(2):
        hists[j].zero_()
        stats[j].zero_()
    torch.cuda.synchronize()
    # every batch's arrays stay referenced until the end, so no later allocation can reuse
    # them while a persistent kernel still claims primaries from them, whatever stream it is on
    keep = []
    t0 = time.perf_counter()
    for k in range(k_steps):
        j = k % 2
        with torch.cuda.stream(streams[j]):
            b = R.sample_primaries(ctxs[j], sampler, 0, n, stream=streams[j])
            keep.append(b)
            R.run(ctxs[j], species, b, cfg, hist=hists[j], stats=stats[j], stream=streams[j])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = 0
    per_ctx = []
    for j in range(2):
        st = R.parse_stats(stats[j])
        per_ctx.append({k: st[k] for k in ("primaries", "finished", "clones", "pair_evals", "n_cancelled",
                                            "w_quarantined", "error_flags")})
        pairs += st["pair_evals"]
        batches = (k_steps + 1 - j) // 2
        tot = float(hists[j].sum().item()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
            st["w_quarantined"] + st["w_cancelled"]
        assert tot == float(n * batches), ("weight ledger broken", j, tot)
        assert st["primaries"] == n * batches and st["error_flags"] == 0, ("batches incomplete", j, st)
    for c in ctxs:
        c.close()
    return dict(batches=k_steps, ms_per_batch=1e3 * wall / k_steps, force_evals_per_s=pairs / wall,
                per_context=per_ctx,
                method="two streams and contexts, batches alternate, no host synchronisation between them")


def fp32_leg(R, ctx, torch, w, sampler, slices, base, stream, form, lanes=0, waves=0):
    """The same workload with the FP32 pair term (FP64 integration and step control): its
    own autotuned shape (or the one given), one warm launch, then the given (id0, n) slices
    timed.  Reported beside the FP64 headline, never as it."""
    f = R.FORM_PLAIN if form == "plain" else R.FORM_PERSISTENT
    id0, n = slices[0]
    batch = R.sample_primaries(ctx, sampler, 0, n, id0=id0)
    if lanes == 0:
        lanes, waves = R.autotune(ctx, w["species"], batch,
                                  R.RunConfig(form=f, force_precision=R.FORCE_FP32, **base), pilot=n)
    cfg = R.RunConfig(form=f, lanes_per_track=lanes, waves_per_cu=waves, force_precision=R.FORCE_FP32, **base)
    R.run(ctx, w["species"], batch, cfg, id0=id0)
    torch.cuda.synchronize()
    kms, pairs, tracks = [], 0, 0
    t_all = 0.0
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    for id0, n in slices:
        b = R.sample_primaries(ctx, sampler, 0, n, id0=id0, stream=stream)
        hist.zero_()
        stats.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        st = R.parse_stats(stats)
        pairs += st["pair_evals"]
        tracks += st["finished"]
        kms.append(e0.elapsed_time(e1))
    k_total = sum(kms) * 1e-3
    # ideal time at the two vector peaks over the measured kernel time
    t_ideal = pairs * ((FLOP_PER_PAIR - FLOP_PER_PAIR_F32_PART) / FP64_VECTOR_PEAK_TFLOPS +
                       FLOP_PER_PAIR_F32_PART / FP32_VECTOR_PEAK_TFLOPS) * 1e-12
    return dict(force_evals_per_s=pairs / t_all, tracks_per_s=tracks / t_all,
                kernel_ms_per_step=[round(x, 1) for x in kms], lanes_per_track=lanes, waves_per_cu=waves,
                slices=[list(x) for x in slices],
                roofline={"bound": "alu", "peak": f"FP64 {FP64_VECTOR_PEAK_TFLOPS} + FP32 {FP32_VECTOR_PEAK_TFLOPS} TFLOP/s",
                          "fp64_flop_per_pair": FLOP_PER_PAIR - FLOP_PER_PAIR_F32_PART,
                          "fp32_flop_per_pair": FLOP_PER_PAIR_F32_PART,
                          "frac": t_ideal / k_total},
                tolerance="1e-5 relative per step against the FP64 oracle")


def domain_leg(R, torch, pilot=8192):
    """The interaction-set autotuner on the 10 keV As workload (65,536 primaries, 8 cloning
    depths, persistent form, autotuned lanes): a pilot of the first primaries with the 27 cells
    and with cut-offs of 5 and 6 A, each gated against the 27-cell pilot (weighted KS p > 0.01,
    mean and std within 1 % or three standard errors) and timed; the recorded set is then timed
    on the whole batch (r_cut < 0) beside the 27 cells."""
    n = 65536
    ctx = R.Context()
    w, sampler, thr, _ = workload_setup(R, "c1", n)
    base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=thr, form=R.FORM_PERSISTENT)
    batch = R.sample_primaries(ctx, sampler, 0, n)
    lanes, waves = R.autotune(ctx, w["species"], batch, R.RunConfig(**base), pilot=n)
    cfg = dict(lanes_per_track=lanes, waves_per_cu=waves, **base)
    best, rows = R.autotune_domain(ctx, w["species"], batch, R.RunConfig(**cfg), candidates=(0.0, 5.0, 6.0),
                                   pilot=pilot)
    out = dict(pilot=pilot, lanes_per_track=lanes, chosen_r_cut_A=best,
               candidates=[dict(r_cut_A=r[0], pilot_ms=round(r[1], 1), ks_p=r[2], rel_mean_diff=r[3],
                                rel_std_diff=r[4], passed=r[5]) for r in rows])
    timed = {}
    for name, rc in (("27_cells", 0.0), ("recorded_set", -1.0)):
        if name == "recorded_set" and best == 0.0:
            break
        st = R.new_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.run(ctx, w["species"], batch, R.RunConfig(r_cut=rc, **cfg), stats=st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = R.parse_stats(st)
        timed[name] = dict(ms=round(1e3 * dt, 1), tracks_per_s=s["finished"] / dt, force_evals_per_s=s["pair_evals"] / dt,
                           pair_terms_per_step=s["pair_evals"] / s["track_steps"])
    out["whole_batch"] = timed
    ctx.close()
    return out


def fkbk_leg(R, torch, n=65536):
    """The paper's stopping model (Firsov local loss + Brandt-Kitagawa, interstitial electron
    density of silicon's valence electrons) beside the local Lindhard-Scharff reading on the
    same batch: B at 1 keV, 7 degree tilt, plain form."""
    from tests.workloads import WORKLOADS
    w = WORKLOADS["c0_b1kev"]
    out = {}
    for name, kw in (("local_lindhard_scharff", dict()),
                     ("firsov_brandt_kitagawa", dict(stop_mode=R.STOP_FKBK, n_e=R.SILICON_VALENCE_DENSITY))):
        ctx = R.Context(**kw)
        b = R.sample_primaries(ctx, R.SamplerConfig(**w["sampler"]), 0, n)
        cfg = R.RunConfig(n_bins=w["n_bins"])
        R.run(ctx, w["species"], b, cfg)
        st = R.new_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.run(ctx, w["species"], b, cfg, stats=st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = R.parse_stats(st)
        out[name] = dict(ms=round(1e3 * dt, 1), force_evals_per_s=s["pair_evals"] / dt, tracks_per_s=s["finished"] / dt,
                         mean_depth_A=s["sum_wz"] / max(s["w_stopped"], 1e-300), steps_per_track=s["track_steps"] / n)
        ctx.close()
    out["workload"] = f"{n} B at 1 keV into Si, 7 deg tilt, no cloning, plain form"
    return out


def uo2_leg(R, torch, n_override=0):
    """The 85 keV U recoil workload in fluorite UO2 (5,120 primaries, on-site start with the
    site left vacant, random directions, 8 cloning distances from the start point): autotuned
    shape (64 or 32 lanes), one warm launch, two timed launches."""
    from tests.workloads import C5_THRESHOLDS, UO2, WORKLOADS
    w = dict(WORKLOADS["c5_u85kev_uo2"])
    if n_override > 0:
        w["n"] = n_override
    ctx = R.Context(structure=R.FLUORITE, **UO2)
    sc = R.SamplerConfig(**w["sampler"])
    base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=[list(C5_THRESHOLDS)],
                range_mode=w["range_mode"], vacancy=w["vacancy"], form=R.FORM_PERSISTENT)
    batch = R.sample_primaries(ctx, sc, 0, w["n"])
    lanes, waves = R.autotune(ctx, w["species"], batch, R.RunConfig(**base), pilot=w["n"])
    cfg = R.RunConfig(lanes_per_track=lanes, waves_per_cu=waves, **base)
    R.run(ctx, w["species"], batch, cfg)
    torch.cuda.synchronize()
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    pairs = tracks = 0
    t_all = 0.0
    kms = []
    stream = torch.cuda.current_stream()
    for _ in range(2):
        b = R.sample_primaries(ctx, sc, 0, w["n"], stream=stream)
        hist.zero_()
        stats.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        st = R.parse_stats(stats)
        pairs += st["pair_evals"]
        tracks += st["finished"]
        kms.append(e0.elapsed_time(e1))
    mean_range = st["sum_wz"] / max(st["w_stopped"], 1e-300)
    shape = R.launch_shape(ctx, batch, cfg)
    ctx.close()
    k = sum(kms) / len(kms)
    return dict(primaries=w["n"], workload="U at 85 keV in UO2 (a=5.47 A, sigma U 0.050 / O 0.067 A), on-site recoils "
                         "at 1,094 A depth, random direction, vacant start site, radial range, 8 cloning "
                         "distances, 0.5 A bins",
                force_evals_per_s=pairs / t_all, tracks_per_s=tracks / t_all, kernel_ms_per_step=[round(x, 1) for x in kms],
                launch=shape, mean_range_A=mean_range,
                roofline={"bound": "alu", "achieved": FLOP_PER_PAIR * pairs / 2 / (k * 1e-3) / 1e12,
                          "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": FLOP_PER_PAIR * pairs / 2 / (k * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS})


def grad_forward_ratio(R, ctx, torch):
    """T(reedmd_grad) / T(reedmd_run) on the adjoint workload: 4,096 P at 5 keV into Si
    [001] at 7 degree tilt, no cloning, d(mean range)/d(k, s) with a checkpoint every 64 steps.
    Beside the cost: per-track derivatives against central differences on the same seeded
    crystal.  A track is linear in k (or s) where the differences at h = 1e-7 and 1e-8 agree to
    1e-4; the fraction of such tracks, the adjoint's agreement with the h = 1e-7 difference on
    them, and the all-track mean of the pathwise derivative with its standard error (which the
    few exploding, non-linear tracks dominate) are reported."""
    import math
    import numpy as np
    sc = R.SamplerConfig(choice=(0,), E_min=5000.0, E_max=5000.0, tilt=math.radians(7.0))
    b = R.sample_primaries(ctx, sc, 0, 4096)
    cfg = R.RunConfig(max_steps=16384, lanes_per_track=64)
    R.run(ctx, ("P",), b, cfg)
    R.grad(ctx, ("P",), b, cfg, 1.0, 1.0)
    torch.cuda.synchronize()
    tf, tg = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        h, st, _ = R.run(ctx, ("P",), b, cfg)
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        g = R.grad(ctx, ("P",), b, cfg, 1.0, 1.0)
        torch.cuda.synchronize()
        tg.append(time.perf_counter() - t0)
    steps = R.parse_stats(st)["track_steps"]
    tr = R.grad(ctx, ("P",), b, cfg, 1.0, 1.0, per_track=True)["tracks"].cpu().numpy()
    stopped = tr[:, 3] == R.STOPPED

    def fd(which, hh):
        up, dn = dict(k=1.0, s=1.0), dict(k=1.0, s=1.0)
        up[which] += hh
        dn[which] -= hh
        zu = R.grad(ctx, ("P",), b, cfg, up["k"], up["s"], per_track=True)["tracks"].cpu().numpy()
        zd = R.grad(ctx, ("P",), b, cfg, dn["k"], dn["s"], per_track=True)["tracks"].cpu().numpy()
        ok = (zu[:, 3] == R.STOPPED) & (zd[:, 3] == R.STOPPED)
        mean_fd = (zu[zu[:, 3] == R.STOPPED, 0].mean() - zd[zd[:, 3] == R.STOPPED, 0].mean()) / (2 * hh)
        return (zu[:, 0] - zd[:, 0]) / (2 * hh), ok, mean_fd

    check = {}
    for col, which in ((1, "k"), (2, "s")):
        f1, ok1, _ = fd(which, 1e-7)
        f2, ok2, _ = fd(which, 1e-8)
        _, _, mean4 = fd(which, 1e-4)
        ok = stopped & ok1 & ok2
        lin = ok & (np.abs(f1 - f2) <= 1e-4 * np.maximum(np.maximum(np.abs(f1), np.abs(f2)), 1e-3))
        adj = tr[:, col]
        d = dict(tracks_stopped=int(ok.sum()), linear=int(lin.sum()), linear_fraction=float(lin.sum() / max(ok.sum(), 1)),
                 all_track_mean=float(adj[stopped].mean()),
                 all_track_se=float(adj[stopped].std(ddof=1) / math.sqrt(max(stopped.sum(), 2))),
                 fd_of_mean_range_h_1em4=float(mean4))
        if lin.any():
            d.update(linear_mean_adjoint=float(adj[lin].mean()), linear_mean_fd_h_1em7=float(f1[lin].mean()),
                     linear_mean_rel_diff=float(abs(adj[lin].mean() - f1[lin].mean()) / max(np.abs(f1[lin]).mean(), 1e-3)),
                     linear_worst_track_rel_diff=float((np.abs(adj[lin] - f1[lin]) / np.maximum(np.abs(f1[lin]), 1e-3)).max()),
                     linear_tracks_beyond_1e_3=int(((np.abs(adj[lin] - f1[lin]) / np.maximum(np.abs(f1[lin]), 1e-3)) > 1e-3).sum()))
        check["d_d" + which] = d
    return dict(workload="4,096 P at 5 keV, 7 deg tilt, no cloning, checkpoint every 64 steps",
                forward_ms=1e3 * min(tf), grad_ms=1e3 * min(tg), ratio=min(tg) / min(tf),
                steps_per_track=steps / 4096, mean_range_A=g["mean"], dR_dk=g["dk"], dR_ds=g["ds"],
                stopped=g["count"], finite_difference_check=check,
                note="the pathwise mean over all tracks is dominated by a few exploding chaotic tracks and is "
                     "not an estimate of the derivative of the expected range; the FD agreement is shown on "
                     "the tracks that are linear at h = 1e-7 / 1e-8 (agreement 1e-4); a few strongly amplifying "
                     "tracks among them have step-size branches that switch within ~1e-9 of k = 1, so their "
                     "differences average slopes the pathwise derivative does not see (counted beyond 1e-3)")


def progress(msg):
    """One line per finished launch or leg on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def plan_steps(N, K, W, whole):
    """(primaries per step, timed (id0, n) slices, warm-up slices).  Sliced: timed step k runs
    ids [k s, (k+1) s) with s = ceil(N / K), so the timed steps together run ids 0..N-1 once;
    warm-up step j runs ids [N + j s, N + (j+1) s), disjoint from them.  Whole: every step runs
    ids 0..N-1."""
    K = max(1, K)
    if whole:
        return N, [(0, N)] * K, [(0, N)] * W
    s = -(-N // K)
    return s, [(j * s, min(s, N - j * s)) for j in range(K) if j * s < N], [(N + j * s, s) for j in range(W)]


def timed_launches(R, torch, ctx, w, sampler, cfg, slices, stream, log_first=False):
    """Runs each (id0, n) slice: sample on the device, clear the outputs, run; HIP events on
    the launch stream bracket the run.  Returns per-launch kernel ms, summed statistics and
    the wall time, and checks every launch's weight ledger."""
    hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
    stats = R.new_stats()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in slices]
    tot = dict(pairs=0, tracks=0, prims=0, steps=0)
    kms, queue_use, log = [], [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (id0, n) in enumerate(slices):
        b = R.sample_primaries(ctx, sampler, 0, n, id0=id0, stream=stream)
        hist.zero_()
        stats.zero_()
        ev[k][0].record(stream)
        if log_first and k == 0:
            _, _, lg, _ = R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, log_cap=40 * n,
                                stream=stream)
        else:
            R.run(ctx, w["species"], b, cfg, hist=hist, stats=stats, id0=id0, stream=stream)
        ev[k][1].record(stream)
        torch.cuda.synchronize()
        st = R.parse_stats(stats)
        if log_first and k == 0:
            log = R.parse_log(lg, min(st["log_count"], 40 * n))
        ledger = float(hist.sum().item()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
            st["w_quarantined"] + st["w_cancelled"]
        assert ledger == float(n) and st["primaries"] == n, ("weight ledger broken", k, ledger, n)
        tot["pairs"] += st["pair_evals"]
        tot["tracks"] += st["finished"]
        tot["prims"] += st["primaries"]
        tot["steps"] += st["track_steps"]
        kms.append(ev[k][0].elapsed_time(ev[k][1]))
        queue_use.append([st["max_queue"], st["stack_overflow"], st["handed_off"]])
        progress(f"launch {k + 1}/{len(slices)} ids {id0}..{id0 + n - 1}: {kms[-1]:.1f} ms, "
                 f"{st['pair_evals'] / (kms[-1] * 1e-3):.4g} force evals/s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return kms, tot, wall, queue_use, log


def stream_launches(R, torch, ctxs, w, sampler, cfg, slices, streams, first=0):
    """Runs the (id0, n) slices round-robin over the streams, slice k on stream (first + k) mod
    S with its own context (clone queue, stacks, graph), histogram and statistics, and no host
    synchronisation until the last one is issued: a slice whose last long tracks occupy a few
    compute units leaves the rest to the slices after it.  HIP events on each slice's stream
    bracket its run.  Returns per-slice kernel ms, summed statistics, the wall time, the GPU
    span (first start event to the last end event) and the per-slice queue use, after checking
    every slice's weight ledger."""
    S = len(streams)
    hists = [torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda") for _ in slices]
    stats = [R.new_stats() for _ in slices]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in slices]
    keep = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, (id0, n) in enumerate(slices):
        j = (first + k) % S
        with torch.cuda.stream(streams[j]):
            b = R.sample_primaries(ctxs[j], sampler, 0, n, id0=id0, stream=streams[j])
            keep.append(b)
            ev[k][0].record(streams[j])
            keep.append(R.run(ctxs[j], w["species"], b, cfg, hist=hists[k], stats=stats[k], id0=id0,
                              stream=streams[j]))
            ev[k][1].record(streams[j])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = dict(pairs=0, tracks=0, prims=0, steps=0)
    kms, queue_use = [], []
    for k, (id0, n) in enumerate(slices):
        st = R.parse_stats(stats[k])
        ledger = float(hists[k].sum().item()) + st["w_underflow"] + st["w_overflow"] + st["w_backscattered"] + \
            st["w_quarantined"] + st["w_cancelled"]
        assert ledger == float(n) and st["primaries"] == n, ("weight ledger broken", k, ledger, n)
        tot["pairs"] += st["pair_evals"]
        tot["tracks"] += st["finished"]
        tot["prims"] += st["primaries"]
        tot["steps"] += st["track_steps"]
        kms.append(ev[k][0].elapsed_time(ev[k][1]))
        queue_use.append([st["max_queue"], st["stack_overflow"], st["handed_off"]])
    span = max(ev[0][0].elapsed_time(e[1]) for e in ev)
    progress(f"{len(slices)} slices on {S} streams: {wall:.2f} s wall, GPU span {span / 1e3:.2f} s, "
             f"{tot['pairs'] / wall:.4g} force evals/s")
    return kms, tot, wall, span, queue_use


def c1_leg(R, torch, np, args):
    """The 10 keV As workload (65,536 primaries, 8 cloning depths) in its autotuned persistent
    shape: one warm launch that logs every finished track (profile accuracy against the same
    primaries without cloning), then two timed launches of the whole batch."""
    n = 65536
    ctx = R.Context()
    w, sampler, thr, tail_depth = workload_setup(R, "c1", n)
    base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=thr, queue_capacity=args.queue)
    batch = R.sample_primaries(ctx, sampler, 0, n)
    lanes, waves = R.autotune(ctx, w["species"], batch, R.RunConfig(form=R.FORM_PERSISTENT, **base), pilot=n)
    cfg = R.RunConfig(form=R.FORM_PERSISTENT, lanes_per_track=lanes, waves_per_cu=waves, **base)
    stream = torch.cuda.current_stream()
    kw, _, t_w, _, reed_log = timed_launches(R, torch, ctx, w, sampler, cfg, [(0, n)], stream, log_first=True)
    kms, tot, wall, queue_use, _ = timed_launches(R, torch, ctx, w, sampler, cfg, [(0, n)] * 2, stream)
    k = sum(kms) / len(kms)
    achieved = FLOP_PER_PAIR * tot["pairs"] / len(kms) / (k * 1e-3) / 1e12
    out = dict(workload="65,536 As at 10 keV into Si, half within 0.5 deg of [110], half at 7 deg tilt; "
                        "8 cloning depths x 2 clones; 1 A bins 0-8192 A",
               force_evals_per_s=tot["pairs"] / wall, tracks_per_s=tot["tracks"] / wall,
               kernel_ms_per_step=[round(x, 1) for x in kms], launch=R.launch_shape(ctx, batch, cfg),
               queue_max_overflow_handoff_per_step=queue_use,
               roofline={"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VECTOR_PEAK_TFLOPS})
    out["profile_accuracy"] = profile_accuracy(R, torch, np, ctx, w, sampler, n, cfg, reed_log, kw[0] * 1e-3,
                                               tail_depth)
    if args.refine_epochs > 0:
        from tests.workloads import C1_THRESHOLDS
        out["refined"] = dict(epochs=args.refine_epochs, fixed_depths_ms=k)
        for name, inl in (("epoch_launches", False), ("in_launch", True)):
            b = R.sample_primaries(ctx, sampler, 0, n, stream=stream)
            hist = torch.zeros(w["n_bins"], dtype=torch.float64, device="cuda")
            stats = R.new_stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, depths = R.run_refined(ctx, w["species"], b, cfg, args.refine_epochs,
                                         [2.0 ** -j for j in range(1, len(C1_THRESHOLDS) + 1)], 1.0,
                                         hist=hist, stats=stats, stream=stream, in_launch=inl)
            torch.cuda.synchronize()
            tr = time.perf_counter() - t0
            sr = R.parse_stats(stats)
            ledger = float(hist.sum().item()) + sr["w_underflow"] + sr["w_overflow"] + sr["w_backscattered"] + \
                sr["w_quarantined"]
            assert ledger == float(n) and sr["primaries"] == n, ("weight ledger broken", name, ledger)
            out["refined"][name] = dict(ms=1e3 * tr, force_evals_per_s=sr["pair_evals"] / tr,
                                        tracks=sr["finished"],
                                        last_depths=[round(x, 1) for x in depths[-1, 0].tolist()])
            progress(f"refined depths, {name}: {tr:.2f} s, {sr['finished']} tracks, "
                     f"{sr['pair_evals'] / tr:.4g} force evals/s")
    if args.pipelined > 0:
        out["pipelined"] = pipelined_leg(R, torch, w, sampler, n, cfg, args.pipelined, w["species"])
    ctx.close()
    return out


DESCR = {
    "c1": "c1_as10kev: 65,536 As at 10 keV into diamond Si (a=5.431 A, sigma=0.076 A), "
          "half within 0.5 deg of [110], half at 7 deg tilt; ZBL + local LSS k=1; "
          "dx_max 0.05 A; 8 cloning depths x 2 clones; 1 A bins 0-8192 A",
    "c2": "c2_mixed: 1,048,576 primaries, species uniform over B/P/As, energy log-uniform 1-100 keV, "
          "7 deg tilt into diamond Si (a=5.431 A, sigma=0.076 A); ZBL + local LSS k=1; dx_max 0.05 A; "
          "12 cloning depths x 2 clones per (species, energy decade) table; 1 A bins 0-8192 A; "
          "persistent kernel, device queue, hipGraph, autotuned shape",
    "c4": "c4_as100kev: 262,144 As at 100 keV along [001] (0 deg); 16 cloning depths to 1e-6; "
          "0-500 nm in 0.5 nm bins",
}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        # a plain copy of known size: reads 1 GiB and writes 1 GiB of HBM per launch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "launches": 3}))
        return

    import paper_0810_4737_amd as R
    from tests.workloads import WORKLOADS

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    key = args.workload
    N = args.n if args.n > 0 else WORKLOADS[WORKLOAD_NAMES[key]]["n"]
    whole = args.whole or key == "c1"
    sl, timed, warm = plan_steps(N, args.steps, args.warmup, whole)
    ctx = R.Context()
    w, sampler, thr, _ = workload_setup(R, key, N)
    base = dict(n_bins=w["n_bins"], bin_width=w["bin_width"], thresholds=thr, queue_capacity=args.queue)
    stream = torch.cuda.current_stream()

    # launch shape: explicit, or the autotuner on a batch of the same workload (the first
    # warm-up slice, or the first timed one when there is no warm-up)
    tid0, tn = (warm or timed)[0]
    tb = R.sample_primaries(ctx, sampler, 0, tn, id0=tid0)
    if args.lanes == 0:
        f = R.FORM_PLAIN if args.form == "plain" else R.FORM_PERSISTENT
        lanes, waves = R.autotune(ctx, w["species"], tb, R.RunConfig(form=f, **base), pilot=tn)
    else:
        f, lanes, waves = (R.FORM_PLAIN if args.form == "plain" else R.FORM_PERSISTENT), args.lanes, args.waves
    cfg = R.RunConfig(form=f, lanes_per_track=lanes, waves_per_cu=waves, **base)
    shape = R.launch_shape(ctx, tb, cfg)
    S = max(1, args.streams) if not whole else 1
    if S > 1 and args.waves == 0 and f == R.FORM_PERSISTENT and args.grid_share == "half":
        # steps on several streams share the GPU: each persistent grid takes half of the
        # workgroups that fit (at least one per CU), so that the bulk of the next steps and the
        # tail launches of the earlier ones run side by side
        bpc = max(1, waves // 4) if waves > 0 else shape["blocks_per_cu"]
        waves = 4 * max(1, bpc // 2)
        cfg = R.RunConfig(form=f, lanes_per_track=lanes, waves_per_cu=waves, **base)
        shape = R.launch_shape(ctx, tb, cfg)

    progress(f"workload {key}: {N} primaries, {sl} per step, shape {shape}")
    if S == 1:
        if warm:
            progress("warm-up")
            timed_launches(R, torch, ctx, w, sampler, cfg, warm, stream)
        progress("timed steps")
        kernel_ms, tot, wall, queue_use, _ = timed_launches(R, torch, ctx, w, sampler, cfg, timed, stream)
        span = sum(kernel_ms)
    else:
        # the first context is the one the autotuner ran on; the others take its launch shape
        ctxs = [ctx] + [R.Context() for _ in range(S - 1)]
        streams = [torch.cuda.Stream() for _ in range(S)]
        if warm:
            progress("warm-up")
            stream_launches(R, torch, ctxs, w, sampler, cfg, warm, streams)
        progress("timed steps")
        kernel_ms, tot, wall, span, queue_use = stream_launches(R, torch, ctxs, w, sampler, cfg, timed, streams,
                                                                first=len(warm))
        for c in ctxs[1:]:
            c.close()

    steps = len(timed)
    ms_step = wall * 1e3 / steps
    value = tot["pairs"] / wall
    # GPU time of the timed steps: the sum of the launches one after another, or with several
    # streams the span from the first launch's start to the last one's end (launches overlap)
    k_sum = span * 1e-3
    achieved = FLOP_PER_PAIR * tot["pairs"] / k_sum / 1e12
    m = MEASURED_TRAFFIC
    traffic = None
    if (kernel_sources_hash() == m["sources_sha256_prefix"] and key == m["workload"] and not whole
            and cfg.form == R.FORM_PERSISTENT and shape["lanes"] == m["lanes"] and shape["blocks"] == m["blocks"]
            and N == m["primaries"]
            and sl == m["slice"]):
        traffic = m["fetch_bytes"] + m["write_bytes"]
    out = {
        "metric": "ion-atom force evaluations per second (REED-MD track throughput)",
        "value": value,
        "unit": "force evals/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": DESCR[key],
            "primaries": N,
            "primaries_per_step": sl,
            "step": ("the whole batch" if whole else
                     f"ids [k*{sl}, (k+1)*{sl}) of step k; the {steps} timed steps run all {N} primaries, "
                     f"warm-up steps ids from {N} on"),
            "form": "persistent" if cfg.form == R.FORM_PERSISTENT else "plain",
            "lanes_per_track": lanes,
            "waves_per_cu": waves,
            "launch": shape,
            "streams": S,
        },
        "tracks_per_s": tot["tracks"] / wall,
        "primaries_per_s": tot["prims"] / wall,
        "track_steps_per_s": tot["steps"] / wall,
        "kernel_ms_per_step": [round(x, 1) for x in kernel_ms],
        "queue_max_overflow_handoff_per_step": queue_use,
        "grad_fwd_ratio": None,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "kernel": "track_kernel (reedmd_run)",
            "kernel_ms": k_sum * 1e3 / steps,
            "gpu_time": ("sum of the launches" if S == 1 else
                         f"span of the {steps} launches on {S} streams (first start to last end event)"),
            "flop_per_pair": FLOP_PER_PAIR,
            "pairs_per_launch": tot["pairs"] / steps,
        },
    }
    if not args.no_fp32:
        progress("fp32 leg")
        out["fp32_pair_variant"] = fp32_leg(R, ctx, torch, w, sampler, timed[:2], base, stream, args.form,
                                            args.lanes, args.waves)
    ctx.close()
    if key != "c1" and not args.no_c1:
        progress("c1 leg")
        out["c1_as10kev"] = c1_leg(R, torch, np, args)
    if not args.no_c4:
        progress("c4 leg")
        out["c4_as100kev_tail_accuracy"] = c4_leg(R, torch, np)
    if not args.no_domain:
        progress("interaction-set leg")
        out["interaction_set"] = domain_leg(R, torch)
    if not args.no_fkbk:
        progress("fkbk leg")
        out["fkbk_stopping"] = fkbk_leg(R, torch)
    if not args.no_uo2:
        progress("uo2 leg")
        out["uo2_recoil"] = uo2_leg(R, torch, args.uo2_n)
    if not args.no_grad:
        progress("grad leg")
        gctx = R.Context()
        gr = grad_forward_ratio(R, gctx, torch)
        gctx.close()
        out["grad_fwd_ratio"] = gr["ratio"]
        out["grad"] = gr
    if not args.no_cpu:
        progress("cpu leg")
        out["cpu_baseline"] = cpu_baseline(key, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

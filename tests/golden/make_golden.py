"""Writes the stored oracle results used by the GPU statistical parity tests.

Calls only the oracle (``oracle/``).
Usage:  python tests/golden/make_golden.py [pilot|pilot2|pilot4|c0|c1|c2|c4|refine]
  pilot: unsplit survival quantiles of the 10 keV As workload (source of C1_THRESHOLDS)
  pilot2: cloning-depth tables of the mixed B/P/As 1-100 keV workload (C2_THRESHOLDS)
  pilot4: cloning depths of the 100 keV As [001] channeling workload (C4_THRESHOLDS)
  pilot5: cloning distances of the 85 keV U recoils in UO2 (C5_THRESHOLDS)
  c5:    256 U recoils at 85 keV in UO2 (ids 0..255) with the 8 cloning distances
  c5refine: 512 U recoils at 85 keV in UO2 with 8 distances at survival 2^-k re-placed between
         4 epochs from a deliberately short first table
  c0:    65,536 B at 1 keV, 7 degree tilt, no splitting (the c0 sampler, ids 0..65535)
  c0fkbk: 32,768 B at 1 keV (the c0 sampler, ids 0..32767) with the Firsov + Brandt-Kitagawa
         stopping, interstitial electron density 32 / a^3 (silicon's valence electrons)
  c1:    1,024 As at 10 keV with the 8 cloning depths: ids 0..511 (channel) and 32768..33279 (tilt)
  refine: 2,048 B at 1 keV (the c0 sampler, ids 0..2047) with 6 adaptive cloning depths at
         survival 2^-k, re-placed between 4 epochs from a deliberately shallow first table
  c1big: 8,192 As at 10 keV with the 8 cloning depths: ids 0..4095 (channel) and 32768..36863 (tilt)
  c2big: 16,384 primaries of the mixed B/P/As 1-100 keV workload (ids 0..16383), 6 x 12 depths
  c4big: 1,024 As at 100 keV along [001] (ids 0..1023), 16 depths to 1e-6
  (the *big runs use the library's default step cap of 2,000,000 steps per track)
Outputs go next to this file as JSON (histogram, totals, moments) plus gzipped text of every
stopped track's depth and weight.
"""
import gzip
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from tests.workloads import C1_THRESHOLDS, C2_THRESHOLDS, C4_THRESHOLDS, C5_THRESHOLDS, WORKLOADS  # noqa: E402


def sampler(w):
    return oracle.SamplerCfg(**w["sampler"])


def save(name, cfg_desc, r, extra=None, lineage=False):
    """lineage=True adds each stopped track's primary id as a third column (standard errors
    by primary family)."""
    st = r["stats"]
    log = r["log"]
    stopped = log[log["status"] == oracle.STOPPED]
    order = np.lexsort((stopped["lineage"], stopped["w"], stopped["z_stop"]))
    z = stopped["z_stop"][order]
    w = stopped["w"][order]
    lin = stopped["lineage"][order]
    W = w.sum()
    mean = float((w * z).sum() / W)
    std = float(math.sqrt((w * (z - mean) ** 2).sum() / W))
    out = dict(workload=cfg_desc, stats=st, hist=r["hist"].tolist(), mean=mean, std=std,
               n_stopped=int(len(z)), nthreads=r["nthreads"])
    if extra:
        out.update(extra)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)
    with gzip.open(os.path.join(HERE, name + "_stopped.txt.gz"), "wt") as f:
        if lineage:
            for zi, wi, li in zip(z, w, lin):
                f.write(f"{zi:.17g} {wi:.17g} {int(li)}\n")
        else:
            for zi, wi in zip(z, w):
                f.write(f"{zi:.17g} {wi:.17g}\n")


def pilot():
    w = WORKLOADS["c1_as10kev"]
    sc = sampler(w)
    sc.n_cone = 256
    prim = oracle.sample_primaries(sc, 0, 512)
    r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"]), prim, log=True)
    log = r["log"]
    z = np.sort(log["z_stop"][log["status"] == oracle.STOPPED])
    q = [float(np.quantile(z, 1 - 2.0 ** -k)) for k in range(1, 9)]
    print("survival 2^-k depths:", [round(x, 1) for x in q])
    print("stored:", C1_THRESHOLDS)


def survival_depths(z, probs, min_tail=4, min_gap=2.0):
    """Depths at which the empirical unsplit survival S(z) = P(z_stop > z) equals each target
    probability.  Where fewer than min_tail pilot ions lie beyond, the tail is extrapolated
    with an exponential fitted (least squares on ln S) to the pilot's last decade of
    survival; the result is made strictly increasing with at least min_gap between depths."""
    z = np.sort(np.asarray(z, float))
    n = len(z)
    S = 1.0 - (np.arange(1, n + 1) / n)          # survival just above each sorted depth
    sel = (S >= min_tail / n) & (S <= 0.1)
    if sel.sum() < 3:
        sel = S >= min_tail / n
    slope, icept = np.polyfit(z[sel], np.log(S[sel]), 1)
    out = []
    for p in probs:
        if p * n >= min_tail:
            d = float(np.quantile(z, 1.0 - p))
        else:
            d = float((math.log(p) - icept) / slope)
        if out and d < out[-1] + min_gap:
            d = out[-1] + min_gap
        out.append(round(d, 1))
    return out


def pilot2():
    """12 depths per (species, energy decade) table at survival 10^(-5k/12), k = 1..12."""
    w = WORKLOADS["c2_mixed"]
    probs = [10.0 ** (-5.0 * k / 12.0) for k in range(1, 13)]
    tables = []
    for si in range(3):
        for band, (e0, e1) in enumerate(((1000.0, 10000.0), (10000.0, 100000.0))):
            sc = oracle.SamplerCfg(choice=(si,), E_min=e0, E_max=e1, tilt=w["sampler"]["tilt"])
            prim = oracle.sample_primaries(sc, 1, 256)
            r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"]), prim, log=True)
            lg = r["log"]
            tables.append(survival_depths(lg["z_stop"][lg["status"] == oracle.STOPPED], probs))
    print("C2_THRESHOLDS =", tables)
    print("stored:", C2_THRESHOLDS)


def pilot4():
    """16 depths at survival 10^(-6k/16), k = 1..16."""
    w = WORKLOADS["c4_as100kev"]
    probs = [10.0 ** (-6.0 * k / 16.0) for k in range(1, 17)]
    sc = oracle.SamplerCfg(**w["sampler"])
    prim = oracle.sample_primaries(sc, 2, 128)
    r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"]),
                   prim, log=True)
    lg = r["log"]
    print("C4_THRESHOLDS =", survival_depths(lg["z_stop"][lg["status"] == oracle.STOPPED], probs))
    print("stored:", C4_THRESHOLDS)


def c5_config(w, thresholds=None):
    t = w["target"]
    return oracle.Config(species=w["species"], structure=oracle.FLUORITE, a=t["a"], Z2=t["Z2"], M2=t["M2"],
                         sigma=t["sigma"], Z2b=t["Z2b"], M2b=t["M2b"], sigma_b=t["sigma_b"],
                         range_mode=w["range_mode"], vacancy=w["vacancy"], n_bins=w["n_bins"],
                         bin_width=w["bin_width"], thresholds=thresholds if thresholds is not None else np.zeros((1, 0)))


def pilot5():
    """8 cloning distances of the 85 keV U recoils in UO2 at unsplit survival 2^-k."""
    w = WORKLOADS["c5_u85kev_uo2"]
    probs = [2.0 ** -k for k in range(1, 9)]
    prim = oracle.sample_primaries(sampler(w), 5, 512)
    t = time.time()
    r = oracle.run(c5_config(w), prim, log=True)
    lg = r["log"]
    print("pilot5 seconds", time.time() - t, r["stats"])
    print("C5_THRESHOLDS =", survival_depths(lg["z_stop"][lg["status"] == oracle.STOPPED], probs, min_gap=1.0))
    print("stored:", C5_THRESHOLDS)


def c5():
    """256 primaries of the 85 keV U recoil workload (ids 0..255), 8 cloning distances."""
    w = WORKLOADS["c5_u85kev_uo2"]
    prim = oracle.sample_primaries(sampler(w), 0, 256)
    t = time.time()
    r = oracle.run(c5_config(w, [list(C5_THRESHOLDS)]), prim, log=True)
    print("c5 oracle seconds", time.time() - t, r["stats"])
    save("c5_subset", dict(name="c5_u85kev_uo2", ids=[[0, 256]], seed=0), r)


def c0():
    w = WORKLOADS["c0_b1kev"]
    n = 65536
    prim = oracle.sample_primaries(sampler(w), 0, n)
    t = time.time()
    r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"]),
                   prim, log=True)
    print("c0 oracle seconds", time.time() - t, r["stats"])
    save("c0_accept", dict(name="c0_b1kev", n=n, seed=0, id0=0), r)


def c0fkbk():
    w = WORKLOADS["c0_b1kev"]
    n = 32768
    prim = oracle.sample_primaries(sampler(w), 0, n)
    n_e = 32.0 / 5.431 ** 3
    t = time.time()
    r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                                 stop_mode=oracle.STOP_FKBK, n_e=n_e), prim, log=True)
    print("c0fkbk oracle seconds", time.time() - t, r["stats"])
    save("c0_fkbk", dict(name="c0_b1kev", n=n, seed=0, id0=0, stopping="fkbk", n_e=n_e), r)


def c1():
    w = WORKLOADS["c1_as10kev"]
    sc = sampler(w)
    a = oracle.sample_primaries(sc, 0, 512, id0=0)
    b = oracle.sample_primaries(sc, 0, 512, id0=32768)
    prim = {k: np.concatenate([a[k], b[k]], axis=-1) for k in a}
    lineage = np.concatenate([np.arange(512), 32768 + np.arange(512)]).astype(np.int64)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=[list(C1_THRESHOLDS)])
    t = time.time()
    r = oracle.run(cfg, prim, log=True, lineage=lineage)
    print("c1 oracle seconds", time.time() - t, r["stats"])
    save("c1_subset", dict(name="c1_as10kev", ids=[[0, 512], [32768, 33280]], seed=0,
                           thresholds=list(C1_THRESHOLDS)), r)


REFINE = dict(n=2048, n_epochs=4, probs=[2.0 ** -k for k in range(1, 7)],
              first=[10.0, 20.0, 30.0, 40.0, 50.0, 60.0], min_gap=1.0)


def refine():
    """Adaptive cloning depths: the oracle's epoch runner on 2,048 B at 1 keV."""
    w = WORKLOADS["c0_b1kev"]
    prim = oracle.sample_primaries(sampler(w), 0, REFINE["n"])
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=[REFINE["first"]])
    t = time.time()
    r = oracle.run_refined(cfg, prim, REFINE["n_epochs"], REFINE["probs"], REFINE["min_gap"])
    print("refine oracle seconds", time.time() - t, r["stats"])
    print("depths", np.round(r["depths"], 2).tolist())
    save("c0_refined", dict(name="c0_b1kev", ids=[[0, REFINE["n"]]], seed=0, **REFINE), r,
         extra=dict(depths=r["depths"].tolist()))


REFINE5 = dict(n=512, n_epochs=4, probs=[2.0 ** -k for k in range(1, 9)],
               first=[40.0, 60.0, 80.0, 100.0, 120.0, 140.0, 160.0, 180.0], min_gap=1.0)


def c5refine():
    """Eight dynamically placed cloning distances for the 85 keV U recoils in UO2 (the setting
    of Sec. 4): the oracle's epoch runner on 512 primaries from a deliberately short table."""
    w = WORKLOADS["c5_u85kev_uo2"]
    prim = oracle.sample_primaries(sampler(w), 0, REFINE5["n"])
    cfg = c5_config(w, [REFINE5["first"]])
    t = time.time()
    r = oracle.run_refined(cfg, prim, REFINE5["n_epochs"], REFINE5["probs"], REFINE5["min_gap"])
    print("c5refine oracle seconds", time.time() - t, r["stats"])
    print("distances", np.round(r["depths"], 2).tolist())
    save("c5_refined", dict(name="c5_u85kev_uo2", ids=[[0, REFINE5["n"]]], seed=0, **REFINE5), r,
         extra=dict(depths=r["depths"].tolist()))


def c2():
    """256 primaries of the mixed workload (ids 0..255), all 12-depth tables."""
    w = WORKLOADS["c2_mixed"]
    prim = oracle.sample_primaries(sampler(w), 0, 256)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=C2_THRESHOLDS)
    t = time.time()
    r = oracle.run(cfg, prim, log=True)
    print("c2 oracle seconds", time.time() - t, r["stats"])
    save("c2_subset", dict(name="c2_mixed", ids=[[0, 256]], seed=0), r)


def c4():
    """32 primaries of the 100 keV As channeling workload (ids 0..31), 16 depths."""
    w = WORKLOADS["c4_as100kev"]
    prim = oracle.sample_primaries(sampler(w), 0, 32)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=[list(C4_THRESHOLDS)])
    t = time.time()
    r = oracle.run(cfg, prim, log=True)
    print("c4 oracle seconds", time.time() - t, r["stats"])
    save("c4_subset", dict(name="c4_as100kev", ids=[[0, 32]], seed=0), r)


# step cap of the larger stored runs: the HIP library's default, so that both sides quarantine
# the same (rare) tracks that never slow below the stopping energy
BIG_MAX_STEPS = 2_000_000


def c1big():
    """8,192 primaries of the 10 keV As workload: ids 0..4095 (channel) and 32768..36863 (tilt)."""
    w = WORKLOADS["c1_as10kev"]
    sc = sampler(w)
    a = oracle.sample_primaries(sc, 0, 4096, id0=0)
    b = oracle.sample_primaries(sc, 0, 4096, id0=32768)
    prim = {k: np.concatenate([a[k], b[k]], axis=-1) for k in a}
    lineage = np.concatenate([np.arange(4096), 32768 + np.arange(4096)]).astype(np.int64)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=[list(C1_THRESHOLDS)], max_steps=BIG_MAX_STEPS)
    t = time.time()
    r = oracle.run(cfg, prim, log=True, lineage=lineage)
    print("c1big oracle seconds", time.time() - t, r["stats"], flush=True)
    save("c1_accept", dict(name="c1_as10kev", ids=[[0, 4096], [32768, 36864]], seed=0,
                           thresholds=list(C1_THRESHOLDS), max_steps=BIG_MAX_STEPS), r,
         lineage=True)


def c2big():
    """16,384 primaries of the mixed workload (ids 0..16383), all 12-depth tables."""
    w = WORKLOADS["c2_mixed"]
    prim = oracle.sample_primaries(sampler(w), 0, 16384)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=C2_THRESHOLDS, max_steps=BIG_MAX_STEPS)
    t = time.time()
    r = oracle.run(cfg, prim, log=True)
    print("c2big oracle seconds", time.time() - t, r["stats"], flush=True)
    save("c2_accept", dict(name="c2_mixed", ids=[[0, 16384]], seed=0, max_steps=BIG_MAX_STEPS), r, lineage=True)


def c4big():
    """1,024 primaries of the 100 keV As channeling workload (ids 0..1023), 16 depths."""
    w = WORKLOADS["c4_as100kev"]
    prim = oracle.sample_primaries(sampler(w), 0, 1024)
    cfg = oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"],
                        thresholds=[list(C4_THRESHOLDS)], max_steps=BIG_MAX_STEPS)
    t = time.time()
    r = oracle.run(cfg, prim, log=True)
    print("c4big oracle seconds", time.time() - t, r["stats"], flush=True)
    save("c4_accept", dict(name="c4_as100kev", ids=[[0, 1024]], seed=0, max_steps=BIG_MAX_STEPS), r,
         lineage=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["c0", "c1"]
    for w in what:
        {"pilot": pilot, "pilot2": pilot2, "pilot4": pilot4, "pilot5": pilot5, "c0": c0, "c0fkbk": c0fkbk,
         "c1": c1, "c2": c2,
         "c4": c4, "c5": c5, "c5refine": c5refine, "refine": refine, "c1big": c1big, "c2big": c2big,
         "c4big": c4big}[w]()

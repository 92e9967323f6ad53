"""Writes the stored oracle results used by the GPU statistical parity tests.

Calls only the oracle (``oracle/``).  Usage:  python tests/golden/make_golden.py [pilot|c0|c1]
  pilot: unsplit survival quantiles of the 10 keV As workload (source of C1_THRESHOLDS)
  c0:    65,536 B at 1 keV, 7 degree tilt, no splitting (the c0 sampler, ids 0..65535)
  c1:    1,024 As at 10 keV with the 8 cloning depths: ids 0..511 (channel) and 32768..33279 (tilt)
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
from tests.workloads import C1_THRESHOLDS, WORKLOADS  # noqa: E402


def sampler(w):
    return oracle.SamplerCfg(**w["sampler"])


def save(name, cfg_desc, r, extra=None):
    st = r["stats"]
    log = r["log"]
    stopped = log[log["status"] == oracle.STOPPED]
    order = np.lexsort((stopped["w"], stopped["z_stop"]))
    z = stopped["z_stop"][order]
    w = stopped["w"][order]
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


def c0():
    w = WORKLOADS["c0_b1kev"]
    n = 65536
    prim = oracle.sample_primaries(sampler(w), 0, n)
    t = time.time()
    r = oracle.run(oracle.Config(species=w["species"], n_bins=w["n_bins"], bin_width=w["bin_width"]),
                   prim, log=True)
    print("c0 oracle seconds", time.time() - t, r["stats"])
    save("c0_accept", dict(name="c0_b1kev", n=n, seed=0, id0=0), r)


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


if __name__ == "__main__":
    what = sys.argv[1:] or ["c0", "c1"]
    for w in what:
        {"pilot": pilot, "c0": c0, "c1": c1}[w]()

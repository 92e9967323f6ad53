"""The synthetic implantation workloads (seeded; no method arithmetic here).

Shared by the tests, the smoke check and the benchmark: each workload is a
sampler description plus run settings, consumed separately by the oracle
(``oracle.SamplerCfg`` / ``oracle.Config``) and by the HIP library
(``paper_0810_4737_amd.SamplerConfig`` / ``RunConfig``).
"""
from __future__ import annotations

import math

SQ2 = 1.0 / math.sqrt(2.0)

# Cloning depths (A) for 10 keV As into Si with the 50/50 [110]-channel / 7-degree mix:
# the depths at which the unsplit survival probability is 2^-k, k = 1..8 (geometric in
# probability: with 2 clones per depth every interval then receives the same expected
# number of tracks, the paper's equal-count rule), read off an oracle pilot of 512
# unsplit primaries of the same sampler with seed 0 (tests/golden/make_golden.py, "pilot").
C1_THRESHOLDS = (197.0, 906.0, 1876.0, 2680.0, 3096.0, 3384.0, 3571.0, 3694.0)

WORKLOADS = {
    # 256 B at 1 keV, [100] surface, 7 degree tilt, uniform azimuth, no splitting, 1 A bins
    "c0_b1kev": dict(species=("B",), n=256, sampler=dict(choice=(0,), E_min=1000.0, E_max=1000.0,
                                                         dir_mode=0, tilt=math.radians(7.0)),
                     thresholds=None, n_bins=1024, bin_width=1.0),
    # 65,536 As at 10 keV: half within 0.5 degree of [110], half 7 degree tilt; 8 cloning depths
    "c1_as10kev": dict(species=("As",), n=65536,
                       sampler=dict(choice=(0,), E_min=10000.0, E_max=10000.0, dir_mode=2,
                                    n_cone=32768, half_angle=math.radians(0.5),
                                    axis=(0.0, SQ2, SQ2), tilt=math.radians(7.0)),
                       thresholds="c1", n_bins=8192, bin_width=1.0),
}

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

# Cloning-depth tables (A) of the mixed workload, one per (species, energy decade):
# [B 1-10 keV, B 10-100 keV, P 1-10, P 10-100, As 1-10, As 10-100]; 12 depths each at unsplit
# survival 10^(-5k/12), k = 1..12 (5 decades), from 256-primary oracle pilots per table with
# the exponential tail extrapolation of make_golden.survival_depths (pilot2).
C2_THRESHOLDS = (
    (228.1, 406.1, 599.4, 865.4, 1107.2, 1359.3, 1611.3, 1863.4, 2115.5, 2367.5, 2619.6, 2871.7),
    (2019.6, 3187.4, 4047.1, 4818.9, 5806.4, 6693.9, 7581.5, 8469.0, 9356.6, 10244.1, 11131.7, 12019.2),
    (101.1, 189.4, 317.8, 454.5, 580.1, 707.2, 834.3, 961.4, 1088.5, 1215.6, 1342.7, 1469.8),
    (689.1, 1263.5, 1585.6, 1979.0, 2416.3, 2820.8, 3225.2, 3629.7, 4034.1, 4438.6, 4843.0, 5247.5),
    (75.3, 128.3, 207.0, 253.3, 312.3, 368.1, 424.0, 479.8, 535.7, 591.6, 647.4, 703.3),
    (343.2, 589.7, 772.0, 1116.5, 1440.5, 1754.9, 2069.2, 2383.6, 2698.0, 3012.3, 3326.7, 3641.0),
)

# Cloning depths (A) of the 100 keV As [001] channeling workload: 16 depths at unsplit
# survival 10^(-6k/16), k = 1..16 (down to 1e-6), same procedure from a 128-primary pilot (pilot4).
C4_THRESHOLDS = (3613.4, 5090.6, 6132.5, 6481.5, 6911.2, 7315.8, 7720.5, 8125.1, 8529.7, 8934.3,
                 9338.9, 9743.6, 10148.2, 10552.8, 10957.4, 11362.0)

# Fluorite UO2 target (cations U, anions O); cubic constant and masses from the literature, the
# rms thermal displacements representative 300 K Debye-Waller amplitudes (Sec. 4 takes its
# values from MD runs it does not print).
UO2 = dict(a=5.470, Z2=92, M2=238.03, sigma=0.050, Z2b=8, M2b=15.999, sigma_b=0.067)

# Cloning distances (A from the start point) of the 85 keV U recoils in UO2: 8 distances at unsplit
# survival 2^-k, k = 1..8 (the paper uses eight cloning points for this case), from a 512-primary
# oracle pilot of the same sampler (pilot5).
C5_THRESHOLDS = (141.8, 203.7, 249.2, 302.1, 368.0, 428.2, 487.3, 546.9)

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
    # 1,048,576 tracks: species uniform over {B, P, As}, energy log-uniform 1-100 keV, 7 degree tilt;
    # 12 cloning depths per (species, energy decade) table; 1 A bins 0-8192 A
    "c2_mixed": dict(species=("B", "P", "As"), n=1048576,
                     sampler=dict(choice=(0, 1, 2), E_min=1000.0, E_max=100000.0, n_energy_tables=2,
                                  dir_mode=0, tilt=math.radians(7.0)),
                     thresholds="c2", n_bins=8192, bin_width=1.0),
    # 262,144 As at 100 keV exactly along [001] (0 degree tilt); 16 cloning depths down to 1e-6;
    # 0-500 nm in 0.5 nm bins
    "c4_as100kev": dict(species=("As",), n=262144,
                        sampler=dict(choice=(0,), E_min=100000.0, E_max=100000.0, dir_mode=0, tilt=0.0),
                        thresholds="c4", n_bins=1000, bin_width=5.0),
    # 5,120 U recoils at 85 keV in UO2 (a plutonium alpha-decay recoil, Sec. 4): each primary is the
    # U atom of the cation site at the origin of cell (0, 0, 200), 1,094 A below the surface, moving
    # in a uniformly random direction, its own site left empty; the range is the distance from the
    # start point; 8 cloning distances; 0.5 A bins over 0-1024 A
    "c5_u85kev_uo2": dict(species=("U",), n=5120, target=UO2,
                          sampler=dict(choice=(0,), E_min=85000.0, E_max=85000.0, dir_mode=3, start_mode=1,
                                       a=UO2["a"], z_start=200 * UO2["a"]),
                          thresholds="c5", n_bins=2048, bin_width=0.5, range_mode=1, vacancy=1),
}

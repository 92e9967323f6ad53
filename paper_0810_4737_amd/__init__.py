"""MI355X-native REED-MD ion-track engine (thin Python binding over libreedmd.so).

Every step of the track simulation runs in the HIP kernels of ``libreedmd.so``;
this module only marshals torch device tensors (PyTorch provides device memory
and streams) into the C ABI declared in ``include/reedmd.h``.  If the library
is missing, importing the binding's functions raises: there is no CPU path.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi
from ._abi import (ACTIVE, BACKSCATTERED, CANCELLED, DIAMOND, DIR_CONE, DIR_ISOTROPIC, DIR_MIXED,  # noqa: F401
                   DIR_TILT, FLUORITE, FORCE_FP32, FORCE_FP64, FORM_PERSISTENT, FORM_PLAIN, NONFINITE, NSLOT,
                   NSLOT_FLUORITE, POT_NONE, POT_ZBL, RANGE_DEPTH, RANGE_RADIAL, RECORD_WORDS,
                   RECORD_WORDS_FLUORITE, START_SITE, START_SURFACE, STEPCAP, STOP_FKBK, STOP_LOCAL,
                   STOP_OFF, STOP_UNIFORM, STOPPED)

SPECIES = {"B": (5, 10.81), "P": (15, 30.97), "As": (33, 74.92), "U": (92, 238.03)}
SILICON = dict(a=5.431, Z2=14, M2=28.0855, sigma=0.076)
# valence electron density of silicon (4 per atom, 8 atoms per cubic cell), electrons per A^3:
# the interstitial electron gas of the Brandt-Kitagawa term when every valence electron counts
SILICON_VALENCE_DENSITY = 32.0 / 5.431 ** 3
# Fluorite UO2 (cations U, anions O); rms thermal displacements are representative
# 300 K Debye-Waller amplitudes
UO2 = dict(a=5.470, Z2=92, M2=238.03, sigma=0.050, Z2b=8, M2b=15.999, sigma_b=0.067, structure=FLUORITE)


class ReedmdError(RuntimeError):
    pass


def _check(rc, ctx=None):
    if rc != 0:
        L = _abi.load()
        msg = L.reedmd_last_error(ctx).decode() if ctx is not None or rc != 0 else ""
        raise ReedmdError(f"reedmd status {rc}: {msg}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _on(stream):
    """Makes `stream` current while a call allocates its outputs, so that their zero fills are
    ordered before the launches on that stream (torch fills on the current stream)."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """One target crystal + interaction model on the current device."""

    def __init__(self, a=SILICON["a"], Z2=SILICON["Z2"], M2=SILICON["M2"], sigma=SILICON["sigma"],
                 pot_mode=POT_ZBL, s=1.0, stop_mode=STOP_LOCAL, k=1.0, structure=DIAMOND,
                 Z2b=0, M2b=0.0, sigma_b=0.0, n_e=0.0):
        L = _abi.load()
        self._lib = L
        lat = _abi.Lattice(a=a, M2=M2, sigma=sigma, Z2=Z2, structure=structure, M2b=M2b,
                           sigma_b=sigma_b, Z2b=Z2b)
        pot = _abi.Potential(mode=pot_mode, s=s)
        stp = _abi.Stopping(mode=stop_mode, k=k, n_e=n_e)
        h = C.c_void_p()
        rc = L.reedmd_create(C.byref(lat), C.byref(pot), C.byref(stp), C.byref(h))
        if rc != 0:
            raise ReedmdError(f"reedmd_create failed ({rc}): {L.reedmd_last_error(None).decode()}")
        self.handle = h
        self.a = a
        self.structure = structure
        self.record_words = RECORD_WORDS_FLUORITE if structure == FLUORITE else RECORD_WORDS

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.reedmd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cached_graphs(self):
        """Persistent-form pipelines kept as instantiated graphs (one per launch shape)."""
        return int(self._lib.reedmd_cached_graphs(self.handle))

    def check(self, rc):
        if rc != 0:
            raise ReedmdError(f"reedmd status {rc}: {self._lib.reedmd_last_error(self.handle).decode()}")


def species_table(names):
    st = _abi.Species()
    st.n_species = len(names)
    for i, nm in enumerate(names):
        Z, M = SPECIES[nm] if isinstance(nm, str) else nm
        st.Z1[i], st.M1[i] = Z, M
    return st


@dataclass
class RunConfig:
    dx_max: float = 0.05
    dt_max: float = 1.0
    E_stop: float = 5.0
    z_start: float = -3.0
    max_steps: int = 0
    seed: int = 0
    thresholds: object = None      # array [n_tables][n_thresh] or None
    n_clones: int = 2
    n_bins: int = 1024
    bin_width: float = 1.0
    form: int = FORM_PLAIN
    lanes_per_track: int = 0
    waves_per_cu: int = 0
    queue_capacity: int = 0
    force_precision: int = FORCE_FP64
    range_mode: int = RANGE_DEPTH
    vacancy: int = 0
    no_tail_handoff: int = 0
    # interaction set: 0 = the 27 cells, > 0 = cut-off radius (A), < 0 = the domain autotuner's choice
    r_cut: float = 0.0

    def struct(self, device, keep):
        p = _abi.RunParams()
        p.dx_max, p.dt_max, p.E_stop, p.z_start = self.dx_max, self.dt_max, self.E_stop, self.z_start
        p.max_steps, p.seed = int(self.max_steps), int(self.seed)
        if self.thresholds is not None and np.asarray(self.thresholds).size:
            thr = torch.as_tensor(np.atleast_2d(np.asarray(self.thresholds, np.float64)), device=device)
            keep.append(thr)
            p.n_tables, p.n_thresh = thr.shape
            p.thresholds = thr.data_ptr()
        p.n_clones, p.n_bins, p.bin_width = self.n_clones, self.n_bins, self.bin_width
        p.form, p.lanes_per_track = self.form, self.lanes_per_track
        p.waves_per_cu, p.queue_capacity = self.waves_per_cu, self.queue_capacity
        p.force_precision = self.force_precision
        p.range_mode, p.vacancy = self.range_mode, self.vacancy
        p.no_tail_handoff = self.no_tail_handoff
        p.r_cut = float(self.r_cut)
        return p


@dataclass
class SamplerConfig:
    choice: tuple = (0,)
    dir_mode: int = DIR_TILT
    n_energy_tables: int = 1
    E_min: float = 1000.0
    E_max: float = 1000.0
    tilt: float = math.radians(7.0)
    axis: tuple = (0.0, 0.0, 1.0)
    half_angle: float = 0.0
    n_cone: int = 0
    a: float = SILICON["a"]
    z_start: float = -3.0
    start_mode: int = START_SURFACE

    def struct(self):
        s = _abi.Sampler()
        s.n_choice = len(self.choice)
        for i, c in enumerate(self.choice):
            s.choice[i] = c
        s.dir_mode, s.n_energy_tables = self.dir_mode, self.n_energy_tables
        s.E_min, s.E_max, s.tilt = self.E_min, self.E_max, self.tilt
        for i in range(3):
            s.axis[i] = self.axis[i]
        s.half_angle, s.n_cone, s.a, s.z_start = self.half_angle, self.n_cone, self.a, self.z_start
        s.start_mode = self.start_mode
        return s


def empty_batch(n, device="cuda"):
    return dict(species=torch.zeros(n, dtype=torch.int32, device=device),
                energy=torch.zeros(n, dtype=torch.float64, device=device),
                pos=torch.zeros((3, n), dtype=torch.float64, device=device),
                dir=torch.zeros((3, n), dtype=torch.float64, device=device),
                key=torch.zeros(n, dtype=torch.int64, device=device),
                table=torch.zeros(n, dtype=torch.int32, device=device))


def _batch_struct(batch, id0=0):
    b = _abi.Batch()
    b.n = int(batch["energy"].shape[0])
    b.id0 = int(id0)
    for name in ("species", "energy", "pos", "dir", "key", "table"):
        t = batch[name]
        assert t.is_contiguous() and t.is_cuda, name
        setattr(b, name, t.data_ptr())
    return b


def batch_from_numpy(d, device="cuda"):
    """Uploads a host batch (e.g. one made by a test) into device tensors."""
    return dict(species=torch.as_tensor(np.ascontiguousarray(d["species"], np.int32), device=device),
                energy=torch.as_tensor(np.ascontiguousarray(d["E0"] if "E0" in d else d["energy"], np.float64), device=device),
                pos=torch.as_tensor(np.ascontiguousarray(d["pos"], np.float64), device=device),
                dir=torch.as_tensor(np.ascontiguousarray(d["dir"], np.float64), device=device),
                key=torch.as_tensor(np.ascontiguousarray(d["key"]).view(np.int64), device=device),
                table=torch.as_tensor(np.ascontiguousarray(d["table"], np.int32), device=device))


def sample_primaries(ctx: Context, sampler: SamplerConfig, seed: int, n: int, id0: int = 0,
                     device="cuda", stream=None):
    with _on(stream):
        batch = empty_batch(n, device)
    b = _batch_struct(batch, id0)
    s = sampler.struct()
    ctx.check(ctx._lib.reedmd_sample_primaries(ctx.handle, C.byref(s), int(seed), C.byref(b), _stream(stream)))
    return batch


def new_stats(device="cuda"):
    return torch.zeros(_abi.STATS_WORDS, dtype=torch.int64, device=device)


def parse_stats(stats: torch.Tensor):
    raw = stats.detach().cpu().numpy().astype(np.int64)
    out = {}
    i = 0
    for n in _abi.STATS_INT_A:
        out[n] = int(raw[i]); i += 1
    dbl = raw[i:i + len(_abi.STATS_DBL)].view(np.float64)
    for j, n in enumerate(_abi.STATS_DBL):
        out[n] = float(dbl[j])
    i += len(_abi.STATS_DBL)
    for n in _abi.STATS_INT_B:
        out[n] = int(raw[i]); i += 1
    return out


def run(ctx: Context, species, batch, cfg: RunConfig, hist=None, stats=None, id0=0, log_cap=0,
        cancel=None, stream=None):
    """Runs every primary of `batch` with all its clones; returns (hist, stats[, log])."""
    dev = batch["energy"].device
    keep = []
    log = None
    with _on(stream):
        # the depth tables are allocated on the launch stream, so their memory cannot be
        # handed to work on another stream while the kernel may still read them
        p = cfg.struct(dev, keep)
        if hist is None:
            hist = torch.zeros(cfg.n_bins, dtype=torch.float64, device=dev)
        if stats is None:
            stats = new_stats(dev)
        if log_cap > 0:
            log = torch.zeros((log_cap, _abi.RESULT_WORDS), dtype=torch.int64, device=dev)
            p.track_log = log.data_ptr()
            p.track_log_cap = log_cap
    if cancel is not None:
        p.cancel = cancel.data_ptr()
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch, id0)
    ctx.check(ctx._lib.reedmd_run(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), _ptr(hist), _ptr(stats),
                                  _stream(stream)))
    if log is not None:
        return hist, stats, log, keep
    return hist, stats, keep


def run_noalloc(ctx: Context, species, batch, cfg: RunConfig, hist, stats, thresholds=None, id0=0, stream=None):
    """The plain form through the library's allocation-free entry point, whose scratch memory is
    a static device array.  Every device buffer is the caller's: hist, stats, and the cloning
    depth tables as a float64 device tensor [n_tables, n_thresh] (cfg.thresholds must be None).
    Returns (hist, stats)."""
    if cfg.thresholds is not None:
        raise ReedmdError("give an allocation-free run its depth tables as the device tensor `thresholds`")
    p = cfg.struct(batch["energy"].device, [])
    if thresholds is not None:
        assert thresholds.is_cuda and thresholds.dtype == torch.float64 and thresholds.dim() == 2
        assert thresholds.is_contiguous()
        p.n_tables, p.n_thresh = thresholds.shape
        p.thresholds = thresholds.data_ptr()
    return _run_noalloc(ctx, species, batch, p, hist, stats, id0, stream)


def _run_noalloc(ctx, species, batch, p, hist, stats, id0, stream):
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch, id0)
    ctx.check(ctx._lib.reedmd_run_noalloc(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), _ptr(hist), _ptr(stats),
                                          _stream(stream)))
    return hist, stats


def run_refined(ctx: Context, species, batch, cfg: RunConfig, n_epochs: int, probs, min_gap: float = 1.0,
                hist=None, stats=None, id0=0, log_cap=0, stream=None, in_launch=False, snapshots=None,
                min_weight=1.0):
    """Runs the batch in n_epochs epochs with the cloning depths re-placed between epochs from
    the survival of the tracks booked so far (cfg.thresholds: the tables of epoch 0).
    in_launch: every epoch inside one persistent launch (epochs by claim position, each
    version placed from the caller's tables); snapshots: optional float64 device tensor
    [n_epochs, n_tables, n_bins + 2] that receives the statistics each version was placed from;
    min_weight: a target is placed only if target x booked weight (primaries' worth) reaches it.
    Returns (hist, stats, depths[n_epochs, n_tables, n_thresh][, log])."""
    dev = batch["energy"].device
    keep = []
    log = None
    with _on(stream):
        # the depth tables are allocated on the launch stream, so their memory cannot be
        # handed to work on another stream while the kernel may still read them
        p = cfg.struct(dev, keep)
        if hist is None:
            hist = torch.zeros(cfg.n_bins, dtype=torch.float64, device=dev)
        if stats is None:
            stats = new_stats(dev)
        if log_cap > 0:
            log = torch.zeros((log_cap, _abi.RESULT_WORDS), dtype=torch.int64, device=dev)
            p.track_log = log.data_ptr()
            p.track_log_cap = log_cap
    pr = np.ascontiguousarray(np.asarray(probs, dtype=np.float64))
    rf = _abi.Refine()
    rf.n_epochs = int(n_epochs)
    rf.probs = pr.ctypes.data_as(C.POINTER(C.c_double))
    rf.min_gap = float(min_gap)
    rf.in_launch = 1 if in_launch else 0
    rf.min_weight = float(min_weight)
    if snapshots is not None:
        E = max(1, min(int(n_epochs), int(batch["energy"].shape[0])))
        if snapshots.dtype != torch.float64 or not snapshots.is_contiguous() or \
                tuple(snapshots.shape) != (E, p.n_tables, p.n_bins + 2):
            raise ValueError("snapshots must be a contiguous float64 tensor [n_epochs, n_tables, n_bins + 2]")
        rf.snapshots = snapshots.data_ptr()
    with _on(stream):
        depths = torch.zeros((max(1, min(int(n_epochs), int(batch["energy"].shape[0]))), p.n_tables,
                              p.n_thresh), dtype=torch.float64, device=dev)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch, id0)
    ctx.check(ctx._lib.reedmd_run_refined(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), C.byref(rf),
                                          _ptr(hist), _ptr(stats), _ptr(depths), _stream(stream)))
    if log is not None:
        return hist, stats, depths, log
    return hist, stats, depths


def parse_log(log: torch.Tensor, count: int):
    raw = log[:count].detach().cpu().numpy()
    dt = np.dtype([("lineage", np.int64), ("status", np.int32), ("next_k", np.int32),
                   ("z_stop", np.float64), ("w", np.float64), ("steps", np.int64), ("key", np.uint64)])
    return raw.copy().view(dt).reshape(-1)


def track_init(ctx: Context, species, batch, cfg: RunConfig, id0=0, stream=None):
    dev = batch["energy"].device
    keep = []
    n = int(batch["energy"].shape[0])
    with _on(stream):
        p = cfg.struct(dev, keep)
        rec = torch.zeros((n, ctx.record_words), dtype=torch.float64, device=dev)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch, id0)
    ctx.check(ctx._lib.reedmd_track_init(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), _ptr(rec),
                                         _stream(stream)))
    return rec


def debug_step(ctx: Context, species, records: torch.Tensor, cfg: RunConfig, nsteps=1, stream=None):
    keep = []
    with _on(stream):
        p = cfg.struct(records.device, keep)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    assert records.is_contiguous() and records.dtype == torch.float64
    if records.dim() != 2 or records.shape[1] != ctx.record_words:
        raise ReedmdError(f"records must be [n, {ctx.record_words}] for this target")
    ctx.check(ctx._lib.reedmd_debug_step(ctx.handle, C.byref(sp), C.byref(p), _ptr(records),
                                         int(records.shape[0]), int(nsteps), _stream(stream)))
    return records


def autotune(ctx: Context, species, batch, cfg: RunConfig, pilot: int, stream=None):
    keep = []
    p = cfg.struct(batch["energy"].device, keep)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch)
    bl, bw = C.c_int32(), C.c_int32()
    ctx.check(ctx._lib.reedmd_autotune(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), int(pilot),
                                       _stream(stream), C.byref(bl), C.byref(bw)))
    return bl.value, bw.value


def autotune_domain(ctx: Context, species, batch, cfg: RunConfig, candidates=(0.0, 5.0, 6.0), pilot: int = 4096,
                    gate_p: float = 0.01, gate_rel: float = 0.01, stream=None):
    """Interaction-set autotuner: runs the pilot with the 27 cells and with each cut-off
    candidate, gates each (weighted KS p > gate_p, mean and std within gate_rel or three
    standard errors) and records the fastest passing one for cfg.r_cut < 0.  Returns
    (best r_cut, report rows (r_cut, ms, ks_p, rel mean diff, rel std diff, passed))."""
    keep = []
    p = cfg.struct(batch["energy"].device, keep)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch)
    nc = len(candidates)
    cand = (C.c_double * max(nc, 1))(*[float(c) for c in candidates])
    rep = (C.c_double * (5 * max(nc, 1)))()
    best = C.c_double()
    ctx.check(ctx._lib.reedmd_autotune_domain(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), cand, nc, int(pilot),
                                              float(gate_p), float(gate_rel), _stream(stream), C.byref(best), rep))
    rows = [(float(candidates[i]), rep[5 * i], rep[5 * i + 1], rep[5 * i + 2], rep[5 * i + 3], bool(rep[5 * i + 4]))
            for i in range(nc)]
    return best.value, rows


def launch_shape(ctx: Context, batch, cfg: RunConfig):
    """The launch shape run() would use: dict(lanes, blocks, segments, blocks_per_cu, queue)."""
    keep = []
    p = cfg.struct(batch["energy"].device, keep)
    b = _batch_struct(batch)
    out = (C.c_int64 * 5)()
    ctx.check(ctx._lib.reedmd_launch_shape(ctx.handle, C.byref(b), C.byref(p), out))
    return dict(lanes=out[0], blocks=out[1], segments=out[2], blocks_per_cu=out[3], queue=out[4])


def grad(ctx: Context, species, batch, cfg: RunConfig, k: float, s: float, per_track=False, stream=None):
    """Mean projected range and its derivatives w.r.t. the stopping scale k and the screening
    scale s (reverse mode, 64-step checkpoints).  Returns dict(mean, dk, ds, count[, tracks])."""
    keep = []
    p = cfg.struct(batch["energy"].device, keep)
    sp = species_table(species) if not isinstance(species, _abi.Species) else species
    b = _batch_struct(batch)
    res = (C.c_double * 4)()
    out = None
    if per_track:
        with _on(stream):
            out = torch.zeros((int(batch["energy"].shape[0]), 5), dtype=torch.float64,
                              device=batch["energy"].device)
    ctx.check(ctx._lib.reedmd_grad(ctx.handle, C.byref(sp), C.byref(b), C.byref(p), float(k), float(s),
                                   _ptr(out), res, _stream(stream)))
    d = dict(mean=res[0], dk=res[1], ds=res[2], count=int(res[3]))
    if per_track:
        d["tracks"] = out
    return d


class ReedMDRange(torch.autograd.Function):
    """R(k, s): mean projected range of a batch as a differentiable function of the
    electronic-stopping scale k and the ZBL screening-length scale s (0-d float64 tensors).
    forward runs the adjoint once and keeps both partial derivatives; backward scales them."""

    @staticmethod
    def forward(fctx, k, s, engine, species, batch, cfg):
        r = grad(engine, species, batch, cfg, float(k.detach().cpu()), float(s.detach().cpu()))
        fctx.save_for_backward(torch.tensor([r["dk"], r["ds"]], dtype=torch.float64, device=k.device))
        return torch.tensor(r["mean"], dtype=torch.float64, device=k.device)

    @staticmethod
    def backward(fctx, g):
        (d,) = fctx.saved_tensors
        return g * d[0], g * d[1], None, None, None, None


def eval_log(x: torch.Tensor, stream=None, one_plus=False):
    """The library's ln x (or ln(1 + x) with one_plus=True) on a float64 device tensor."""
    L = _abi.load()
    with _on(stream):
        x = x.contiguous()
        out = torch.empty_like(x)
    rc = L.reedmd_eval_log(_ptr(x), _ptr(out), int(x.numel()), 1 if one_plus else 0, _stream(stream))
    if rc != 0:
        raise ReedmdError(f"reedmd_eval_log failed ({rc})")
    return out


def eval_exp_neg(y: torch.Tensor, stream=None, pair=False):
    """The library's exp(-y) on a float64 device tensor: the friction factors' exponential, or
    with pair=True the one of the ion-atom pair terms."""
    L = _abi.load()
    with _on(stream):
        y = y.contiguous()
        out = torch.empty_like(y)
    fn = L.reedmd_eval_exp_neg_pair if pair else L.reedmd_eval_exp_neg
    rc = fn(_ptr(y), _ptr(out), int(y.numel()), _stream(stream))
    if rc != 0:
        raise ReedmdError(f"reedmd_eval_exp_neg failed ({rc})")
    return out

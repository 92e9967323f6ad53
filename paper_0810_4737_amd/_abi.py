"""ctypes mirror of include/reedmd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

MAX_SPECIES = 8
NSLOT = 216
RECORD_WORDS = 32 + 9 * NSLOT
NSLOT_FLUORITE = 344
RECORD_WORDS_FLUORITE = 32 + 9 * NSLOT_FLUORITE

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -5
DIAMOND, FLUORITE = 0, 1
RANGE_DEPTH, RANGE_RADIAL = 0, 1
START_SURFACE, START_SITE = 0, 1
POT_ZBL, POT_NONE = 0, 1
STOP_OFF, STOP_UNIFORM, STOP_LOCAL, STOP_FKBK = 0, 1, 2, 3
FORM_PLAIN, FORM_PERSISTENT = 0, 1
FORCE_FP64, FORCE_FP32 = 0, 1
DIR_TILT, DIR_CONE, DIR_MIXED, DIR_ISOTROPIC = 0, 1, 2, 3
ACTIVE, STOPPED, BACKSCATTERED, NONFINITE, STEPCAP, CANCELLED, LOST = range(7)

LIB_PATH = os.environ.get("REEDMD_LIBRARY") or \
    os.path.join(os.path.dirname(os.path.abspath(__file__)), "libreedmd.so")


class Lattice(C.Structure):
    _fields_ = [("a", C.c_double), ("M2", C.c_double), ("sigma", C.c_double),
                ("Z2", C.c_int32), ("structure", C.c_int32),
                ("M2b", C.c_double), ("sigma_b", C.c_double), ("Z2b", C.c_int32), ("reserved", C.c_int32)]


class Potential(C.Structure):
    _fields_ = [("mode", C.c_int32), ("reserved", C.c_int32), ("s", C.c_double)]


class Stopping(C.Structure):
    _fields_ = [("mode", C.c_int32), ("reserved", C.c_int32), ("k", C.c_double), ("n_e", C.c_double)]


class Species(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("reserved", C.c_int32),
                ("Z1", C.c_int32 * MAX_SPECIES), ("M1", C.c_double * MAX_SPECIES)]


class Batch(C.Structure):
    _fields_ = [("n", C.c_int64), ("id0", C.c_int64), ("species", C.c_void_p),
                ("energy", C.c_void_p), ("pos", C.c_void_p), ("dir", C.c_void_p),
                ("key", C.c_void_p), ("table", C.c_void_p)]


class Sampler(C.Structure):
    _fields_ = [("n_choice", C.c_int32), ("choice", C.c_int32 * MAX_SPECIES),
                ("dir_mode", C.c_int32), ("n_energy_tables", C.c_int32), ("start_mode", C.c_int32),
                ("E_min", C.c_double), ("E_max", C.c_double), ("tilt", C.c_double),
                ("axis", C.c_double * 3), ("half_angle", C.c_double), ("n_cone", C.c_int64),
                ("a", C.c_double), ("z_start", C.c_double)]


class RunParams(C.Structure):
    _fields_ = [("dx_max", C.c_double), ("dt_max", C.c_double), ("E_stop", C.c_double),
                ("z_start", C.c_double), ("max_steps", C.c_int64), ("seed", C.c_uint64),
                ("n_thresh", C.c_int32), ("n_tables", C.c_int32), ("thresholds", C.c_void_p),
                ("n_clones", C.c_int32), ("n_bins", C.c_int32), ("bin_width", C.c_double),
                ("form", C.c_int32), ("lanes_per_track", C.c_int32), ("waves_per_cu", C.c_int32),
                ("queue_capacity", C.c_int32), ("cancel", C.c_void_p), ("track_log", C.c_void_p),
                ("track_log_cap", C.c_int64), ("force_precision", C.c_int32), ("range_mode", C.c_int32),
                ("vacancy", C.c_int32), ("no_tail_handoff", C.c_int32), ("r_cut", C.c_double)]


class Refine(C.Structure):
    _fields_ = [("n_epochs", C.c_int32), ("in_launch", C.c_int32), ("probs", C.POINTER(C.c_double)),
                ("min_gap", C.c_double), ("snapshots", C.c_void_p), ("min_weight", C.c_double)]


class Result(C.Structure):
    _fields_ = [("lineage", C.c_int64), ("status", C.c_int32), ("next_k", C.c_int32),
                ("z_stop", C.c_double), ("w", C.c_double), ("steps", C.c_int64), ("key", C.c_uint64)]


RESULT_WORDS = 6   # 64-bit words per finished-track log entry


STATS_INT_A = ("primaries", "finished", "clones", "track_steps", "pair_evals", "n_stopped",
               "n_backscattered", "n_nonfinite", "n_stepcap", "n_cancelled")
STATS_DBL = ("w_stopped", "w_backscattered", "w_underflow", "w_overflow", "w_quarantined",
             "sum_wz", "sum_wz2", "w_cancelled")
STATS_INT_B = ("max_queue", "stack_overflow", "log_count", "error_flags", "handed_off")
STATS_WORDS = len(STATS_INT_A) + len(STATS_DBL) + len(STATS_INT_B)

# every entry point declared in include/reedmd.h
EXPORTS = ("reedmd_version", "reedmd_create", "reedmd_destroy", "reedmd_last_error",
           "reedmd_sample_primaries", "reedmd_run", "reedmd_track_init", "reedmd_debug_step",
           "reedmd_autotune", "reedmd_grad", "reedmd_eval_exp_neg", "reedmd_eval_exp_neg_pair", "reedmd_eval_log", "reedmd_launch_shape",
           "reedmd_run_refined", "reedmd_cached_graphs", "reedmd_run_noalloc", "reedmd_autotune_domain")

_lib = None


def load():
    """Loads the built HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"reedmd HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or paper_0810_4737_amd.build.build())")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    V = C.c_void_p
    L.reedmd_version.restype = C.c_int32
    L.reedmd_create.argtypes = [P(Lattice), P(Potential), P(Stopping), P(V)]
    L.reedmd_create.restype = C.c_int
    L.reedmd_destroy.argtypes = [V]
    L.reedmd_last_error.argtypes = [V]
    L.reedmd_last_error.restype = C.c_char_p
    L.reedmd_cached_graphs.argtypes = [V]
    L.reedmd_cached_graphs.restype = C.c_int32
    L.reedmd_sample_primaries.argtypes = [V, P(Sampler), C.c_uint64, P(Batch), V]
    L.reedmd_sample_primaries.restype = C.c_int
    L.reedmd_run.argtypes = [V, P(Species), P(Batch), P(RunParams), V, V, V]
    L.reedmd_run.restype = C.c_int
    L.reedmd_run_noalloc.argtypes = [V, P(Species), P(Batch), P(RunParams), V, V, V]
    L.reedmd_run_noalloc.restype = C.c_int
    L.reedmd_track_init.argtypes = [V, P(Species), P(Batch), P(RunParams), V, V]
    L.reedmd_track_init.restype = C.c_int
    L.reedmd_debug_step.argtypes = [V, P(Species), P(RunParams), V, C.c_int64, C.c_int32, V]
    L.reedmd_debug_step.restype = C.c_int
    L.reedmd_autotune.argtypes = [V, P(Species), P(Batch), P(RunParams), C.c_int64, V,
                                  P(C.c_int32), P(C.c_int32)]
    L.reedmd_autotune.restype = C.c_int
    L.reedmd_autotune_domain.argtypes = [V, P(Species), P(Batch), P(RunParams), P(C.c_double), C.c_int32, C.c_int64,
                                         C.c_double, C.c_double, V, P(C.c_double), P(C.c_double)]
    L.reedmd_autotune_domain.restype = C.c_int
    L.reedmd_grad.argtypes = [V, P(Species), P(Batch), P(RunParams), C.c_double, C.c_double, V,
                              P(C.c_double), V]
    L.reedmd_grad.restype = C.c_int
    L.reedmd_eval_exp_neg.argtypes = [V, V, C.c_int64, V]
    L.reedmd_eval_exp_neg.restype = C.c_int
    L.reedmd_eval_exp_neg_pair.argtypes = [V, V, C.c_int64, V]
    L.reedmd_eval_exp_neg_pair.restype = C.c_int
    L.reedmd_eval_log.argtypes = [V, V, C.c_int64, C.c_int32, V]
    L.reedmd_eval_log.restype = C.c_int
    L.reedmd_launch_shape.argtypes = [V, P(Batch), P(RunParams), P(C.c_int64)]
    L.reedmd_launch_shape.restype = C.c_int
    L.reedmd_run_refined.argtypes = [V, P(Species), P(Batch), P(RunParams), P(Refine), V, V, V, V]
    L.reedmd_run_refined.restype = C.c_int
    _lib = L
    return L

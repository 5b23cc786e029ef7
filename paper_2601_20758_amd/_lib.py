"""ctypes declarations of libsfkde (include/sfkde.h). Loads the in-tree
library built by paper_2601_20758_amd/build.py and fails loudly if it is
missing: there is no fallback implementation."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfkde.so")

# enums (include/sfkde.h)
SFK_OK = 0
# size of the static scratch array of sfk_eval_roi_noalloc (SFK_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20
# tile shapes sfk_eval_opts.tile_shape can name, 1..NUM_TILE_SHAPES (SFK_NUM_TILE_SHAPES)
NUM_TILE_SHAPES = 7
STATUS = {0: "SFK_OK", 1: "SFK_E_INVAL", 2: "SFK_E_NOMEM", 3: "SFK_E_BUDGET", 4: "SFK_E_DEVICE",
          5: "SFK_E_NOT_READY", 6: "SFK_E_CANCELLED", 7: "SFK_E_UNSUPPORTED", 8: "SFK_E_INTERNAL"}
KERNEL = {"epanechnikov": 0, "gauss_trunc3": 1}
BW = {"fixed": 0, "roi_scaled": 1, "per_point": 2, "mbe": 3}
NORM = {"paper": 0, "count": 1}
SET = {"cloud": 0, "in_roi": 1}


class Allocator(C.Structure):
    ALLOC = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
    FREE = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)
    _fields_ = [("alloc", ALLOC), ("free", FREE), ("user", C.c_void_p)]


class TreeOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("knn_k", C.c_int32), ("key_bits", C.c_int32),
                ("curve", C.c_int32)]


CURVES = {"hilbert": 0, "morton": 1}


class RoiC(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("res", C.c_int32 * 3),
                ("kernel", C.c_int32), ("bw", C.c_int32), ("norm", C.c_int32), ("set", C.c_int32),
                ("h", C.c_float * 3), ("d_out", C.c_void_p), ("tag", C.c_uint64)]


class EvalOpts(C.Structure):
    _fields_ = [("tile_shape", C.c_int32), ("chunk_leaves", C.c_int32),
                ("persistent_waves_per_cu", C.c_int32), ("list_capacity", C.c_int32),
                ("disable_graphs", C.c_int32), ("partial_capacity", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("roi", RoiC)]


class ServeOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("n_slots", C.c_int32), ("max_batch", C.c_int32),
                ("interleave", C.c_int32), ("budget_bytes", C.c_double),
                ("max_batch_work", C.c_double)]


class RequestResult(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double),
                ("latency_ms", C.c_double), ("batch", C.c_int32), ("status", C.c_int32)]


class ServeSummary(C.Structure):
    _fields_ = [("wall_s", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("max_ms", C.c_double), ("evals_per_s", C.c_double), ("n_batches", C.c_int64),
                ("mean_batch", C.c_double), ("mean_in_flight", C.c_double),
                ("budget_waits", C.c_int64)]


class Profile(C.Structure):
    _fields_ = [("tile_count_ms", C.c_double), ("plan_ms", C.c_double),
                ("tile_fill_ms", C.c_double), ("eval_ms", C.c_double), ("build_ms", C.c_double),
                ("knn_ms", C.c_double), ("eval_launches", C.c_int64), ("builds", C.c_int64),
                ("last_total_leaves", C.c_int64), ("last_items", C.c_int64)]


class ViewOpts(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("bw", C.c_int32), ("norm", C.c_int32), ("res", C.c_int32),
                ("h", C.c_float * 3), ("block", C.c_int32), ("scale_threshold", C.c_double),
                ("margin", C.c_double), ("max_blocks", C.c_int64)]


class ViewFrameInfo(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("g0", C.c_int64 * 3),
                ("res", C.c_int32 * 3), ("new_lattice", C.c_int32), ("spacing", C.c_double),
                ("lattice_id", C.c_int64), ("blocks_needed", C.c_int64),
                ("blocks_evaluated", C.c_int64)]


class Brick(C.Structure):
    _fields_ = [("level", C.c_int32), ("parent", C.c_int32), ("cell0", C.c_int32 * 3),
                ("res", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("offset", C.c_int64)]


class AdaptiveOpts(C.Structure):
    _fields_ = [("brick", C.c_int32), ("max_level", C.c_int32), ("threshold", C.c_float),
                ("reserved", C.c_int32)]


class AdaptiveResult(C.Structure):
    _fields_ = [("n_bricks", C.c_int32), ("levels", C.c_int32), ("complete", C.c_int32),
                ("peak", C.c_float), ("floats_used", C.c_int64)]


EXPORTS = {
    # name: (restype, argtypes)
    "sfk_version": (C.c_char_p, []),
    "sfk_status_string": (C.c_char_p, [C.c_int]),
    "sfk_last_error": (C.c_char_p, [C.c_void_p]),
    "sfk_ctx_create": (C.c_int, [C.c_int, C.POINTER(Allocator), C.c_size_t, C.POINTER(C.c_void_p)]),
    "sfk_ctx_destroy": (C.c_int, [C.c_void_p]),
    "sfk_build_tree": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.POINTER(TreeOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "sfk_tree_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                C.POINTER(C.c_size_t)]),
    "sfk_tree_destroy": (C.c_int, [C.c_void_p]),
    "sfk_eval_roi": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_void_p]),
    "sfk_eval_roi_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_void_p]),
    "sfk_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_int32,
                             C.POINTER(C.c_int64)]),
    "sfk_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]),
    "sfk_wait": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64]),
    "sfk_cancel": (C.c_int, [C.c_void_p, C.c_int64]),
    "sfk_set_eval_opts": (C.c_int, [C.c_void_p, C.POINTER(EvalOpts)]),
    "sfk_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_int32]),
    "sfk_autotune_table": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.c_int32, C.POINTER(C.c_int32)]),
    "sfk_autotune_costs": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.c_int32, C.POINTER(C.c_int32)]),
    "sfk_autotune_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "sfk_autotune_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "sfk_serve": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(Request), C.c_int64,
                            C.POINTER(ServeOpts), C.POINTER(RequestResult),
                            C.POINTER(ServeSummary)]),
    "sfk_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "sfk_profile_read": (C.c_int, [C.c_void_p, C.POINTER(Profile), C.c_int32]),
    "sfk_debug_candidates": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_int64,
                                       C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.POINTER(C.c_int64)]),
    "sfk_sample_density": (C.c_int, [C.c_void_p, C.POINTER(RoiC), C.c_void_p, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_void_p]),
    "sfk_select_points": (C.c_int, [C.c_void_p, C.POINTER(RoiC), C.c_void_p, C.c_double,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                    C.POINTER(C.c_int64), C.c_void_p]),
    "sfk_iso_cells": (C.c_int, [C.c_void_p, C.POINTER(RoiC), C.c_void_p, C.c_double, C.c_void_p,
                                C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_void_p]),
    "sfk_debug_mc_case": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(C.c_int32)]),
    "sfk_iso_surface": (C.c_int, [C.c_void_p, C.POINTER(RoiC), C.c_void_p, C.c_double,
                                  C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_void_p]),
    "sfk_view_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(ViewOpts),
                                  C.POINTER(C.c_void_p)]),
    "sfk_view_destroy": (C.c_int, [C.c_void_p]),
    "sfk_view_frame": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_void_p, C.c_int64, C.POINTER(ViewFrameInfo), C.c_void_p]),
    "sfk_eval_adaptive": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC),
                                    C.POINTER(AdaptiveOpts), C.c_void_p, C.c_int64,
                                    C.POINTER(Brick), C.c_int32, C.POINTER(AdaptiveResult),
                                    C.c_void_p]),
    "sfk_debug_point_h2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sfk_debug_poison": (C.c_int, [C.c_void_p, C.c_int32]),
    "sfk_debug_tile_leaves": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_void_p,
                                        C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sfk_debug_leaf_boxes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sfk_debug_tree_order": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sfk_debug_curve_keys": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
    "sfk_debug_particle_estimate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.POINTER(C.c_double)]),
    "sfk_debug_eval_count": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sfk_debug_support_counts": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_void_p,
                                           C.c_void_p]),
    "sfk_debug_mbe": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RoiC), C.c_void_p,
                                C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_double), C.c_void_p, C.c_int64]),
}

_LIB = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libsfkde.so is not built (%s); run `python paper_2601_20758_amd/build.py` "
                "or __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB

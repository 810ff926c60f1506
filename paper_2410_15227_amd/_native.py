"""Loader of the HIP library libsphmap.so and its C signatures.

The library is built in-tree by paper_2410_15227_amd.build (hipcc, gfx950).
There is no fallback: if the library is missing every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphmap.so")

OK, EINVAL, ENOMEM, EGEOM, EHIP, ERANGE = 0, -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED = 0, 1

# every symbol include/sphmap.h declares
EXPORTS = [
    "sphmap_version", "sphmap_create", "sphmap_destroy", "sphmap_last_error",
    "sphmap_tess_upload", "sphmap_tess_free", "sphmap_tess_cell_info",
    "map_particles_to_cells", "map_particles_to_cells_batch", "sphmap_pairs_info", "sphmap_pairs_export", "sphmap_pairs_free",
    "map_cells_to_particles", "build_pseudo_particles", "build_pseudo_particles_open", "select_underresolved",
    "interpolate_to_particles", "sphmap_sync_status", "sphmap_estimate_footprint",
    "sphmap_tess_build_voronoi", "sphmap_tess_counts", "sphmap_tess_export", "build_pseudo_particles_kd",
    "sphmap_tess_set_face_neighbours",
    "sphmap_set_timing", "sphmap_kernel_time", "sphmap_reset_timing",
    "sphmap_set_counting", "sphmap_work_counters", "sphmap_set_autotune", "sphmap_tuned_shape",
    "sphmap_set_pool_limit", "sphmap_set_workspace_limit", "sphmap_workspace_info",
    "interpolate_to_particles_noalloc", "sphmap_batch_create", "sphmap_batch_run", "sphmap_batch_check",
    "sphmap_batch_free",
]


class PseudoOpts(ctypes.Structure):
    _fields_ = [("r_part", ctypes.c_double), ("theta", ctypes.c_double), ("h_fact", ctypes.c_double),
                ("eps_h", ctypes.c_double), ("leaf_max", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("bypass_threshold", ctypes.c_int64)]


class PseudoStats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_units", ctypes.c_int64), ("n_pseudo", ctypes.c_int64),
                ("n_real", ctypes.c_int64), ("branch_count", ctypes.c_int64 * 4), ("s_root", ctypes.c_double)]


class KdOpts(ctypes.Structure):
    _fields_ = [("r_leaf", ctypes.c_double), ("leaf_split", ctypes.c_int32), ("up_levels", ctypes.c_int32),
                ("nf_threshold", ctypes.c_int64)]


class Footprint(ctypes.Structure):
    _fields_ = [("workspace", ctypes.c_size_t), ("pairs", ctypes.c_size_t), ("tessellation", ctypes.c_size_t)]


class SphmapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sphmap error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2410_15227_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.sphmap_version.restype = ctypes.c_int
        L.sphmap_version.argtypes = []
        L.sphmap_create.restype = ctypes.c_int
        L.sphmap_create.argtypes = [i32, ctypes.c_size_t, pp]
        L.sphmap_set_workspace_limit.restype = ctypes.c_int
        L.sphmap_set_workspace_limit.argtypes = [vp, ctypes.c_size_t]
        L.sphmap_workspace_info.restype = ctypes.c_int
        L.sphmap_workspace_info.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                            ctypes.POINTER(ctypes.c_size_t)]
        L.sphmap_destroy.restype = ctypes.c_int
        L.sphmap_destroy.argtypes = [vp]
        L.sphmap_last_error.restype = ctypes.c_char_p
        L.sphmap_last_error.argtypes = [vp]
        L.sphmap_tess_upload.restype = ctypes.c_int
        L.sphmap_tess_upload.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, vp, vp, pp]
        L.sphmap_tess_free.restype = ctypes.c_int
        L.sphmap_tess_free.argtypes = [vp, vp]
        L.sphmap_tess_set_face_neighbours.restype = ctypes.c_int
        L.sphmap_tess_set_face_neighbours.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i64)]
        L.sphmap_tess_cell_info.restype = ctypes.c_int
        L.sphmap_tess_cell_info.argtypes = [vp, vp, vp, vp, vp]
        L.map_particles_to_cells.restype = ctypes.c_int
        L.map_particles_to_cells.argtypes = [vp, vp, i64, vp, vp, vp, i32, i32, vp, vp, vp, vp, pp]
        L.map_particles_to_cells_batch.restype = ctypes.c_int
        L.map_particles_to_cells_batch.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.sphmap_set_autotune.restype = ctypes.c_int
        L.sphmap_set_autotune.argtypes = [vp, i32]
        L.sphmap_tuned_shape.restype = ctypes.c_int
        L.sphmap_tuned_shape.argtypes = [vp, i64, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                         ctypes.POINTER(ctypes.c_double)]
        L.sphmap_pairs_info.restype = ctypes.c_int
        L.sphmap_pairs_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.sphmap_pairs_export.restype = ctypes.c_int
        L.sphmap_pairs_export.argtypes = [vp, vp, vp, vp, vp, vp]
        L.sphmap_pairs_free.restype = ctypes.c_int
        L.sphmap_pairs_free.argtypes = [vp, vp]
        L.sphmap_set_pool_limit.restype = ctypes.c_int
        L.sphmap_set_pool_limit.argtypes = [vp, ctypes.c_uint64]
        L.map_cells_to_particles.restype = ctypes.c_int
        L.map_cells_to_particles.argtypes = [vp, vp, i64, vp, vp, i32, vp, vp, i32, vp, vp]
        L.build_pseudo_particles_open.restype = ctypes.c_int
        L.build_pseudo_particles_open.argtypes = [vp, i64, vp, vp, vp, i32, vp, ctypes.POINTER(PseudoOpts), i64, vp,
                                                  i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64),
                                                  ctypes.POINTER(PseudoStats), vp]
        L.select_underresolved.restype = ctypes.c_int
        L.select_underresolved.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp,
                                           ctypes.POINTER(i64), vp]
        L.build_pseudo_particles_kd.restype = ctypes.c_int
        L.build_pseudo_particles_kd.argtypes = ([vp, i64, vp, vp, vp, i32, vp, ctypes.POINTER(PseudoOpts),
                                                 ctypes.POINTER(KdOpts), i64, vp, i64] + [vp] * 11
                                                + [ctypes.POINTER(i64), ctypes.POINTER(PseudoStats),
                                                   ctypes.POINTER(i32), vp])
        L.sphmap_tess_build_voronoi.restype = ctypes.c_int
        L.sphmap_tess_build_voronoi.argtypes = [vp, i64, vp, vp, vp, i32, vp, vp, ctypes.POINTER(vp)]
        L.sphmap_tess_counts.restype = ctypes.c_int
        L.sphmap_tess_counts.argtypes = [vp] + [ctypes.POINTER(i64)] * 4
        L.sphmap_tess_export.restype = ctypes.c_int
        L.sphmap_tess_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.sphmap_sync_status.restype = ctypes.c_int
        L.sphmap_sync_status.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.sphmap_estimate_footprint.restype = ctypes.c_int
        L.sphmap_estimate_footprint.argtypes = [vp, i64, i64, i64, i64, i64, i64, ctypes.POINTER(Footprint)]
        L.interpolate_to_particles.restype = ctypes.c_int
        L.interpolate_to_particles.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, i32, vp, vp]
        L.sphmap_batch_create.restype = ctypes.c_int
        L.sphmap_batch_create.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, dbl, vp, pp]
        L.sphmap_batch_run.restype = ctypes.c_int
        L.sphmap_batch_run.argtypes = [vp, vp, vp]
        L.sphmap_batch_check.restype = ctypes.c_int
        L.sphmap_batch_check.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i32)]
        L.sphmap_batch_free.restype = ctypes.c_int
        L.sphmap_batch_free.argtypes = [vp, vp]
        L.interpolate_to_particles_noalloc.restype = ctypes.c_int
        L.interpolate_to_particles_noalloc.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, vp, i32, vp, vp]
        L.build_pseudo_particles.restype = ctypes.c_int
        L.build_pseudo_particles.argtypes = [vp, i64, vp, vp, vp, i32, vp, ctypes.POINTER(PseudoOpts), i64,
                                             vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64),
                                             ctypes.POINTER(PseudoStats), vp]
        L.sphmap_set_timing.restype = ctypes.c_int
        L.sphmap_set_timing.argtypes = [vp, i32]
        L.sphmap_kernel_time.restype = ctypes.c_int
        L.sphmap_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.sphmap_reset_timing.restype = ctypes.c_int
        L.sphmap_reset_timing.argtypes = [vp]
        L.sphmap_set_counting.restype = ctypes.c_int
        L.sphmap_set_counting.argtypes = [vp, i32]
        L.sphmap_work_counters.restype = ctypes.c_int
        L.sphmap_work_counters.argtypes = [vp, ctypes.POINTER(i64)]
        _lib = L
    return _lib


def check(rc: int, ctx_handle=None):
    if rc != OK:
        msg = ""
        if ctx_handle is not None:
            msg = lib().sphmap_last_error(ctx_handle).decode(errors="replace")
        raise SphmapError(rc, msg)

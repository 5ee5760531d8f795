"""ctypes view of libusv.so (the C ABI in include/usv.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libusv.so")

USV_OK, USV_E_ARG, USV_E_OOM, USV_E_DEVICE, USV_E_STATE, USV_E_COUNT_OVERFLOW, USV_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "USV_OK", -1: "USV_E_ARG", -2: "USV_E_OOM", -3: "USV_E_DEVICE", -4: "USV_E_STATE",
                -5: "USV_E_COUNT_OVERFLOW", -6: "USV_E_UNSUPPORTED"}

# every entry point declared in include/usv.h
EXPORTS = [
    "usv_accumulator_bytes", "usv_create_volume", "usv_add_probe", "usv_reset", "usv_sync",
    "usv_export_accumulators", "usv_import_accumulators", "usv_destroy_volume", "usv_last_error",
    "usv_ingest_frames", "usv_ingest_frames_cut", "usv_set_ingest_overlap", "usv_join", "usv_cut_rows_alg1", "usv_cut_rows_alg2", "usv_vnn_create", "usv_vnn_reset", "usv_vnn_ingest",
    "usv_vnn_finalize", "usv_vnn_destroy", "usv_extract_slices", "usv_finalize", "usv_segment_project", "usv_segment_project_noalloc", "usv_ingest_batched", "usv_autotune",
    "usv_probe_tiling", "usv_probe_chunk", "usv_probe_set_tiling", "usv_graph_create", "usv_graph_launch",
    "usv_graph_destroy", "usv_pipeline_create", "usv_pipeline_push", "usv_pipeline_flush", "usv_pipeline_stats",
    "usv_pipeline_destroy", "usv_splat_create", "usv_splat_destroy", "usv_splat_forward", "usv_overlap_loss",
    "usv_splat_backward", "usv_dw_clear", "usv_dw_ingest", "usv_dw_finalize", "usv_refine_motion", "usv_fold_pose", "usv_dirty_box", "usv_version",
]


class Box(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]

    def as_tuple(self):
        return tuple(self.lo), tuple(self.hi)

    @property
    def empty(self):
        return any(self.lo[a] >= self.hi[a] for a in range(3))


class GridDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("origin_mm", C.c_double * 3), ("voxel_mm", C.c_double),
                ("fill_min", C.c_int32)]


class ProbeDesc(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pixel_mm", C.c_double * 2),
                ("calib", C.c_double * 16), ("mask_host", C.c_void_p)]


class SegParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("y_lo", C.c_int32), ("k", C.c_int32), ("tau_I", C.c_int32),
                ("tau_G", C.c_int32), ("r", C.c_int32), ("fallback_y", C.c_int32), ("n_half", C.c_int32),
                ("half", C.c_int32 * 4), ("K", C.c_double), ("D_mm", C.c_double), ("L_mm", C.c_double),
                ("z1_mm", C.c_double), ("yref_mm", C.c_double)]


class CutParams(C.Structure):
    _fields_ = [("half_rows", C.c_int32), ("axis", C.c_int32), ("K", C.c_double), ("D_mm", C.c_double),
                ("L_mm", C.c_double), ("z1_mm", C.c_double), ("y_lo", C.c_int32), ("k", C.c_int32),
                ("tau_I", C.c_int32), ("tau_G", C.c_int32), ("r", C.c_int32), ("fallback_row", C.c_int32)]


class RefineParams(C.Structure):
    _fields_ = [("iters", C.c_int32), ("lr_rho", C.c_double), ("lr_omega", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double)]


class UsvError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s%s" % (STATUS_NAMES.get(status, str(status)), (": " + msg) if msg else ""))


_lib = None


def lib():
    """Load libusv.so; fail loudly when it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libusv.so not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(or python paper_2412_00058_amd/build.py)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    PP = C.POINTER(C.c_void_p)
    sig = {
        "usv_accumulator_bytes": (C.c_size_t, [C.POINTER(GridDesc)]),
        "usv_create_volume": (I32, [C.POINTER(GridDesc), P, P, PP]),
        "usv_add_probe": (I32, [P, C.POINTER(ProbeDesc), C.POINTER(I32)]),
        "usv_reset": (I32, [P]),
        "usv_sync": (I32, [P]),
        "usv_export_accumulators": (I32, [P, P]),
        "usv_import_accumulators": (I32, [P, P]),
        "usv_destroy_volume": (I32, [P]),
        "usv_last_error": (C.c_char_p, [P]),
        "usv_ingest_frames": (I32, [P, I32, P, I64, I64, P, I32, C.POINTER(Box)]),
        "usv_set_ingest_overlap": (I32, [P, I32]),
        "usv_join": (I32, [P]),
        "usv_ingest_frames_cut": (I32, [P, I32, P, I64, I64, P, P, I32, C.POINTER(Box)]),
        "usv_cut_rows_alg1": (I32, [C.POINTER(ProbeDesc), P, I32, C.POINTER(CutParams), P]),
        "usv_extract_slices": (I32, [P, C.POINTER(C.c_int32 * 3), I32, I32, I32, P, P]),
        "usv_vnn_create": (I32, [C.POINTER(GridDesc), C.POINTER(ProbeDesc), D, P, P, PP]),
        "usv_vnn_reset": (I32, [P]),
        "usv_vnn_ingest": (I32, [P, P, I64, I64, P, I32]),
        "usv_vnn_finalize": (I32, [P, P, P]),
        "usv_vnn_destroy": (I32, [P]),
        "usv_cut_rows_alg2": (I32, [P, I64, I64, I32, I32, I32, C.POINTER(CutParams), P, P, P]),
        "usv_finalize": (I32, [P, C.POINTER(Box), P, P]),
        "usv_segment_project": (I32, [P, C.POINTER(SegParams), P, P, P, P, P]),
        "usv_segment_project_noalloc": (I32, [C.POINTER(GridDesc), C.POINTER(SegParams), P, P, P, P, P, P]),
        "usv_ingest_batched": (I32, [P, P, P, P, P, P, P, I32, P]),
        "usv_autotune": (I32, [P, I32, P, I64, I64, P, I32, C.c_char_p]),
        "usv_probe_tiling": (I32, [P, I32, C.POINTER(I32), C.POINTER(I32)]),
        "usv_probe_chunk": (I32, [P, I32, C.POINTER(I32)]),
        "usv_probe_set_tiling": (I32, [P, I32, I32, I32]),
        "usv_graph_create": (I32, [P, I32, PP]),
        "usv_graph_launch": (I32, [P, P, P, C.POINTER(Box)]),
        "usv_graph_destroy": (I32, [P]),
        "usv_pipeline_create": (I32, [P, I32, P, I32, P, P, P, P, P, PP]),
        "usv_pipeline_push": (I32, [P, P, P]),
        "usv_pipeline_flush": (I32, [P]),
        "usv_pipeline_stats": (I32, [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "usv_pipeline_destroy": (I32, [P]),
        "usv_splat_create": (I32, [C.POINTER(GridDesc), I32, I32, D, D, I32, P, PP]),
        "usv_splat_destroy": (I32, [P]),
        "usv_splat_forward": (I32, [P, P, P, P, I32, P]),
        "usv_overlap_loss": (I32, [P, P, P, P]),
        "usv_splat_backward": (I32, [P, P, P, P, I32, P, P, P]),
        "usv_dw_clear": (I32, [P, P]),
        "usv_dw_ingest": (I32, [P, P, I64, I64, P, I32, P]),
        "usv_dw_finalize": (I32, [P, P, C.c_float, P, P]),
        "usv_refine_motion": (I32, [P, P, P, I32, C.POINTER(RefineParams), P, P, P, P]),
        "usv_fold_pose": (I32, [C.POINTER(GridDesc), C.POINTER(ProbeDesc), P, P]),
        "usv_dirty_box": (I32, [C.POINTER(GridDesc), C.POINTER(ProbeDesc), P, I32, C.POINTER(Box)]),
        "usv_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status, handle=None):
    if status != USV_OK:
        msg = ""
        if handle is not None:
            try:
                msg = lib().usv_last_error(handle).decode()
            except Exception:
                msg = ""
        raise UsvError(status, msg)

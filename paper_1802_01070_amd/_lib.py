"""ctypes binding of libpct.so (the C ABI declared in include/pct.h).

Argument marshalling only: every step of the reconstruction path runs in the
HIP kernels of libpct.  Device memory and streams come from PyTorch.  There is
no fallback: if the library is missing or the GPU is absent, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpct.so")

PCT_OK = 0
PCT_F32, PCT_F64 = 0, 1
CHORDS = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
PCT_DROP_CHECK_FINITE = 0x1
PCT_DROP_NO_GRAPH = 0x2
PCT_DROP_PROFILE = 0x4
PCT_DROP_SEPARATE_COMMIT = 0x8
PCT_DROP_NO_TRACE_AHEAD = 0x10
PCT_DROP_FUSED_COMMIT = 0x20
PCT_DROP_NO_COMPENSATION = 0x40
PCT_DROP_CANCELLABLE = 0x80
PCT_DROP_DETERMINISTIC = 0x100
PCT_ERR_CANCELLED = -8
DEV_BITS = {0x1: "row_overflow", 0x2: "nonfinite", 0x4: "reentry", 0x8: "acc_range", 0x10: "bad_row",
            0x20: "cancelled"}
FIELDS = ("t_in", "v_in", "th_in", "ph_in", "t_out", "v_out", "th_out", "ph_out", "gantry")

EXPORTS = ("pct_plan_create", "pct_plan_destroy", "pct_plan_segments", "pct_plan_table", "pct_workspace_size",
           "pct_plan_upload", "pct_device_status", "pct_mlp_trace", "pct_forward", "pct_backproject",
           "pct_drop_iterate", "pct_tv", "pct_tv_static", "pct_status_string", "pct_last_hip_error", "pct_profile_read",
           "pct_region_layout", "pct_plan_region", "pct_region_select", "pct_select_slices",
           "pct_slice_span_histogram", "pct_rows_count", "pct_rows_build", "pct_drop_iterate_rows",
           "pct_order_blocks", "pct_plan_set_hull", "pct_fbp_workspace_size", "pct_fbp_sinogram", "pct_fbp_filter",
           "pct_fbp_backproject", "pct_fbp", "pct_sort_scan_workspace_size", "pct_sort_scan", "pct_drop_cancel",
           "pct_drop_progress")


class PctError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class pct_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("pitch", C.c_double * 3), ("origin", C.c_double * 3)]


class pct_mlp(C.Structure):
    _fields_ = [("u_in", C.c_double), ("u_out", C.c_double), ("step", C.c_double), ("poly", C.c_double * 6),
                ("E0", C.c_double), ("X0", C.c_double), ("log_term", C.c_int32)]


class pct_protons(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in FIELDS] + [("n", C.c_int64)]


class pct_hull(C.Structure):
    _fields_ = [("cx", C.c_double), ("cy", C.c_double), ("radius", C.c_double)]


class pct_protons_buf(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in FIELDS] + [("capacity", C.c_int64)]


class pct_rows(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("vox", C.c_void_p), ("chord", C.c_void_p), ("n2", C.c_void_p),
                ("n", C.c_int64), ("chord_type", C.c_int32), ("reserved", C.c_int32)]


class pct_fbp_geom(C.Structure):
    _fields_ = [("n_angles", C.c_int32), ("n_t", C.c_int32), ("t0", C.c_double), ("dt", C.c_double)]


class pct_sort_opts(C.Structure):
    _fields_ = [("n_angles", C.c_int32), ("reserved", C.c_int32), ("slab_mm", C.c_double)]


class pct_drop_opts(C.Structure):
    _fields_ = [("block", C.c_int64), ("lambda_", C.c_double), ("n_iter", C.c_int32), ("dtype", C.c_int32),
                ("chord", C.c_int32), ("flags", C.c_uint32), ("block_begin", C.c_int64),
                ("block_end", C.c_int64), ("lanes", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python paper_1802_01070_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, vp, i32, i64, sz = C.POINTER, C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "pct_plan_create": ([P(pct_grid), P(pct_mlp), P(vp)], C.c_int),
            "pct_plan_destroy": ([vp], None),
            "pct_plan_segments": ([vp, P(i32)], C.c_int),
            "pct_plan_table": ([vp, P(C.c_double), i64], C.c_int),
            "pct_workspace_size": ([vp, i64, i32, P(sz)], C.c_int),
            "pct_plan_upload": ([vp, vp, sz, vp], C.c_int),
            "pct_device_status": ([vp, vp, sz, C.c_int, P(C.c_uint32), vp], C.c_int),
            "pct_mlp_trace": ([vp, P(pct_protons), i64, i64, i32, vp, vp, vp, vp, sz, vp], C.c_int),
            "pct_forward": ([vp, P(pct_protons), vp, i32, vp, vp, vp, sz, vp], C.c_int),
            "pct_backproject": ([vp, P(pct_protons), vp, i32, vp, vp, sz, vp], C.c_int),
            "pct_drop_iterate": ([vp, P(pct_protons), vp, vp, P(pct_drop_opts), vp, sz, vp], C.c_int),
            "pct_drop_cancel": ([vp, vp, sz, i32], C.c_int),
            "pct_drop_progress": ([vp, vp, sz, P(i64), vp], C.c_int),
            "pct_tv": ([vp, vp, i32, C.c_double, vp, vp, vp, sz, vp], C.c_int),
            "pct_tv_static": ([vp, vp, i32, C.c_double, vp, vp, vp], C.c_int),
            "pct_status_string": ([C.c_int], C.c_char_p),
            "pct_last_hip_error": ([], C.c_int),
            "pct_profile_read": ([vp, P(C.c_double), P(i64)], C.c_int),
            "pct_region_layout": ([i32, i32, i32, P(i32), P(i32), P(i32), P(i32)], C.c_int),
            "pct_plan_region": ([vp, i32, i32, P(vp)], C.c_int),
            "pct_region_select": ([vp, P(pct_protons), vp, i32, i32, P(pct_protons_buf), vp, vp, vp, sz, vp],
                                  C.c_int),
            "pct_select_slices": ([vp, vp, i32, vp, i32, i32, i32, i32, vp], C.c_int),
            "pct_slice_span_histogram": ([vp, P(pct_protons), vp, vp, sz, vp], C.c_int),
            "pct_rows_count": ([vp, P(pct_protons), vp, vp, sz, vp], C.c_int),
            "pct_order_blocks": ([vp, P(pct_protons), vp, i64, P(pct_protons_buf), vp, vp], C.c_int),
            "pct_plan_set_hull": ([vp, P(pct_hull)], C.c_int),
            "pct_rows_build": ([vp, P(pct_protons), i32, vp, vp, vp, vp, vp, sz, vp], C.c_int),
            "pct_drop_iterate_rows": ([vp, P(pct_rows), vp, vp, P(pct_drop_opts), vp, sz, vp], C.c_int),
            "pct_fbp_workspace_size": ([vp, P(pct_fbp_geom), P(sz)], C.c_int),
            "pct_fbp_sinogram": ([vp, P(pct_fbp_geom), P(pct_protons), vp, vp, vp, vp, sz, vp], C.c_int),
            "pct_fbp_filter": ([vp, P(pct_fbp_geom), vp, vp, vp], C.c_int),
            "pct_fbp_backproject": ([vp, P(pct_fbp_geom), vp, vp, i32, vp], C.c_int),
            "pct_fbp": ([vp, P(pct_fbp_geom), P(pct_protons), vp, vp, i32, vp, sz, vp], C.c_int),
            "pct_sort_scan_workspace_size": ([i64, P(sz)], C.c_int),
            "pct_sort_scan": ([vp, P(pct_protons), vp, P(pct_sort_opts), P(pct_protons_buf), vp, vp, vp, sz, vp],
                              C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().pct_status_string(int(st)).decode()


def check(st: int, what: str):
    if st != PCT_OK:
        raise PctError(st, what)


def make_grid(grid) -> pct_grid:
    return pct_grid(int(grid.nx), int(grid.ny), int(grid.nz), (C.c_double * 3)(*map(float, grid.pitch)),
                    (C.c_double * 3)(*map(float, grid.origin)))


def make_mlp(mlp) -> pct_mlp:
    return pct_mlp(float(mlp.u_in), float(mlp.u_out), float(mlp.step), (C.c_double * 6)(*map(float, mlp.poly)),
                   float(mlp.E0), float(mlp.X0), int(mlp.log_term))


def make_protons(ptrs: dict, n: int) -> pct_protons:
    """ptrs: field -> device address (int)."""
    return pct_protons(*[C.c_void_p(int(ptrs[k])) for k in FIELDS], int(n))


def make_protons_buf(ptrs: dict, capacity: int) -> pct_protons_buf:
    return pct_protons_buf(*[C.c_void_p(int(ptrs[k])) for k in FIELDS], int(capacity))


def make_opts(block: int, lam: float, n_iter: int, dtype: int, chord: str = "f64", flags: int = 0,
              block_begin: int = 0, block_end: int = -1, lanes: int = 0) -> pct_drop_opts:
    return pct_drop_opts(int(block), float(lam), int(n_iter), int(dtype), CHORDS[chord], int(flags),
                         int(block_begin), int(block_end), int(lanes), 0)

"""ctypes binding of librgcsr.so (the C ABI in include/rgcsr.h).

Argument marshalling only: every function here has the name of the C entry
point it calls and does no arithmetic of its own.  The library must have been
built (``__graft_entry__.build()`` or ``python -m paper_1012_2270_amd.build``);
there is no fallback, a missing library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librgcsr.so")

RGCSR_F64, RGCSR_F32, RGCSR_F16, RGCSR_BF16 = 0, 1, 2, 3
STATUS = {0: "RGCSR_OK", 1: "RGCSR_EINVAL", 2: "RGCSR_ECSR", 3: "RGCSR_ENOMEM",
          4: "RGCSR_EOVERFLOW", 5: "RGCSR_EHIP", 6: "RGCSR_EUNSUPPORTED"}

c_i64, c_i32, c_vp, c_int = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int
P_I64 = ctypes.POINTER(ctypes.c_int64)
P_I32 = ctypes.POINTER(ctypes.c_int32)


class Opts(ctypes.Structure):
    _fields_ = [("group_size", c_i32), ("lanes_per_row", c_i32), ("sort_window", c_i64),
                ("long_row_threshold", c_i64), ("value_dtype", c_i32), ("keep_csr_map", c_i32),
                ("build_transpose", c_i32), ("validate", c_i32), ("rows_per_lane", c_i32),
                ("pad_loads", c_i32), ("load_policy", c_i32), ("tile_min_len", c_i32),
                ("col_panels", c_i32)]


class Info(ctypes.Structure):
    _fields_ = [("n_rows", c_i64), ("n_cols", c_i64), ("nnz", c_i64), ("n_groups", c_i64),
                ("n_short", c_i64), ("n_long", c_i64), ("slots", c_i64), ("long_nnz", c_i64),
                ("n_matrices", c_i64), ("long_work", c_i64), ("partials", c_i64),
                ("group_size", c_i32), ("lanes_per_row", c_i32), ("value_dtype", c_i32),
                ("has_transpose", c_i32), ("sort_window", c_i64), ("long_row_threshold", c_i64),
                ("device_bytes", c_i64), ("rows_per_lane", c_i32), ("pad_loads", c_i32),
                ("load_policy", c_i32), ("tiled_rows", c_i64), ("tile_entries", c_i64), ("n_tiles", c_i64),
                ("col_panels", c_i64), ("panel_pieces", c_i64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class HybInfo(ctypes.Structure):
    _fields_ = [("n_rows", c_i64), ("n_cols", c_i64), ("nnz", c_i64), ("n_pad", c_i64),
                ("ell_width", c_i64), ("coo_nnz", c_i64), ("device_bytes", c_i64),
                ("value_dtype", c_i32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class CGStats(ctypes.Structure):
    _fields_ = [("outer_iterations", c_i32), ("inner_iterations", c_i32), ("relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("converged", c_i32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


# name -> (restype, argtypes); the ABI contract as seen from Python
SIGNATURES = {
    "rgcsr_default_opts": (None, [ctypes.POINTER(Opts)]),
    "rgcsr_layout_sizes": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]),
    "rgcsr_panel_sizes": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, ctypes.POINTER(Opts), c_vp, P_I64, P_I64, P_I64,
                                  P_I64, P_I64]),
    "rgcsr_tile_sizes": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, ctypes.POINTER(Opts), P_I64, P_I64, P_I64, P_I64,
                                 P_I64]),
    "rgcsr_layout_host": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts),
                                  c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rgcsr_from_csr": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts), c_int,
                               c_vp, ctypes.POINTER(c_vp)]),
    "rgcsr_plan_from_csr": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts),
                                    ctypes.POINTER(c_vp)]),
    "rgcsr_plan_device_bytes": (c_int, [c_vp, P_I64]),
    "rgcsr_build": (c_int, [c_vp, c_vp, c_i64, c_vp, ctypes.POINTER(c_vp)]),
    "rgcsr_plan_destroy": (c_int, [c_vp]),
    "rgcsr_plan_from_csr_batch": (c_int, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts), c_vp]),
    "rgcsr_from_csr_batch": (c_int, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts), c_vp,
                                     ctypes.POINTER(c_vp)]),
    "rgcsr_batch_offsets": (c_int, [c_vp, c_vp, c_vp]),
    "rgcsr_spmv": (c_int, [c_vp, c_vp, c_vp, c_int, c_vp]),
    "rgcsr_spmv_batched": (c_int, [c_vp, c_i32, c_vp, c_i64, c_vp, c_i64, c_int, c_i32, c_vp]),
    "rgcsr_spmv_transpose_grad": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, c_vp]),
    "rgcsr_set_values": (c_int, [c_vp, c_vp, c_int, c_int, c_vp]),
    "rgcsr_export": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rgcsr_to_csr": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "rgcsr_info": (c_int, [c_vp, ctypes.POINTER(Info)]),
    "rgcsr_destroy": (c_int, [c_vp]),
    "rgcsr_clone": (c_int, [c_vp, c_vp, ctypes.POINTER(c_vp)]),
    "hyb_clone": (c_int, [c_vp, c_vp, ctypes.POINTER(c_vp)]),
    "hyb_from_csr": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, c_int, c_i64, c_int, c_vp,
                             ctypes.POINTER(c_vp)]),
    "hyb_choose_width": (c_int, [c_i64, c_vp, c_int, P_I64]),
    "hyb_spmv": (c_int, [c_vp, c_vp, c_vp, c_int, c_vp]),
    "hyb_export": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "hyb_info": (c_int, [c_vp, ctypes.POINTER(HybInfo)]),
    "hyb_destroy": (c_int, [c_vp]),
    "rgcsr_cg_solve": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_double, ctypes.c_double, c_i32, c_i32, c_vp,
                               ctypes.POINTER(CGStats)]),
    "rgcsr_cg_solve_noalloc": (c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_double, ctypes.c_double, c_i32, c_i32,
                                       c_vp, ctypes.POINTER(CGStats)]),
    "rgcsr_cg_solve_f64": (c_int, [c_vp, c_vp, c_vp, ctypes.c_double, c_i32, c_vp, ctypes.POINTER(CGStats)]),
    "rgcsr_autotune": (c_int, [c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts), c_vp, c_vp,
                               c_int, c_i32, c_i32, c_vp, c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(Opts),
                               c_vp]),
    "rgcsr_autotune_batch": (c_int, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_int, ctypes.POINTER(Opts), c_vp, c_vp,
                                     c_int, c_i32, c_i32, c_vp, c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(Opts),
                                     c_vp]),
    "rgcsr_status_string": (ctypes.c_char_p, [c_int]),
    "rgcsr_last_error": (ctypes.c_char_p, []),
    "rgcsr_version": (ctypes.c_char_p, []),
    "rgcsr_stream_read": (c_int, [c_vp, c_i64, c_vp, c_vp]),
    "rgcsr_gather_floor": (c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "rgcsr_rcm_order": (c_int, [c_i64, c_i64, c_vp, c_vp, c_vp]),
}

_lib = None


class RgcsrError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librgcsr.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                               "or python -m paper_1012_2270_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def call(name: str, *args) -> None:
    """Call a status-returning entry point; raise RgcsrError on failure."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise RgcsrError(st, name, lib.rgcsr_last_error().decode(errors="replace"))

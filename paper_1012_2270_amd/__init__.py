"""RgCSR sparse matrix-vector multiplication on AMD Instinct MI355X.

Row-grouped CSR (Oberhuber, Suzuki, Vacata; Section 3.4 of their paper)
rebuilt for gfx950: the format conversion, the SpMV/SpMM kernels, the Hybrid
ELL+COO comparison (Section 3.3), a backward pass and a mixed-precision CG all
live in the native library ``librgcsr.so`` behind the C ABI of
``include/rgcsr.h``.  This package is the thin Python binding: the functions
named ``rgcsr_*`` / ``hyb_*`` marshal torch tensors and numpy arrays into those
C calls and do no arithmetic themselves.  PyTorch provides device memory and
streams only.

Importing the package does not load the library; the first call does, and
fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import RGCSR_BF16, RGCSR_F16, RGCSR_F32, RGCSR_F64, RgcsrError  # noqa: F401

DTYPE_CODES = {"f64": RGCSR_F64, "f32": RGCSR_F32, "f16": RGCSR_F16, "bf16": RGCSR_BF16}
CODE_BYTES = {RGCSR_F64: 8, RGCSR_F32: 4, RGCSR_F16: 2, RGCSR_BF16: 2}


def _code_of_numpy(a: np.ndarray, bf16_bits: bool = False) -> int:
    if bf16_bits:
        return RGCSR_BF16
    return {np.dtype(np.float64): RGCSR_F64, np.dtype(np.float32): RGCSR_F32,
            np.dtype(np.float16): RGCSR_F16}[a.dtype]


def _np_of_code(code: int):
    return {RGCSR_F64: np.float64, RGCSR_F32: np.float32, RGCSR_F16: np.float16,
            RGCSR_BF16: np.uint16}[code]


def _torch():
    import torch
    return torch


def _code_of_tensor(t) -> int:
    torch = _torch()
    return {torch.float64: RGCSR_F64, torch.float32: RGCSR_F32, torch.float16: RGCSR_F16,
            torch.bfloat16: RGCSR_BF16}[t.dtype]


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _astream(A, stream=None) -> int:
    """_stream for a call on matrix A; a matrix in torch memory (built from a
    plan) notes the stream, so that close() can hold the block until the work
    queued there has run."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    if getattr(A, "_memory", None) is not None:
        A._streams[s.cuda_stream] = s
    return s.cuda_stream


def _ptr(a) -> int:
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev_check(t, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _size_check(t, name: str, n: int, dtype=None) -> None:
    """t must hold exactly n elements (of dtype, when given)."""
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")


def _on_device_of(A, t, name: str) -> None:
    """t must be a contiguous device tensor on the device of matrix A."""
    _dev_check(t, name)
    dev = getattr(A, "device", None)
    if dev is not None and t.device.index != dev:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the matrix on cuda:{dev}")


def make_opts(G: int = 64, T: int = 1, sigma: int = 1, tau: int = -1, value_dtype: str = "f32",
              keep_csr_map: bool = False, build_transpose: bool = False, validate: bool = True,
              rows_per_lane: int = 0, pad_loads: int = -1, load_policy: int = 0,
              tile_min_len: int = -1, col_panels: int = 0) -> _lib.Opts:
    o = _lib.Opts()
    o.group_size, o.lanes_per_row, o.sort_window, o.long_row_threshold = G, T, sigma, tau
    o.value_dtype = DTYPE_CODES[value_dtype]
    o.keep_csr_map, o.build_transpose, o.validate = int(keep_csr_map), int(build_transpose), int(validate)
    o.rows_per_lane, o.pad_loads, o.load_policy = rows_per_lane, pad_loads, load_policy
    o.tile_min_len = tile_min_len
    o.col_panels = col_panels
    return o


def _csr_arrays(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.ascontiguousarray(A.val)
    return rp, col, val


# ----------------------------------------------------------------------------
# Host-only layout (no GPU)
# ----------------------------------------------------------------------------
def rgcsr_layout_sizes(A, opts: _lib.Opts) -> dict:
    rp, col, _ = _csr_arrays(A)
    info = _lib.Info()
    _lib.call("rgcsr_layout_sizes", A.n_rows, A.n_cols, int(rp[-1]) if rp.size else 0, _ptr(rp),
              _ptr(col), ctypes.byref(opts), ctypes.byref(info))
    return info.as_dict()


def rgcsr_panel_sizes(A, opts: _lib.Opts) -> dict:
    """Column bounds and piece counts of the column-panel copy (no GPU)."""
    rp, col, _ = _csr_arrays(A)
    cb = np.zeros(max(opts.col_panels, 0) + 1, np.int64)  # the library refuses a bad count
    outs = [ctypes.c_int64() for _ in range(5)]
    _lib.call("rgcsr_panel_sizes", A.n_rows, A.n_cols, int(rp[-1]) if rp.size else 0, _ptr(rp), _ptr(col),
              ctypes.byref(opts), _ptr(cb), *[ctypes.byref(o) for o in outs])
    keys = ("pieces", "split_rows", "split_pieces", "slots", "long_nnz")
    return dict(col_bounds=cb, **{k: o.value for k, o in zip(keys, outs)})


def rgcsr_tile_sizes(A, opts: _lib.Opts) -> dict:
    """Tiles, tiled rows and entries, tile-kernel workgroups and the row
    length threshold of the column-tiled copy (no GPU)."""
    rp, col, _ = _csr_arrays(A)
    outs = [ctypes.c_int64() for _ in range(5)]
    _lib.call("rgcsr_tile_sizes", A.n_rows, A.n_cols, int(rp[-1]) if rp.size else 0, _ptr(rp), _ptr(col),
              ctypes.byref(opts), *[ctypes.byref(o) for o in outs])
    keys = ("n_tiles", "tiled_rows", "tile_entries", "units", "min_len")
    return {k: o.value for k, o in zip(keys, outs)}


def rgcsr_layout_host(A, opts: _lib.Opts, bf16_bits: bool = False) -> dict:
    rp, col, val = _csr_arrays(A)
    s = rgcsr_layout_sizes(A, opts)
    vt = _np_of_code(opts.value_dtype)
    out = dict(gp=np.zeros(s["n_groups"] + 1, np.int64), short_len=np.zeros(s["n_short"], np.int32),
               short_row=np.zeros(s["n_short"], np.int32), slot_val=np.zeros(s["slots"], vt),
               slot_col=np.zeros(s["slots"], np.int32), long_row=np.zeros(s["n_long"], np.int32),
               long_ptr=np.zeros(s["n_long"] + 1, np.int64), long_val=np.zeros(s["long_nnz"], vt),
               long_col=np.zeros(s["long_nnz"], np.int32))
    _lib.call("rgcsr_layout_host", A.n_rows, A.n_cols, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(val),
              _code_of_numpy(val, bf16_bits), ctypes.byref(opts),
              *[_ptr(out[k]) for k in ("gp", "short_len", "short_row", "slot_val", "slot_col",
                                       "long_row", "long_ptr", "long_val", "long_col")])
    out.update(s)
    return out


def hyb_choose_width(A, value_dtype: str = "f32") -> int:
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    k = ctypes.c_int64(0)
    _lib.call("hyb_choose_width", A.n_rows, _ptr(rp), DTYPE_CODES[value_dtype], ctypes.byref(k))
    return int(k.value)


# ----------------------------------------------------------------------------
# Device handles
# ----------------------------------------------------------------------------
class RgCSRMatrix:
    """Owns one librgcsr handle (a matrix or a block-diagonal batch)."""

    def __init__(self, handle: int, memory=None):
        self._h = ctypes.c_void_p(handle)
        self._memory = memory  # caller-owned device buffer the handle borrows (rgcsr_build)
        self._streams = {}     # streams that queued work on a borrowing handle
        info = _lib.Info()
        _lib.call("rgcsr_info", self._h, ctypes.byref(info))
        self.info = info.as_dict()
        self.n_rows, self.n_cols, self.nnz = self.info["n_rows"], self.info["n_cols"], self.info["nnz"]
        self.value_dtype = self.info["value_dtype"]
        # the device the handle lives on (the current one when it was made)
        self.device = _torch().cuda.current_device()
        # bumped by every rgcsr_set_values; the autograd function uses it to
        # see whether the stored values changed between forward and backward
        self.value_version = 0

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.call("rgcsr_destroy", self._h)
        self._h = None
        if self._memory is not None:
            # destroying a handle in torch memory does not wait for its work:
            # the caching allocator reuses the block only once the work queued
            # so far on each stream that used the handle has run
            for st in self._streams.values():
                self._memory.record_stream(st)
        self._memory = None  # released only after the handle is gone
        self._streams = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # convenience forwarding to the module-level C-named functions
    def spmv(self, x, y=None, stream=None):
        torch = _torch()
        if y is None:
            y = torch.empty(self.n_rows, dtype=x.dtype, device=x.device)
        rgcsr_spmv(self, x, y, stream)
        return y

    def spmm(self, X, Y=None, persistent: bool = False, stream=None):
        torch = _torch()
        if Y is None:
            Y = torch.empty((self.n_rows, X.shape[1]), dtype=X.dtype, device=X.device)
        rgcsr_spmv_batched(self, X, Y, persistent, stream)
        return Y

    def export(self, stream=None) -> dict:
        return rgcsr_export(self, stream)

    def clone(self, stream=None) -> "RgCSRMatrix":
        return rgcsr_clone(self, stream)

    def to_csr(self, stream=None):
        return rgcsr_to_csr(self, stream)

    def batch_offsets(self):
        return rgcsr_batch_offsets(self)


def rgcsr_from_csr(A, opts: _lib.Opts | None = None, stream=None, bf16_bits: bool = False,
                   **kw) -> RgCSRMatrix:
    """Convert a host CSR matrix (workloads.CSR) to a device RgCSR handle
    (device CSR arrays: rgcsr_from_csr_device)."""
    opts = opts if opts is not None else make_opts(**kw)
    rp, col, val = _csr_arrays(A)
    h = ctypes.c_void_p()
    _lib.call("rgcsr_from_csr", A.n_rows, A.n_cols, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(val),
              _code_of_numpy(val, bf16_bits), ctypes.byref(opts), 0, _stream(stream), ctypes.byref(h))
    return RgCSRMatrix(h.value)


class RgCSRPlan:
    """Host-side layout of one matrix (rgcsr_plan_from_csr); build() places
    the device arrays in a torch-allocated buffer the handle borrows."""

    def __init__(self, handle: int):
        self._p = ctypes.c_void_p(handle)
        b = ctypes.c_int64()
        _lib.call("rgcsr_plan_device_bytes", self._p, ctypes.byref(b))
        self.device_bytes = b.value

    def build(self, buffer=None, stream=None) -> RgCSRMatrix:
        """buffer: a CUDA uint8 tensor of at least device_bytes (allocated
        here with torch when None); the returned matrix keeps it alive."""
        torch = _torch()
        if buffer is None:
            buffer = torch.empty(max(1, self.device_bytes), dtype=torch.uint8, device="cuda")
        _dev_check(buffer, "buffer")
        if buffer.device.index != torch.cuda.current_device():
            raise ValueError("buffer must be on the current device")
        h = ctypes.c_void_p()
        _lib.call("rgcsr_build", self._p, _ptr(buffer), int(buffer.numel() * buffer.element_size()), _stream(stream),
                  ctypes.byref(h))
        return RgCSRMatrix(h.value, memory=buffer)

    def close(self):
        if self._p is not None and self._p.value:
            _lib.call("rgcsr_plan_destroy", self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rgcsr_plan_from_csr(A, opts: _lib.Opts | None = None, bf16_bits: bool = False, **kw) -> RgCSRPlan:
    """Host conversion of a host CSR matrix, device memory left to the caller."""
    opts = opts if opts is not None else make_opts(**kw)
    rp, col, val = _csr_arrays(A)
    p = ctypes.c_void_p()
    _lib.call("rgcsr_plan_from_csr", A.n_rows, A.n_cols, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(val),
              _code_of_numpy(val, bf16_bits), ctypes.byref(opts), ctypes.byref(p))
    return RgCSRPlan(p.value)


def rgcsr_from_csr_device(n_rows: int, n_cols: int, row_ptr, col, vals, opts: _lib.Opts, stream=None) -> RgCSRMatrix:
    """Same as rgcsr_from_csr with CSR arrays already in device memory (torch tensors)."""
    h = ctypes.c_void_p()
    _lib.call("rgcsr_from_csr", n_rows, n_cols, int(col.numel()), _ptr(row_ptr), _ptr(col), _ptr(vals),
              _code_of_tensor(vals), ctypes.byref(opts), 1, _stream(stream), ctypes.byref(h))
    return RgCSRMatrix(h.value)


def _batch_arrays(mats):
    """Per-matrix sizes and pointer arrays of a batch (the arrays they point
    into are returned too, to stay alive across the call)."""
    n = len(mats)
    arrs = [_csr_arrays(A) for A in mats]
    nr = np.array([A.n_rows for A in mats], np.int64)
    nc = np.array([A.n_cols for A in mats], np.int64)
    rps = (ctypes.c_void_p * n)(*[_ptr(a[0]) for a in arrs])
    cols = (ctypes.c_void_p * n)(*[_ptr(a[1]) for a in arrs])
    vals = (ctypes.c_void_p * n)(*[_ptr(a[2]) for a in arrs])
    codes = {_code_of_numpy(a[2]) for a in arrs}
    if len(codes) != 1:
        raise ValueError("all matrices of a batch must share one value dtype")
    return arrs, nr, nc, rps, cols, vals, codes.pop()


def rgcsr_from_csr_batch(mats, opts: _lib.Opts | None = None, stream=None, **kw) -> RgCSRMatrix:
    """One handle for a list of host CSR matrices (block-diagonal batch)."""
    opts = opts if opts is not None else make_opts(**kw)
    arrs, nr, nc, rps, cols, vals, code = _batch_arrays(mats)
    h = ctypes.c_void_p()
    _lib.call("rgcsr_from_csr_batch", len(mats), _ptr(nr), _ptr(nc), ctypes.addressof(rps), ctypes.addressof(cols),
              ctypes.addressof(vals), code, ctypes.byref(opts), _stream(stream), ctypes.byref(h))
    return RgCSRMatrix(h.value)


def rgcsr_plan_from_csr_batch(mats, opts: _lib.Opts | None = None, **kw) -> RgCSRPlan:
    """Host conversion of a block-diagonal batch, device memory left to the caller."""
    opts = opts if opts is not None else make_opts(**kw)
    arrs, nr, nc, rps, cols, vals, code = _batch_arrays(mats)
    p = ctypes.c_void_p()
    _lib.call("rgcsr_plan_from_csr_batch", len(mats), _ptr(nr), _ptr(nc), ctypes.addressof(rps),
              ctypes.addressof(cols), ctypes.addressof(vals), code, ctypes.byref(opts), ctypes.byref(p))
    return RgCSRPlan(p.value)


def rgcsr_clone(A: RgCSRMatrix, stream=None) -> RgCSRMatrix:
    h = ctypes.c_void_p()
    _lib.call("rgcsr_clone", A.handle, _stream(stream), ctypes.byref(h))
    return RgCSRMatrix(h.value)


def rgcsr_batch_offsets(A: RgCSRMatrix):
    m = A.info["n_matrices"]
    ro = np.zeros(m + 1, np.int64)
    co = np.zeros(m + 1, np.int64)
    _lib.call("rgcsr_batch_offsets", A.handle, _ptr(ro), _ptr(co))
    return ro, co


def rgcsr_spmv(A: RgCSRMatrix, x, y, stream=None) -> None:
    """y = A x (device tensors, float32 or float64)."""
    _dev_check(x, "x")
    _dev_check(y, "y")
    if x.dtype != y.dtype or x.numel() != A.n_cols or y.numel() != A.n_rows:
        raise ValueError("x/y shape or dtype mismatch")
    _lib.call("rgcsr_spmv", A.handle, _ptr(x), _ptr(y), _code_of_tensor(x), _astream(A, stream))


def rgcsr_spmv_batched(A: RgCSRMatrix, X, Y, persistent: bool = False, stream=None) -> None:
    """Y = A X for X of shape (n_cols, k), row-major; Y of shape (n_rows, k)."""
    _dev_check(X, "X")
    _dev_check(Y, "Y")
    if X.dim() == 1:
        X, Y = X.view(-1, 1), Y.view(-1, 1)
    if X.shape[0] != A.n_cols or Y.shape[0] != A.n_rows or X.shape[1] != Y.shape[1] or X.dtype != Y.dtype:
        raise ValueError("X/Y shape or dtype mismatch")
    k = X.shape[1]
    _lib.call("rgcsr_spmv_batched", A.handle, k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
              _code_of_tensor(X), int(persistent), _astream(A, stream))


def rgcsr_spmv_transpose_grad(A: RgCSRMatrix, x, dy, dx=None, dvals=None, stream=None) -> None:
    """dx = A^T dy and dvals[k] = dy[row(k)] * x[col(k)] (CSR order).  x, dx
    hold n_cols elements, dy n_rows, dvals nnz, all of dy's dtype (float32 or
    float64) on the matrix's device; x is needed only for dvals."""
    # every size and dtype first, then the devices
    if dy.dtype not in (_torch().float32, _torch().float64):
        raise ValueError(f"dy has dtype {dy.dtype}, expected float32 or float64")
    _size_check(dy, "dy", A.n_rows)
    if dvals is not None and x is None:
        raise ValueError("dvals needs x")
    for t, nm, n in ((x, "x", A.n_cols), (dx, "dx", A.n_cols), (dvals, "dvals", A.nnz)):
        if t is not None:
            _size_check(t, nm, n, dy.dtype)
    for t, nm in ((dy, "dy"), (x, "x"), (dx, "dx"), (dvals, "dvals")):
        if t is not None:
            _on_device_of(A, t, nm)
    _lib.call("rgcsr_spmv_transpose_grad", A.handle, _ptr(x), _ptr(dy), _ptr(dx), _ptr(dvals),
              _code_of_tensor(dy), _astream(A, stream))


def rgcsr_set_values(A: RgCSRMatrix, vals, stream=None) -> None:
    """Overwrite stored values from nnz CSR-ordered values (a float64/float32
    device tensor on the matrix's device, or a float64/float32/float16 numpy
    array)."""
    if isinstance(vals, np.ndarray):
        v = np.ascontiguousarray(vals)
        if v.size != A.nnz:
            raise ValueError(f"vals has {v.size} elements, expected {A.nnz}")
        if v.dtype not in (np.float64, np.float32, np.float16):
            raise ValueError(f"vals has dtype {v.dtype}, expected float64, float32 or float16")
        _lib.call("rgcsr_set_values", A.handle, _ptr(v), _code_of_numpy(v), 0, _astream(A, stream))
    else:
        if vals.dtype not in (_torch().float32, _torch().float64):
            raise ValueError(f"vals has dtype {vals.dtype}, expected float32 or float64")
        _size_check(vals, "vals", A.nnz)
        _on_device_of(A, vals, "vals")
        _lib.call("rgcsr_set_values", A.handle, _ptr(vals), _code_of_tensor(vals), 1, _astream(A, stream))
    A.value_version = getattr(A, "value_version", 0) + 1


def rgcsr_export(A: RgCSRMatrix, stream=None) -> dict:
    i = A.info
    vt = _np_of_code(A.value_dtype)
    out = dict(gp=np.zeros(i["n_groups"] + 1, np.int64), short_len=np.zeros(i["n_short"], np.int32),
               short_row=np.zeros(i["n_short"], np.int32), slot_val=np.zeros(i["slots"], vt),
               slot_col=np.zeros(i["slots"], np.int32), long_row=np.zeros(i["n_long"], np.int32),
               long_ptr=np.zeros(i["n_long"] + 1, np.int64), long_val=np.zeros(i["long_nnz"], vt),
               long_col=np.zeros(i["long_nnz"], np.int32))
    _lib.call("rgcsr_export", A.handle, _stream(stream),
              *[_ptr(out[k]) for k in ("gp", "short_len", "short_row", "slot_val", "slot_col",
                                       "long_row", "long_ptr", "long_val", "long_col")])
    return out


def rgcsr_to_csr(A: RgCSRMatrix, stream=None):
    rp = np.zeros(A.n_rows + 1, np.int64)
    col = np.zeros(A.nnz, np.int32)
    val = np.zeros(A.nnz, _np_of_code(A.value_dtype))
    _lib.call("rgcsr_to_csr", A.handle, _stream(stream), _ptr(rp), _ptr(col), _ptr(val))
    return rp, col, val


# ----------------------------------------------------------------------------
# Hybrid ELL + COO
# ----------------------------------------------------------------------------
class HybMatrix:
    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        info = _lib.HybInfo()
        _lib.call("hyb_info", self._h, ctypes.byref(info))
        self.info = info.as_dict()
        self.n_rows, self.n_cols = self.info["n_rows"], self.info["n_cols"]
        self.value_dtype = self.info["value_dtype"]

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            _lib.call("hyb_destroy", self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spmv(self, x, y=None, stream=None):
        torch = _torch()
        if y is None:
            y = torch.empty(self.n_rows, dtype=x.dtype, device=x.device)
        hyb_spmv(self, x, y, stream)
        return y

    def clone(self, stream=None) -> "HybMatrix":
        h = ctypes.c_void_p()
        _lib.call("hyb_clone", self.handle, _stream(stream), ctypes.byref(h))
        return HybMatrix(h.value)


def hyb_from_csr(A, value_dtype: str = "f32", ell_width: int = -1, validate: bool = True,
                 stream=None) -> HybMatrix:
    rp, col, val = _csr_arrays(A)
    h = ctypes.c_void_p()
    _lib.call("hyb_from_csr", A.n_rows, A.n_cols, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(val),
              _code_of_numpy(val), DTYPE_CODES[value_dtype], ell_width, int(validate), _stream(stream),
              ctypes.byref(h))
    return HybMatrix(h.value)


def hyb_spmv(A: HybMatrix, x, y, stream=None) -> None:
    _dev_check(x, "x")
    _dev_check(y, "y")
    if x.numel() != A.n_cols or y.numel() != A.n_rows or x.dtype != y.dtype:
        raise ValueError("x/y shape or dtype mismatch")
    _lib.call("hyb_spmv", A.handle, _ptr(x), _ptr(y), _code_of_tensor(x), _stream(stream))


def hyb_export(A: HybMatrix, stream=None) -> dict:
    i = A.info
    ne = i["n_pad"] * i["ell_width"]
    vt = _np_of_code(A.value_dtype)
    out = dict(ell_col=np.zeros(ne, np.int32), ell_val=np.zeros(ne, vt),
               coo_row=np.zeros(i["coo_nnz"], np.int32), coo_col=np.zeros(i["coo_nnz"], np.int32),
               coo_val=np.zeros(i["coo_nnz"], vt))
    _lib.call("hyb_export", A.handle, _stream(stream),
              *[_ptr(out[k]) for k in ("ell_col", "ell_val", "coo_row", "coo_col", "coo_val")])
    return out


# ----------------------------------------------------------------------------
# Conjugate gradients
# ----------------------------------------------------------------------------
def rgcsr_cg_solve(A_lo: RgCSRMatrix, A_hi: RgCSRMatrix, b, x, tol: float = 1e-10, inner_tol: float = 1e-4,
                   max_outer: int = 50, max_inner: int = 500, stream=None) -> dict:
    """Mixed-precision CG with FP64 refinement; b, x float64 device tensors."""
    _dev_check(b, "b")
    _dev_check(x, "x")
    st = _lib.CGStats()
    _lib.call("rgcsr_cg_solve", A_lo.handle, A_hi.handle, _ptr(b), _ptr(x), tol, inner_tol, max_outer,
              max_inner, _stream(stream), ctypes.byref(st))
    return st.as_dict()


def rgcsr_cg_solve_noalloc(A_lo: RgCSRMatrix, A_hi: RgCSRMatrix, b, x, tol: float = 1e-10, inner_tol: float = 1e-4,
                           max_outer: int = 50, max_inner: int = 500, stream=None) -> dict:
    """rgcsr_cg_solve with the library's static device workspace (no device
    allocation; at most 1,048,576 rows; calls on one device must not overlap)."""
    _dev_check(b, "b")
    _dev_check(x, "x")
    st = _lib.CGStats()
    _lib.call("rgcsr_cg_solve_noalloc", A_lo.handle, A_hi.handle, _ptr(b), _ptr(x), tol, inner_tol, max_outer,
              max_inner, _stream(stream), ctypes.byref(st))
    return st.as_dict()


def rgcsr_cg_solve_f64(A: RgCSRMatrix, b, x, tol: float = 1e-10, max_iter: int = 2000, stream=None) -> dict:
    _dev_check(b, "b")
    _dev_check(x, "x")
    st = _lib.CGStats()
    _lib.call("rgcsr_cg_solve_f64", A.handle, _ptr(b), _ptr(x), tol, max_iter, _stream(stream),
              ctypes.byref(st))
    return st.as_dict()


def opts_dict(o: _lib.Opts) -> dict:
    return {f: getattr(o, f) for f, _ in _lib.Opts._fields_}


def opts_from_dict(d: dict) -> _lib.Opts:
    o = _lib.Opts()
    defaults = opts_dict(make_opts())
    for f, _ in _lib.Opts._fields_:
        setattr(o, f, int(d.get(f, defaults[f])))
    return o


def matrix_fingerprint(A) -> str:
    """Stable key of a matrix's sparsity pattern (sizes and a hash of the row
    pointers and a strided sample of the column indices)."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.array([A.n_rows, A.n_cols, A.nnz], np.int64).tobytes())
    h.update(np.ascontiguousarray(A.row_ptr, np.int64).tobytes())
    step = max(1, A.nnz // 65536)
    h.update(np.ascontiguousarray(np.asarray(A.col)[::step], np.int32).tobytes())
    return h.hexdigest()[:24]


def _cached_tune(key: str, cache_path, run):
    """JSON cache of autotuner results (cache_path, default
    $RGCSR_AUTOTUNE_CACHE if set, else no cache)."""
    import json
    import os
    path = cache_path or os.environ.get("RGCSR_AUTOTUNE_CACHE")
    cache = {}
    if path and os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
        if key in cache:
            return opts_from_dict(cache[key]["best"]), cache[key]["tried"]
    best, tried = run()
    if path:
        cache[key] = {"best": opts_dict(best), "tried": tried}
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, tried


def rgcsr_autotune(A, x, y, base: _lib.Opts | None = None, max_candidates: int = 16, reps: int = 20,
                   cache_path: str | None = None, stream=None) -> tuple[_lib.Opts, list]:
    """Pick layout and schedule for A by a cost-model prefilter and timing
    the best candidates on the device (native search in librgcsr).  Results
    are cached in a JSON file keyed by the matrix fingerprint, the value dtype
    and the vector dtype."""
    base = base if base is not None else make_opts()
    key = f"{matrix_fingerprint(A)}:{base.value_dtype}:{_code_of_tensor(x)}"

    def run():
        _dev_check(x, "x")
        _dev_check(y, "y")
        rp, col, val = _csr_arrays(A)
        cands = (_lib.Opts * max_candidates)()
        times = np.zeros(max_candidates, np.float64)
        n = ctypes.c_int32(0)
        best = _lib.Opts()
        _lib.call("rgcsr_autotune", A.n_rows, A.n_cols, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(val),
                  _code_of_numpy(val), ctypes.byref(base), _ptr(x), _ptr(y), _code_of_tensor(x), max_candidates,
                  reps, ctypes.addressof(cands), _ptr(times), ctypes.byref(n), ctypes.byref(best), _stream(stream))
        return best, [{"opts": opts_dict(cands[i]), "us": float(times[i])} for i in range(n.value)]
    return _cached_tune(key, cache_path, run)


def rgcsr_autotune_batch(mats, x, y, base: _lib.Opts | None = None, max_candidates: int = 12, reps: int = 10,
                         cache_path: str | None = None, stream=None) -> tuple[_lib.Opts, list]:
    """Same for a batch of matrices (rgcsr_from_csr_batch): every candidate
    is built as a batch handle and timed on one launch over all matrices.  x
    and y hold the concatenated per-matrix vectors."""
    import hashlib
    base = base if base is not None else make_opts()
    h = hashlib.sha256()
    for M in mats:
        h.update(matrix_fingerprint(M).encode())
    key = f"batch{len(mats)}:{h.hexdigest()[:24]}:{base.value_dtype}:{_code_of_tensor(x)}"

    def run():
        _dev_check(x, "x")
        _dev_check(y, "y")
        arrs = [_csr_arrays(M) for M in mats]
        count = len(mats)
        nr = np.array([M.n_rows for M in mats], np.int64)
        nc = np.array([M.n_cols for M in mats], np.int64)
        rps = (ctypes.c_void_p * count)(*[_ptr(a[0]) for a in arrs])
        cols = (ctypes.c_void_p * count)(*[_ptr(a[1]) for a in arrs])
        vals = (ctypes.c_void_p * count)(*[_ptr(a[2]) for a in arrs])
        cands = (_lib.Opts * max_candidates)()
        times = np.zeros(max_candidates, np.float64)
        n = ctypes.c_int32(0)
        best = _lib.Opts()
        _lib.call("rgcsr_autotune_batch", count, _ptr(nr), _ptr(nc), ctypes.addressof(rps), ctypes.addressof(cols),
                  ctypes.addressof(vals), _code_of_numpy(arrs[0][2]),
                  ctypes.byref(base), _ptr(x), _ptr(y), _code_of_tensor(x), max_candidates, reps,
                  ctypes.addressof(cands), _ptr(times), ctypes.byref(n), ctypes.byref(best), _stream(stream))
        return best, [{"opts": opts_dict(cands[i]), "us": float(times[i])} for i in range(n.value)]
    return _cached_tune(key, cache_path, run)


def version() -> str:
    return _lib.load().rgcsr_version().decode()


def rgcsr_rcm_order(A) -> np.ndarray:
    """Reverse Cuthill-McKee order of a square host CSR matrix: perm[new] = old."""
    if A.n_rows != A.n_cols:
        raise ValueError("ordering needs a square matrix")
    rp, col, _ = _csr_arrays(A)
    perm = np.empty(A.n_rows, dtype=np.int32)
    _lib.call("rgcsr_rcm_order", A.n_rows, int(rp[-1]), _ptr(rp), _ptr(col), _ptr(perm))
    return perm


def rgcsr_gather_floor(col, val, x, out, stream=None) -> None:
    """The gather-floor probe over device arrays col (int32), val (float32)
    and x (float32); out holds ceil(len(col) / 8) floats."""
    for t, nm in ((col, "col"), (val, "val"), (x, "x"), (out, "out")):
        _dev_check(t, nm)
    n = col.numel()
    if val.numel() != n or out.numel() < (n + 7) // 8:
        raise ValueError("sizes do not match")
    _lib.call("rgcsr_gather_floor", _ptr(col), _ptr(val), n, _ptr(x), x.numel(), _ptr(out), _stream(stream))


def rgcsr_stream_read(buf, sink, stream=None) -> None:
    """One streaming read of the device tensor buf (the achievable-bandwidth
    probe); sink is a small device tensor the kernel may write."""
    _dev_check(buf, "buf")
    _dev_check(sink, "sink")
    _lib.call("rgcsr_stream_read", _ptr(buf), buf.numel() * buf.element_size(), _ptr(sink), _stream(stream))


# ----------------------------------------------------------------------------
# Autograd
# ----------------------------------------------------------------------------
def spmv_function():
    """torch.autograd.Function computing y = A(theta) x with the hand-written
    adjoint (rgcsr_spmv_transpose_grad).  The matrix must be built with
    keep_csr_map or build_transpose; theta holds its values in CSR order."""
    torch = _torch()

    class SpMVFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, x, A):
            rgcsr_set_values(A, theta.detach().contiguous())
            y = torch.empty(A.n_rows, dtype=x.dtype, device=x.device)
            rgcsr_spmv(A, x.detach().contiguous(), y)
            ctx.A = A
            ctx.version = A.value_version
            ctx.save_for_backward(x, theta)
            return y

        @staticmethod
        def backward(ctx, dy):
            x, theta = ctx.saved_tensors
            A = ctx.A
            dy = dy.contiguous()
            need_theta, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            # dx = A(theta)^T dy reads the stored values: when another forward
            # (or any value update) has replaced them since this forward, put
            # this call's theta back first; dvals do not depend on them
            if need_x and A.value_version != ctx.version:
                rgcsr_set_values(A, theta.detach().contiguous())
            dvals = torch.empty(A.nnz, dtype=dy.dtype, device=dy.device) if need_theta else None
            dx = torch.empty(A.n_cols, dtype=dy.dtype, device=dy.device) if need_x else None
            if dvals is not None or dx is not None:
                rgcsr_spmv_transpose_grad(A, x.contiguous(), dy, dx, dvals)
            return dvals, dx, None

    return SpMVFunction

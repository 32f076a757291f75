"""Python face of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this package, and this package never imports the product library; the two share
only the seeded input generators, which hold none of the method's arithmetic.

Every function upcasts its inputs exactly to float64 (float32, float16 and
bfloat16 values are exact in float64) and calls the plain C routine that
follows the paper's definition (Section 3.1 serial CSR SpMV, Section 3.4 RgCSR
layout and kernel walk, Section 3.3 Hybrid ELL+COO).  Parity pins for each
routine live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)
_U8P = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_csr_spmv.restype = None
        lib.orc_csr_spmv_par.restype = None
        lib.orc_csr_absmv.restype = None
        lib.orc_csr_spmm.restype = None
        lib.orc_csr_check.restype = ctypes.c_int
        lib.orc_csr_transpose.restype = None
        lib.orc_adjoint.restype = None
        lib.orc_cg.restype = ctypes.c_int64
        lib.orc_rgcsr_sizes.restype = None
        lib.orc_rgcsr_build.restype = None
        lib.orc_rgcsr_decode.restype = None
        lib.orc_rgcsr_spmv.restype = None
        lib.orc_hyb_k1.restype = ctypes.c_int64
        lib.orc_hyb_coo_count.restype = ctypes.c_int64
        lib.orc_hyb_build.restype = None
        lib.orc_hyb_spmv.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def to_f64(v: np.ndarray, bf16_bits: bool = False) -> np.ndarray:
    """Exact upcast to float64.  ``bf16_bits`` marks a uint16 array holding
    bfloat16 bit patterns (numpy has no bfloat16 type)."""
    v = np.asarray(v)
    if bf16_bits:
        return (v.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return v.astype(np.float64, copy=False)


def round_values(v: np.ndarray, dtype: str) -> np.ndarray:
    """Round-to-nearest-even conversion of stored values, pinned to the library
    routine ``torch.Tensor.to`` on the CPU.  Returns float64/float32/float16
    arrays, or uint16 bit patterns for bfloat16."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(v))
    if dtype == "f64":
        return t.to(torch.float64).numpy()
    if dtype == "f32":
        return t.to(torch.float32).numpy()
    if dtype == "f16":
        return t.to(torch.float16).numpy()
    if dtype == "bf16":
        return t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    raise ValueError(dtype)


# ----------------------------------------------------------------------------
# CSR
# ----------------------------------------------------------------------------
def csr_spmv(A, x, bf16_bits: bool = False) -> np.ndarray:
    """y = A x by the serial CSR SpMV of Section 3.1, in float64."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val, bf16_bits))
    x = np.ascontiguousarray(to_f64(x))
    y = np.empty(A.n_rows, dtype=np.float64)
    lib.orc_csr_spmv(ctypes.c_int64(A.n_rows), _p(rp, _I64P), _p(col, _I32P), _p(val, _F64P),
                     _p(x, _F64P), _p(y, _F64P))
    return y


def csr_spmv_parallel(A, x, threads: int, bf16_bits: bool = False) -> np.ndarray:
    """csr_spmv with the rows split into `threads` equal contiguous ranges, one
    OpenMP thread each; every row keeps its serial order, so the result is
    bit-identical to csr_spmv (for timing the oracle on all host cores)."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val, bf16_bits))
    x = np.ascontiguousarray(to_f64(x))
    y = np.empty(A.n_rows, dtype=np.float64)
    lib.orc_csr_spmv_par(ctypes.c_int64(A.n_rows), _p(rp, _I64P), _p(col, _I32P), _p(val, _F64P),
                         _p(x, _F64P), _p(y, _F64P), ctypes.c_int(int(threads)))
    return y


def csr_absmv(A, x, bf16_bits: bool = False) -> np.ndarray:
    """s = |A| |x| in float64 (the scale of the error tolerance)."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val, bf16_bits))
    x = np.ascontiguousarray(to_f64(x))
    s = np.empty(A.n_rows, dtype=np.float64)
    lib.orc_csr_absmv(ctypes.c_int64(A.n_rows), _p(rp, _I64P), _p(col, _I32P), _p(val, _F64P),
                      _p(x, _F64P), _p(s, _F64P))
    return s


def csr_spmm(A, X) -> np.ndarray:
    """Y = A X, X of shape (n_cols, k) row-major, column by column."""
    lib = _load()
    X = np.ascontiguousarray(to_f64(X))
    k = X.shape[1]
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val))
    Y = np.empty((A.n_rows, k), dtype=np.float64)
    lib.orc_csr_spmm(ctypes.c_int64(A.n_rows), ctypes.c_int64(A.n_cols), ctypes.c_int64(k),
                     _p(rp, _I64P), _p(col, _I32P), _p(val, _F64P), _p(X, _F64P), _p(Y, _F64P))
    return Y


def csr_check(n_rows, n_cols, nnz, row_ptr, col) -> int:
    lib = _load()
    rp, c = _i64(row_ptr), _i32(col)
    return int(lib.orc_csr_check(ctypes.c_int64(n_rows), ctypes.c_int64(n_cols),
                                 ctypes.c_int64(nnz), _p(rp, _I64P), _p(c, _I32P)))


def csr_transpose(A):
    """A^T as (row_ptr, col, val float64)."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val))
    rpT = np.empty(A.n_cols + 1, np.int64)
    colT = np.empty(A.nnz, np.int32)
    valT = np.empty(A.nnz, np.float64)
    lib.orc_csr_transpose(ctypes.c_int64(A.n_rows), ctypes.c_int64(A.n_cols), _p(rp, _I64P),
                          _p(col, _I32P), _p(val, _F64P), _p(rpT, _I64P), _p(colT, _I32P),
                          _p(valT, _F64P))
    return rpT, colT, valT


def adjoint(A, x, b):
    """r = A x - b, dx = A^T r, dval_k = r[row(k)] x[col(k)], L = fsum(r^2)/2."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val))
    x = np.ascontiguousarray(to_f64(x))
    b = np.ascontiguousarray(to_f64(b))
    r = np.empty(A.n_rows, np.float64)
    dx = np.empty(A.n_cols, np.float64)
    dval = np.empty(A.nnz, np.float64)
    lib.orc_adjoint(ctypes.c_int64(A.n_rows), ctypes.c_int64(A.n_cols), _p(rp, _I64P),
                    _p(col, _I32P), _p(val, _F64P), _p(x, _F64P), _p(b, _F64P), _p(r, _F64P),
                    _p(dx, _F64P), _p(dval, _F64P))
    L = 0.5 * math.fsum((r * r).tolist())
    return r, dx, dval, L


def loss(A, x, b) -> float:
    """L = 1/2 ||A x - b||^2 with exactly rounded summation of the squares."""
    r = csr_spmv(A, x) - to_f64(b)
    return 0.5 * math.fsum((r * r).tolist())


def cg(A, b, x0=None, tol: float = 1e-12, maxit: int = 10_000):
    """Plain FP64 conjugate gradients; returns (x, iterations, relres)."""
    lib = _load()
    rp, col = _i64(A.row_ptr), _i32(A.col)
    val = np.ascontiguousarray(to_f64(A.val))
    b = np.ascontiguousarray(to_f64(b))
    x = np.zeros(A.n_rows) if x0 is None else np.array(to_f64(x0), dtype=np.float64)
    rel = ctypes.c_double(0.0)
    it = lib.orc_cg(ctypes.c_int64(A.n_rows), _p(rp, _I64P), _p(col, _I32P), _p(val, _F64P),
                    _p(b, _F64P), _p(x, _F64P), ctypes.c_double(tol), ctypes.c_int64(maxit),
                    ctypes.byref(rel))
    return x, int(it), float(rel.value)


# ----------------------------------------------------------------------------
# RgCSR layout
# ----------------------------------------------------------------------------
def rgcsr_sizes(A, G: int, T: int = 1, sigma: int = 1, tau: int = -1) -> dict:
    lib = _load()
    rp = _i64(A.row_ptr)
    out = np.zeros(5, np.int64)
    lib.orc_rgcsr_sizes(ctypes.c_int64(A.n_rows), _p(rp, _I64P), ctypes.c_int64(G),
                        ctypes.c_int64(T), ctypes.c_int64(sigma), ctypes.c_int64(tau),
                        _p(out, _I64P))
    return dict(groups=int(out[0]), n_short=int(out[1]), n_long=int(out[2]),
                slots=int(out[3]), long_nnz=int(out[4]))


def rgcsr_layout(A, G: int, T: int = 1, sigma: int = 1, tau: int = -1, values=None) -> dict:
    """Every RgCSR array for the given parameters (layout rules in oracle.c).
    ``values`` defaults to A.val; any fixed-width dtype is moved as raw bytes."""
    lib = _load()
    sz = rgcsr_sizes(A, G, T, sigma, tau)
    vals = np.ascontiguousarray(A.val if values is None else values)
    esz = vals.dtype.itemsize
    rp, col = _i64(A.row_ptr), _i32(A.col)
    L = dict(
        n_rows=A.n_rows, n_cols=A.n_cols, G=G, T=T, sigma=sigma, tau=tau, dtype=vals.dtype, **sz,
        gp=np.zeros(sz["groups"] + 1, np.int64),
        short_len=np.zeros(sz["n_short"], np.int32),
        short_row=np.zeros(sz["n_short"], np.int32),
        slot_val=np.zeros(sz["slots"], vals.dtype),
        slot_col=np.zeros(sz["slots"], np.int32),
        long_row=np.zeros(sz["n_long"], np.int32),
        long_ptr=np.zeros(sz["n_long"] + 1, np.int64),
        long_val=np.zeros(sz["long_nnz"], vals.dtype),
        long_col=np.zeros(sz["long_nnz"], np.int32),
    )
    u8 = lambda a: a.view(np.uint8).ctypes.data_as(_U8P)  # noqa: E731
    lib.orc_rgcsr_build(ctypes.c_int64(A.n_rows), _p(rp, _I64P), _p(col, _I32P), u8(vals),
                        ctypes.c_int64(esz), ctypes.c_int64(G), ctypes.c_int64(T),
                        ctypes.c_int64(sigma), ctypes.c_int64(tau),
                        _p(L["gp"], _I64P), _p(L["short_len"], _I32P), _p(L["short_row"], _I32P),
                        u8(L["slot_val"]), _p(L["slot_col"], _I32P), _p(L["long_row"], _I32P),
                        _p(L["long_ptr"], _I64P), u8(L["long_val"]), _p(L["long_col"], _I32P))
    return L


def rgcsr_decode(L: dict):
    """Recover (row_ptr, col, val) from layout arrays; values keep their bits."""
    lib = _load()
    n = L["n_rows"]
    nnz = int(L["short_len"].astype(np.int64).sum()) + L["long_nnz"]
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, L["slot_val"].dtype)
    u8 = lambda a: a.view(np.uint8).ctypes.data_as(_U8P)  # noqa: E731
    lib.orc_rgcsr_decode(ctypes.c_int64(n), ctypes.c_int64(L["G"]), ctypes.c_int64(L["T"]),
                         ctypes.c_int64(L["n_short"]), ctypes.c_int64(L["n_long"]),
                         _p(L["gp"], _I64P), _p(L["short_len"], _I32P), _p(L["short_row"], _I32P),
                         u8(L["slot_val"]), _p(L["slot_col"], _I32P), _p(L["long_row"], _I32P),
                         _p(L["long_ptr"], _I64P), u8(L["long_val"]), _p(L["long_col"], _I32P),
                         ctypes.c_int64(L["slot_val"].dtype.itemsize), _p(rp, _I64P),
                         _p(col, _I32P), u8(val))
    return rp, col, val


def rgcsr_spmv(L: dict, x, bf16_bits: bool = False) -> np.ndarray:
    """The RgCSR kernel's walk over the layout (Section 3.4), FP64."""
    lib = _load()
    sv = np.ascontiguousarray(to_f64(L["slot_val"], bf16_bits))
    lv = np.ascontiguousarray(to_f64(L["long_val"], bf16_bits))
    x = np.ascontiguousarray(to_f64(x))
    y = np.empty(L["n_rows"], np.float64)
    lib.orc_rgcsr_spmv(ctypes.c_int64(L["n_rows"]), ctypes.c_int64(L["G"]), ctypes.c_int64(L["T"]),
                       ctypes.c_int64(L["n_short"]), ctypes.c_int64(L["n_long"]),
                       _p(L["gp"], _I64P), _p(L["short_len"], _I32P), _p(L["short_row"], _I32P),
                       _p(sv, _F64P), _p(L["slot_col"], _I32P), _p(L["long_row"], _I32P),
                       _p(L["long_ptr"], _I64P), _p(lv, _F64P), _p(L["long_col"], _I32P),
                       _p(x, _F64P), _p(y, _F64P))
    return y


def artificial_zeros(L: dict) -> int:
    """Padding slots of the grouped part (Section 4.3 "filling")."""
    return int(L["slots"] - L["short_len"].astype(np.int64).sum())


# ----------------------------------------------------------------------------
# Hybrid ELL + COO
# ----------------------------------------------------------------------------
def hyb_k1(A, s_v: int, c: int = 3) -> int:
    lib = _load()
    rp = _i64(A.row_ptr)
    return int(lib.orc_hyb_k1(ctypes.c_int64(A.n_rows), _p(rp, _I64P), ctypes.c_int64(s_v),
                              ctypes.c_int64(c)))


def hyb_layout(A, K1: int, values=None) -> dict:
    lib = _load()
    n = A.n_rows
    n_pad = (n + 63) // 64 * 64
    vals = np.ascontiguousarray(A.val if values is None else values)
    rp, col = _i64(A.row_ptr), _i32(A.col)
    m = int(lib.orc_hyb_coo_count(ctypes.c_int64(n), _p(rp, _I64P), ctypes.c_int64(K1)))
    H = dict(n_rows=n, n_cols=A.n_cols, K1=K1, n_pad=n_pad, coo_nnz=m,
             ell_col=np.zeros(n_pad * K1, np.int32), ell_val=np.zeros(n_pad * K1, vals.dtype),
             coo_row=np.zeros(m, np.int32), coo_col=np.zeros(m, np.int32),
             coo_val=np.zeros(m, vals.dtype))
    u8 = lambda a: a.view(np.uint8).ctypes.data_as(_U8P)  # noqa: E731
    lib.orc_hyb_build(ctypes.c_int64(n), _p(rp, _I64P), _p(col, _I32P), u8(vals),
                      ctypes.c_int64(vals.dtype.itemsize), ctypes.c_int64(K1),
                      ctypes.c_int64(n_pad), _p(H["ell_col"], _I32P), u8(H["ell_val"]),
                      _p(H["coo_row"], _I32P), _p(H["coo_col"], _I32P), u8(H["coo_val"]))
    return H


def hyb_spmv(H: dict, x, bf16_bits: bool = False) -> np.ndarray:
    lib = _load()
    ev = np.ascontiguousarray(to_f64(H["ell_val"], bf16_bits))
    cv = np.ascontiguousarray(to_f64(H["coo_val"], bf16_bits))
    x = np.ascontiguousarray(to_f64(x))
    y = np.empty(H["n_rows"], np.float64)
    lib.orc_hyb_spmv(ctypes.c_int64(H["n_rows"]), ctypes.c_int64(H["K1"]),
                     ctypes.c_int64(H["n_pad"]), _p(H["ell_col"], _I32P), _p(ev, _F64P),
                     ctypes.c_int64(H["coo_nnz"]), _p(H["coo_row"], _I32P),
                     _p(H["coo_col"], _I32P), _p(cv, _F64P), _p(x, _F64P), _p(y, _F64P))
    return y


# ----------------------------------------------------------------------------
# Judging a floating-point result
# ----------------------------------------------------------------------------
def rcm_order(A) -> np.ndarray:
    """Reverse Cuthill-McKee order of a square CSR matrix, perm[new] = old, in
    plain Python from the published definition (Cuthill and McKee, 1969;
    reversed by George, 1971); the row-ordering study the paper leaves to
    future work (Section 4.4.2, Table 7, Section 5).  Graph: i ~ j for i != j
    when a_ij or a_ji is stored.  Each component starts at the unnumbered
    vertex of smallest (degree, index); a numbered vertex numbers its
    unnumbered neighbours in (degree, index) order; the sequence is reversed.
    For small matrices (a Python loop per edge)."""
    n = A.n_rows
    assert A.n_cols == n
    nbrs = [set() for _ in range(n)]
    for i in range(n):
        for k in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            j = int(A.col[k])
            if j != i:
                nbrs[i].add(j)
                nbrs[j].add(i)
    deg = [len(s) for s in nbrs]
    key = lambda v: (deg[v], v)
    numbered = [False] * n
    order = []
    for s in sorted(range(n), key=key):
        if numbered[s]:
            continue
        numbered[s] = True
        order.append(s)
        head = len(order) - 1
        while head < len(order):
            v = order[head]
            head += 1
            for u in sorted((u for u in nbrs[v] if not numbered[u]), key=key):
                numbered[u] = True
                order.append(u)
    return np.array(order[::-1], dtype=np.int32)


def scaled_error(y, y_ref, s) -> float:
    """max_i |y_i - y_ref_i| / max_i s_i; when max s = 0 the result must be
    exactly zero and the error is 0 or inf."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    smax = float(np.max(s)) if np.size(s) else 0.0
    diff = float(np.max(np.abs(y - y_ref))) if np.size(y) else 0.0
    if smax == 0.0:
        return 0.0 if diff == 0.0 else math.inf
    return diff / smax

"""Seeded synthetic inputs: sparse matrices in CSR and dense vectors.

This module only draws inputs.  It holds none of the SpMV arithmetic, none of
the RgCSR or Hybrid layout rules and no reference result, so both the HIP path
and the CPU oracle can consume what it returns without sharing any code.

The paper measures on a public collection of about 1,600 matrices (Section 4.1,
Table 2) that is not available here; the generators below stand in for it:

* 2D/3D finite-difference stencils (natural x-fastest order, Dirichlet
  boundaries, no wrap) resemble the "first group" of Table 6 (at most six or a
  few dozen nonzeros per row, regular pattern) and the largest set members;
* a Zipf row-length matrix with uniform random columns resembles the "second
  group" of Table 6 (mean row length around 5-7, a few rows with tens of
  thousands of nonzeros);
* the batched set of banded matrices with n between 100 and 20,000 straddles
  the paper's small/large split at 10,000 rows.

Every CSR matrix follows the paper's CSR convention (Section 3.1): row pointers
(int64, n+1 entries, last = nnz), column indices (int32) strictly ascending
within each row, values (float64 or float32).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    """A CSR matrix as plain numpy arrays (Section 3.1)."""

    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int64 [n_rows + 1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 or float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1]) if self.row_ptr.size else 0

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def astype(self, dtype) -> "CSR":
        return CSR(self.n_rows, self.n_cols, self.row_ptr, self.col,
                   self.val.astype(dtype))


# ----------------------------------------------------------------------------
# Stencils
# ----------------------------------------------------------------------------
def _stencil(shape: tuple[int, ...], offsets: list[tuple[int, ...]],
             diag: float, off: float, dtype=np.float64) -> CSR:
    """Finite-difference stencil on a grid with x fastest.

    ``offsets`` lists neighbour displacements per axis, ordered (z, y, x) for
    3D and (y, x) for 2D.  Entries whose neighbour lies outside the grid are
    dropped (Dirichlet boundary).  The centre entry gets ``diag``, every other
    entry ``off``.
    """
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[d + 1:])) for d in range(dims)]
    # Sort offsets by linear displacement so columns come out ascending.
    offs = sorted(offsets, key=lambda o: sum(o[d] * strides[d] for d in range(dims)))
    coords = np.indices(shape, dtype=np.int32).reshape(dims, n)
    cols = np.empty((n, len(offs)), dtype=np.int32)
    mask = np.ones((n, len(offs)), dtype=bool)
    vals = np.empty(len(offs), dtype=np.float64)
    lin = np.arange(n, dtype=np.int64)
    for k, o in enumerate(offs):
        ok = np.ones(n, dtype=bool)
        for d in range(dims):
            c = coords[d] + o[d]
            ok &= (c >= 0) & (c < shape[d])
        mask[:, k] = ok
        disp = sum(o[d] * strides[d] for d in range(dims))
        cols[:, k] = (lin + disp).astype(np.int32) if n else 0
        vals[k] = diag if all(v == 0 for v in o) else off
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask]
    val = np.broadcast_to(vals, (n, len(offs)))[mask].astype(dtype)
    return CSR(n, n, row_ptr, np.ascontiguousarray(col, dtype=np.int32), val)


def laplacian_2d_5pt(N: int, diag: float = 4.0, off: float = -1.0, dtype=np.float64) -> CSR:
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    return _stencil((N, N), offs, diag, off, dtype)


def laplacian_3d_7pt(N: int, diag: float = 6.0, off: float = -1.0, dtype=np.float64) -> CSR:
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _stencil((N, N, N), offs, diag, off, dtype)


def stencil_3d_27pt(N: int, diag: float = 27.0, off: float = -1.0, dtype=np.float64) -> CSR:
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    return _stencil((N, N, N), offs, diag, off, dtype)


def stencil_3d_27pt_spd(N: int, seed: int, spread: float = 0.25) -> CSR:
    """27-point pattern on N^3 with values that are not exact in BF16/FP16:
    each off-diagonal pair a_ij = a_ji = -(1 + spread * u), u ~ U[0, 1) drawn
    per stored entry above the diagonal in CSR order; the diagonal is 1 plus
    the row's sum of |a_ij| (float64), so the matrix is symmetric and strictly
    diagonally dominant with eigenvalues >= 1 (Gershgorin): SPD."""
    A = stencil_3d_27pt(N)
    n = A.n_rows
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    cols = A.col.astype(np.int64)
    upper = cols > rows
    val = np.empty(A.nnz, dtype=np.float64)
    val[upper] = -(1.0 + spread * np.random.default_rng(seed).uniform(size=int(upper.sum())))
    # a lower entry (i, j), j < i, takes the value of the upper entry (j, i);
    # upper keys j * n + i are ascending in CSR order
    ukey = rows[upper] * n + cols[upper]
    lower = cols < rows
    val[lower] = val[upper][np.searchsorted(ukey, cols[lower] * n + rows[lower])]
    offd = ~(upper | lower)
    val[offd] = 1.0 + np.bincount(rows[~offd], weights=np.abs(val[~offd]), minlength=n)
    return CSR(n, n, A.row_ptr, A.col, val)


# ----------------------------------------------------------------------------
# Random-pattern matrices
# ----------------------------------------------------------------------------
def _unique_sorted_columns(rng: np.random.Generator, row_len: np.ndarray,
                           lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Per row r, draw row_len[r] distinct columns uniformly in [lo[r], hi[r]),
    then sort them.  Duplicates are redrawn until every row is unique."""
    nnz = int(row_len.sum())
    rows = np.repeat(np.arange(row_len.size, dtype=np.int64), row_len)
    lo_e = lo[rows].astype(np.int64)
    span = (hi - lo)[rows].astype(np.int64)
    if nnz == 0:
        return np.zeros(0, dtype=np.int32)
    cols = lo_e + rng.integers(0, span, size=nnz, dtype=np.int64)
    big = int(max(1, int(hi.max()) if hi.size else 1)) + 1
    while True:
        key = rows * big + cols
        order = np.argsort(key, kind="stable")
        cols = cols[order]
        lo_e = lo_e[order]
        span = span[order]
        key = key[order]
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        cols[dup] = lo_e[dup] + rng.integers(0, span[dup], size=dup.size, dtype=np.int64)
    return cols.astype(np.int32)


def zipf_matrix(n: int = 1_000_000, alpha: float = 2.0, max_len: int = 10_000,
                seed: int = 1, dtype=np.float32) -> CSR:
    """Square matrix with Zipf(alpha) row lengths clipped to [1, max_len],
    columns uniform without replacement per row, values N(0,1) drawn in float64
    and rounded to ``dtype``."""
    rng = np.random.default_rng(seed)
    lens = np.clip(rng.zipf(alpha, size=n), 1, min(max_len, n)).astype(np.int64)
    cols = _unique_sorted_columns(rng, lens, np.zeros(n, np.int64), np.full(n, n, np.int64))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    vals = rng.standard_normal(int(row_ptr[-1])).astype(dtype)
    return CSR(n, n, row_ptr, cols, vals)


def banded_poisson_matrix(n: int, mean_len: float, half_band: int,
                          rng: np.random.Generator, dtype=np.float32) -> CSR:
    """Square matrix whose row i has Poisson(mean_len) nonzeros (clipped to the
    window size), columns uniform without replacement in
    [max(0, i-half_band), min(n-1, i+half_band)]; values N(0,1)."""
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - half_band)
    hi = np.minimum(n - 1, i + half_band) + 1
    lens = np.minimum(rng.poisson(mean_len, size=n), hi - lo).astype(np.int64)
    cols = _unique_sorted_columns(rng, lens, lo, hi)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    vals = rng.standard_normal(int(row_ptr[-1])).astype(dtype)
    return CSR(n, n, row_ptr, cols, vals)


def batched_set(count: int = 4096, n_lo: int = 100, n_hi: int = 20_000,
                mean_lo: float = 8.0, mean_hi: float = 40.0, half_band: int = 500,
                seed: int = 4, dtype=np.float32) -> list[CSR]:
    """Independent banded matrices with log-uniform sizes (one child seed per
    matrix, spawned from ``seed``)."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for ss in children:
        rng = np.random.default_rng(ss)
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        mu = float(rng.uniform(mean_lo, mean_hi))
        out.append(banded_poisson_matrix(n, mu, half_band, rng, dtype))
    return out


def permute_symmetric(A: CSR, perm: np.ndarray) -> CSR:
    """Rows and columns renumbered by perm (perm[new] = old): A'[i, j] =
    A[perm[i], perm[j]], columns ascending within each row."""
    n = A.n_rows
    assert A.n_cols == n and len(perm) == n
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n, dtype=np.int64)
    lens = np.diff(A.row_ptr)[perm]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    src = np.arange(A.nnz, dtype=np.int64) + np.repeat(A.row_ptr[perm] - row_ptr[:-1], lens)
    new_col = inv[A.col[src]]
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    order = np.lexsort((new_col, rows))
    return CSR(n, n, row_ptr, new_col[order].astype(np.int32), A.val[src][order])


def scrambled(A: CSR, seed: int) -> tuple[CSR, np.ndarray]:
    """A under a seeded random symmetric permutation (a matrix with the same
    structure and no index locality), with that permutation."""
    perm = np.random.default_rng(seed).permutation(A.n_rows).astype(np.int32)
    return permute_symmetric(A, perm), perm


def random_csr(n_rows: int, n_cols: int, seed: int, max_len: int | None = None,
               empty_frac: float = 0.1, long_rows: int = 0, long_len: int | None = None,
               dtype=np.float64, values: str = "normal") -> CSR:
    """Small random CSR for tests: uniform row lengths in [0, max_len] with a
    fraction of empty rows and optionally a few long rows."""
    rng = np.random.default_rng(seed)
    if max_len is None:
        max_len = min(n_cols, 12)
    max_len = min(max_len, n_cols)
    lens = rng.integers(0, max_len + 1, size=n_rows).astype(np.int64)
    if n_rows:
        lens[rng.random(n_rows) < empty_frac] = 0
    if long_rows and n_rows:
        ll = min(n_cols, long_len if long_len is not None else n_cols)
        idx = rng.choice(n_rows, size=min(long_rows, n_rows), replace=False)
        lens[idx] = ll
    cols = _unique_sorted_columns(rng, lens, np.zeros(n_rows, np.int64),
                                  np.full(n_rows, n_cols, np.int64))
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if values == "normal":
        vals = rng.standard_normal(nnz)
    elif values == "int":
        vals = rng.integers(-4, 5, size=nnz).astype(np.float64)
    else:
        raise ValueError(values)
    return CSR(n_rows, n_cols, row_ptr, cols, vals.astype(dtype))


def csr_from_dense(a: np.ndarray) -> CSR:
    """CSR holding exactly the nonzero entries of a dense 2D array."""
    a = np.asarray(a)
    n_rows, n_cols = a.shape
    mask = a != 0
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=row_ptr[1:])
    r, c = np.nonzero(mask)
    return CSR(n_rows, n_cols, row_ptr, c.astype(np.int32), a[r, c].copy())


def identity(n: int, dtype=np.float64) -> CSR:
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
               np.ones(n, dtype=dtype))


def diagonal(d: np.ndarray) -> CSR:
    n = d.size
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), d.copy())


# ----------------------------------------------------------------------------
# Vectors
# ----------------------------------------------------------------------------
def uniform_vector(n: int, seed: int, dtype=np.float64, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """x ~ U[lo, hi) drawn in float64, rounded to ``dtype``."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n).astype(dtype)


def normal_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


def uniform_matrix(n: int, k: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Row-major n x k block of right-hand sides, U[-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, k)).astype(dtype)


# ----------------------------------------------------------------------------
# The named workloads (seeds are part of the recipe)
# ----------------------------------------------------------------------------
SEEDS = {
    "laplace2d_x": 1012,
    "laplace3d_x": 2270,
    "zipf_matrix": 1,
    "zipf_x": 2,
    "spmm_X": 3,
    "batched": 4,
    "grad_x": 5,
    "grad_b": 6,
    "grad_samples": 7,
    "cg_spd": 8,
}


def workload_laplace2d():
    """2D 5-point Laplacian on 64x64 (n = 4,096), float64 values 4 / -1."""
    A = laplacian_2d_5pt(64)
    x = uniform_vector(A.n_cols, SEEDS["laplace2d_x"], np.float64)
    return A, x


def workload_laplace3d(N: int = 128):
    """3D 7-point Laplacian on N^3 (n = 2,097,152 at N = 128), float32 values 6 / -1."""
    A = laplacian_3d_7pt(N, dtype=np.float32)
    x = uniform_vector(A.n_cols, SEEDS["laplace3d_x"], np.float32)
    return A, x


def workload_zipf(n: int = 1_000_000):
    """Zipf(2.0) row lengths clipped to [1, 10,000], n = 1,000,000, float32."""
    A = zipf_matrix(n, 2.0, 10_000, SEEDS["zipf_matrix"], np.float32)
    x = uniform_vector(A.n_cols, SEEDS["zipf_x"], np.float32)
    return A, x

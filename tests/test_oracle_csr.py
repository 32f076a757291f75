"""Pins for the oracle's CSR routines against facts that do not come from the
oracle itself: dense brute force, scipy, closed forms of the stencils."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1012_2270_amd import workloads as W


def dense_of(A) -> np.ndarray:
    M = np.zeros((A.n_rows, A.n_cols), dtype=np.float64)
    for i in range(A.n_rows):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            M[i, A.col[k]] = float(A.val[k])
    return M


def dense_matvec_serial(M: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Sum over every column in ascending order starting from 0.0; the extra
    terms a_ij * x_j with a_ij = 0 are exact zeros and do not move a partial
    sum, so the result equals the sparse serial sum bit for bit (up to the
    sign of zero)."""
    y = np.zeros(M.shape[0])
    for i in range(M.shape[0]):
        acc = 0.0
        for j in range(M.shape[1]):
            acc += M[i, j] * x[j]
        y[i] = acc
    return y


CASES = [
    dict(n_rows=0, n_cols=0),
    dict(n_rows=1, n_cols=1),
    dict(n_rows=7, n_cols=5),
    dict(n_rows=33, n_cols=40, empty_frac=0.3),
    dict(n_rows=64, n_cols=64, long_rows=2),
    dict(n_rows=65, n_cols=17, max_len=17),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spmv_equals_dense_brute_force(oracle, case, seed):
    A = W.random_csr(seed=seed, **case)
    x = np.random.default_rng(100 + seed).uniform(-1, 1, A.n_cols)
    y = oracle.csr_spmv(A, x)
    ref = dense_matvec_serial(dense_of(A), x)
    np.testing.assert_array_equal(y + 0.0, ref + 0.0)


def test_spmv_signed_zero_and_subnormal_inputs(oracle):
    tiny = np.nextafter(0.0, 1.0)
    M = np.array([[-0.0, 2.0, tiny], [tiny, 0.0, -tiny], [1e-300, 1e-300, 0.0]])
    A = W.csr_from_dense(M)
    # csr_from_dense drops the -0.0 entry (it compares equal to 0); add it back
    A = W.CSR(3, 3, np.array([0, 3, 5, 7]), np.array([0, 1, 2, 0, 2, 0, 1], np.int32),
              np.array([-0.0, 2.0, tiny, tiny, -tiny, 1e-300, 1e-300]))
    x = np.array([3.0, -0.5, 0.25])
    y = oracle.csr_spmv(A, x)
    ref = dense_matvec_serial(dense_of(A), x)
    np.testing.assert_array_equal(y + 0.0, ref + 0.0)


@pytest.mark.parametrize("seed", [3, 4])
def test_spmv_matches_scipy(oracle, seed):
    A = W.random_csr(500, 300, seed=seed, max_len=40, long_rows=3)
    x = np.random.default_rng(seed).standard_normal(A.n_cols)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    y = oracle.csr_spmv(A, x)
    s = oracle.csr_absmv(A, x)
    assert oracle.scaled_error(y, S @ x, s) <= 1e-15


def test_absmv_matches_dense(oracle):
    A = W.random_csr(40, 50, seed=9)
    x = np.random.default_rng(9).standard_normal(50)
    s = oracle.csr_absmv(A, x)
    ref = dense_matvec_serial(np.abs(dense_of(A)), np.abs(x))
    np.testing.assert_array_equal(s, ref)


def test_identity_and_diagonal_closed_forms(oracle):
    x = np.random.default_rng(5).standard_normal(1000)
    np.testing.assert_array_equal(oracle.csr_spmv(W.identity(1000), x), x)
    d = np.random.default_rng(6).standard_normal(1000)
    np.testing.assert_array_equal(oracle.csr_spmv(W.diagonal(d), x), d * x)
    # float32 inputs: the oracle upcasts exactly, so d*x in f64 rounded to f32
    # is the single correctly rounded f32 product
    d32, x32 = d.astype(np.float32), x.astype(np.float32)
    y = oracle.csr_spmv(W.diagonal(d32), x32).astype(np.float32)
    np.testing.assert_array_equal(y, d32 * x32)


def _neighbour_count(shape, kind):
    idx = np.indices(shape).reshape(len(shape), -1)
    if kind == "star":
        deg = np.zeros(idx.shape[1], np.int64)
        for d, N in enumerate(shape):
            deg += (idx[d] > 0).astype(np.int64) + (idx[d] < N - 1).astype(np.int64)
        return deg
    # box: product over axes of valid positions among {i-1, i, i+1}, minus the centre
    m = np.ones(idx.shape[1], np.int64)
    for d, N in enumerate(shape):
        m *= 1 + (idx[d] > 0).astype(np.int64) + (idx[d] < N - 1).astype(np.int64)
    return m - 1


def test_laplacian_times_ones_closed_forms(oracle):
    # 5-point: 4 - (number of neighbours): 0 inside, 1 on edges, 2 in corners
    A = W.laplacian_2d_5pt(64)
    y = oracle.csr_spmv(A, np.ones(A.n_cols))
    np.testing.assert_array_equal(y, 4.0 - _neighbour_count((64, 64), "star"))
    assert set(np.unique(y)) == {0.0, 1.0, 2.0}
    # 7-point with diagonal 6
    A = W.laplacian_3d_7pt(12)
    y = oracle.csr_spmv(A, np.ones(A.n_cols))
    np.testing.assert_array_equal(y, 6.0 - _neighbour_count((12, 12, 12), "star"))
    # 27-point with diagonal 27: 28 - prod_d m_d
    A = W.stencil_3d_27pt(9)
    y = oracle.csr_spmv(A, np.ones(A.n_cols))
    np.testing.assert_array_equal(y, 27.0 - _neighbour_count((9, 9, 9), "box"))


def test_stencil_nnz_closed_forms():
    assert W.laplacian_2d_5pt(64).nnz == 64 * 64 + 4 * 64 * 63 == 20_224
    N = 20
    assert W.laplacian_3d_7pt(N).nnz == N ** 3 + 6 * N * N * (N - 1)
    assert W.stencil_3d_27pt(11).nnz == (3 * 11 - 2) ** 3


def test_spmm_column_by_column_equals_dense(oracle):
    A = W.random_csr(50, 30, seed=11, max_len=10)
    X = np.random.default_rng(11).standard_normal((30, 4))
    Y = oracle.csr_spmm(A, X)
    M = dense_of(A)
    for c in range(4):
        np.testing.assert_array_equal(Y[:, c] + 0.0, dense_matvec_serial(M, X[:, c]) + 0.0)


def test_csr_check_codes(oracle):
    rp = np.array([0, 2, 3])
    col = np.array([0, 2, 1], np.int32)
    assert oracle.csr_check(2, 3, 3, rp, col) == 0
    assert oracle.csr_check(2, 3, 3, np.array([1, 2, 3]), col) == 1
    assert oracle.csr_check(2, 3, 3, np.array([0, 3, 2]), col) == 2
    assert oracle.csr_check(2, 3, 4, rp, col) == 3
    assert oracle.csr_check(2, 2, 3, rp, col) == 4
    assert oracle.csr_check(2, 3, 3, rp, np.array([2, 0, 1], np.int32)) == 5
    assert oracle.csr_check(2, 3, 3, rp, np.array([1, 1, 1], np.int32)) == 5  # duplicate


def test_transpose_matches_dense(oracle):
    A = W.random_csr(37, 23, seed=12, max_len=9)
    rpT, colT, valT = oracle.csr_transpose(A)
    AT = W.CSR(23, 37, rpT, colT, valT)
    np.testing.assert_array_equal(dense_of(AT), dense_of(A).T)
    assert oracle.csr_check(23, 37, A.nnz, rpT, colT) == 0


def test_adjoint_dot_product_identity(oracle):
    A = W.random_csr(300, 200, seed=13, max_len=20)
    x = np.random.default_rng(1).standard_normal(200)
    y = np.random.default_rng(2).standard_normal(300)
    rpT, colT, valT = oracle.csr_transpose(A)
    ATy = oracle.csr_spmv(W.CSR(200, 300, rpT, colT, valT), y)
    lhs = float(np.dot(oracle.csr_spmv(A, x), y))
    rhs = float(np.dot(x, ATy))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


# ---------------------------------------------------------------------------
# The tolerance judge: e = max_i |y_i - y_ref_i| / max_i s_i, with e = 0 or inf
# when every s_i is zero.  Every expected value below is worked out by hand.
# ---------------------------------------------------------------------------
def test_scaled_error_hand_cases(oracle):
    # largest difference 0.5 sits at row 1, largest s (4.0) also at row 1:
    # e = 0.5 / 4 = 0.125.  Dividing by the sum of s (7) gives 0.0714...,
    # averaging the differences (0.5 / 3) gives 0.0416...
    assert oracle.scaled_error([1.0, 2.0, 3.0], [1.0, 2.5, 3.0], [1.0, 4.0, 2.0]) == 0.125
    # largest difference (0.75, row 0) is not at the row of largest s (8.0, row 2):
    # e = 0.75 / 8 = 0.09375; taking s at the row of the largest difference
    # (1.0) would give 0.75, the mean of the differences 0.3125 / 8
    assert oracle.scaled_error([0.75, 1.0, 1.0], [0.0, 1.0, 0.875], [1.0, 2.0, 8.0]) == 0.09375
    # differences of both signs: |-0.25| is the largest; e = 0.25 / 2
    assert oracle.scaled_error([-1.25, 0.5], [-1.0, 0.625], [2.0, 0.5]) == 0.125
    # identical vectors
    assert oracle.scaled_error([3.0, -2.0], [3.0, -2.0], [5.0, 1.0]) == 0.0


def test_scaled_error_zero_scale(oracle):
    # every s_i = 0 (e.g. x = 0): y must be exactly zero
    assert oracle.scaled_error([0.0, -0.0], [0.0, 0.0], [0.0, 0.0]) == 0.0
    assert oracle.scaled_error([0.0, 1e-300], [0.0, 0.0], [0.0, 0.0]) == float("inf")
    assert oracle.scaled_error([], [], []) == 0.0


def test_scaled_error_nan_fails_every_tolerance(oracle):
    e = oracle.scaled_error([1.0, float("nan")], [1.0, 2.0], [1.0, 1.0])
    assert not (e <= 1e-5)
    e = oracle.scaled_error([float("nan")], [0.0], [0.0])
    assert not (e <= 1e-5)
    # an infinite result against a finite reference is an infinite error
    assert oracle.scaled_error([float("inf")], [1.0], [1.0]) == float("inf")


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_spmv_bit_identical_to_serial(oracle, threads):
    """Row partition over threads changes no row's summation order."""
    A = W.random_csr(5000, 4000, seed=11, max_len=50, empty_frac=0.1, long_rows=4, long_len=3000)
    x = np.random.default_rng(11).standard_normal(A.n_cols)
    np.testing.assert_array_equal(oracle.csr_spmv_parallel(A, x, threads).view(np.uint64),
                                  oracle.csr_spmv(A, x).view(np.uint64))

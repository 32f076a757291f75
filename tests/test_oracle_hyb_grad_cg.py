"""Pins for the oracle's Hybrid ELL+COO, gradient and CG routines."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_1012_2270_amd import workloads as W


def k1_by_marginal_rule(lens, s_v, c=3):
    """The Hybrid cost is convex in k (the number of rows longer than k never
    grows with k), so the minimiser is the first k at which one more ELL
    column costs at least what it saves in COO entries."""
    n_pad = (len(lens) + 63) // 64 * 64
    k = 0
    while True:
        longer = int((lens > k).sum())
        if longer == 0 or c * (s_v + 8) * longer <= n_pad * (s_v + 4):
            return k
        k += 1


@pytest.mark.parametrize("mk", [
    lambda: W.laplacian_3d_7pt(24),
    lambda: W.laplacian_2d_5pt(40),
    lambda: W.random_csr(3000, 3000, seed=2, max_len=30, long_rows=10, long_len=900),
    lambda: W.zipf_matrix(20_000, seed=5),
])
@pytest.mark.parametrize("s_v", [4, 8])
def test_k1_rule_against_marginal_criterion(oracle, mk, s_v):
    A = mk()
    assert oracle.hyb_k1(A, s_v) == k1_by_marginal_rule(np.diff(A.row_ptr), s_v)


def test_k1_stencil_and_zipf_values(oracle):
    # every interior row of the 7-point stencil has 7 nonzeros
    assert oracle.hyb_k1(W.laplacian_3d_7pt(64), 4) == 7
    # Zipf(2): P(len > k) = 0.39, 0.24, 0.17 for k = 1, 2, 3; an extra ELL
    # column pays for itself while 36 * P(len > k) > 8, i.e. up to k = 3
    assert oracle.hyb_k1(W.zipf_matrix(200_000, seed=3), 4) == 3


@pytest.mark.parametrize("K1", [0, 1, 3, 7, 40])
def test_hybrid_round_trip_and_serial_sum(oracle, K1):
    A = W.random_csr(150, 80, seed=K1, max_len=25, long_rows=2)
    H = oracle.hyb_layout(A, K1)
    # decode: ELL row i then its COO entries
    ell_c = H["ell_col"].reshape(max(K1, 0), H["n_pad"]) if K1 else np.zeros((0, H["n_pad"]), np.int32)
    ell_v = H["ell_val"].reshape(ell_c.shape)
    cols, vals = [[] for _ in range(A.n_rows)], [[] for _ in range(A.n_rows)]
    for i in range(A.n_rows):
        for j in range(K1):
            if ell_c[j, i] >= 0:
                cols[i].append(ell_c[j, i])
                vals[i].append(ell_v[j, i])
    for e in range(H["coo_nnz"]):
        cols[H["coo_row"][e]].append(H["coo_col"][e])
        vals[H["coo_row"][e]].append(H["coo_val"][e])
    np.testing.assert_array_equal(np.concatenate([np.array(c, np.int32) for c in cols]), A.col)
    np.testing.assert_array_equal(np.concatenate([np.array(v) for v in vals]), A.val)
    # padding rows beyond n and padding slots
    assert (ell_c[:, A.n_rows:] == -1).all()
    x = np.random.default_rng(K1).standard_normal(A.n_cols)
    np.testing.assert_array_equal(oracle.hyb_spmv(H, x), oracle.csr_spmv(A, x))


def test_gradient_central_differences_exact_for_quadratic(oracle):
    """L(theta) = 1/2 ||A(theta) x - b||^2 is quadratic in each theta_k and
    each x_j, so the central difference has no truncation term."""
    A = W.random_csr(60, 50, seed=4, max_len=8)
    rng = np.random.default_rng(0)
    x, b = rng.standard_normal(50), rng.standard_normal(60)
    r, dx, dval, L = oracle.adjoint(A, x, b)
    h = 1e-3
    for k in rng.choice(A.nnz, 20, replace=False):
        Ap = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
        Am = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.copy())
        Ap.val[k] += h
        Am.val[k] -= h
        fd = (oracle.loss(Ap, x, b) - oracle.loss(Am, x, b)) / (2 * h)
        assert abs(fd - dval[k]) <= 1e-8 * max(1.0, abs(dval[k]))
    for j in rng.choice(50, 20, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (oracle.loss(A, xp, b) - oracle.loss(A, xm, b)) / (2 * h)
        assert abs(fd - dx[j]) <= 1e-8 * max(1.0, abs(dx[j]))


def test_gradient_matches_torch_autograd(oracle):
    import torch
    A = W.random_csr(40, 30, seed=8, max_len=7)
    rng = np.random.default_rng(1)
    x, b = rng.standard_normal(30), rng.standard_normal(40)
    r, dx, dval, L = oracle.adjoint(A, x, b)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    th = torch.tensor(A.val, dtype=torch.float64, requires_grad=True)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    M = torch.zeros(40, 30, dtype=torch.float64).index_put(
        (torch.tensor(rows), torch.tensor(A.col.astype(np.int64))), th)
    loss = 0.5 * ((M @ xt - torch.tensor(b)) ** 2).sum()
    loss.backward()
    np.testing.assert_allclose(th.grad.numpy(), dval, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(xt.grad.numpy(), dx, rtol=1e-13, atol=1e-13)
    assert abs(loss.item() - L) <= 1e-13 * L


def test_cg_reaches_closed_form_solution(oracle):
    """b = A 1 is exact in FP64 for the 27-point stencil (integers), so the
    solution is the vector of ones."""
    A = W.stencil_3d_27pt(10)
    b = oracle.csr_spmv(A, np.ones(A.n_cols))
    x, it, rel = oracle.cg(A, b, tol=1e-12)
    assert rel <= 1e-11
    assert np.max(np.abs(x - 1.0)) <= 1e-9
    # kappa of this operator is below 37, so CG needs well under 100 steps
    assert it < 100
    # library cross-check
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    xs = spla.spsolve(S.tocsc(), b)
    assert np.max(np.abs(x - xs)) <= 1e-9


def test_k1_tie_goes_to_smallest_width(oracle):
    """n = 576 rows, 128 of length 2, the rest of length 1, s_v = 4, c = 3:
    a second ELL column costs 8 * 576 = 4608 bytes and saves 36 * 128 = 4608,
    an exact tie, which the rule breaks towards the narrower ELL."""
    lens = np.ones(576, np.int64)
    lens[::4][:128] = 2
    assert int((lens == 2).sum()) == 128
    rp = np.zeros(577, np.int64)
    rp[1:] = np.cumsum(lens)
    A = W.CSR(576, 4, rp, np.concatenate([np.arange(l) for l in lens]).astype(np.int32),
              np.ones(rp[-1]))
    assert oracle.hyb_k1(A, 4) == 1


def test_cg_on_values_that_16_bit_storage_rounds(oracle):
    """The SPD 27-point matrix with perturbed values (the mixed-precision CG
    case whose values BF16/FP16 round): exactly symmetric, eigenvalues >= 1,
    and the oracle's CG agrees with a direct solve."""
    A = W.stencil_3d_27pt_spd(8, seed=3)
    S = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    D = S.toarray()
    assert np.array_equal(D, D.T)
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= 1.0 - 1e-12
    # the values are not all exact in bfloat16 (8 significant bits)
    assert np.any(oracle.to_f64(oracle.round_values(A.val.astype(np.float32), "bf16"), bf16_bits=True) != A.val)
    # every row sums to 1: the ones vector is an eigenvector (eigenvalue 1)
    np.testing.assert_allclose(D.sum(axis=1), 1.0, rtol=0, atol=1e-13)
    xstar = np.random.default_rng(4).uniform(-1, 1, A.n_cols)
    b = oracle.csr_spmv(A, xstar)
    x, it, rel = oracle.cg(A, b, tol=1e-12)
    assert rel <= 1e-12 and it > 10
    xs = spla.spsolve(S.tocsc(), b)
    assert np.max(np.abs(x - xs)) <= 1e-10
    assert np.max(np.abs(x - xstar)) <= 1e-10

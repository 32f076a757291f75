"""Seeded random draws over the layout and schedule options: every accepted
combination of group size, lanes per row, sort window, long-row threshold,
storage and vector dtype, rows per lane, load mode, load policy and
right-hand-side count gives the oracle's layout arrays bit for bit and an SpMV
(or SpMM) within tolerance of the FP64 oracle; combinations the library does
not run are refused with RGCSR_EUNSUPPORTED."""
import numpy as np
import pytest

from gpu_util import TOL_F32, TOL_F64, dev, host, say, storage_values

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W

pytestmark = pytest.mark.gpu

INDEX_ARRAYS = ("gp", "short_len", "short_row", "slot_col", "long_row", "long_ptr", "long_col")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg._lib.load()
    return torch


def draw(rng):
    T = int(rng.choice([1, 1, 2, 4, 8]))
    G = int(rng.choice([g for g in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)
                        if (g * T) % 64 == 0 or 64 % (g * T) == 0]))
    vd = str(rng.choice(["f32", "f32", "f64", "bf16", "f16"]))
    vec = "f64" if vd == "f64" else ("f64" if vd == "f32" and rng.random() < 0.3 else "f32")
    return dict(G=G, T=T, sigma=int(rng.choice([1, 7, 64, 1000, 1 << 40])), tau=int(rng.choice([-1, 0, 3, 16, 100])),
                value_dtype=vd, rows_per_lane=int(rng.choice([0, 1, 2, 4, 8])),
                pad_loads=int(rng.choice([-1, 0, 1, 2, 3])), load_policy=int(rng.choice([0, 0, 0, 0, 1, 2]))), vec


@pytest.mark.parametrize("seed", range(40))
def test_random_layout_and_schedule(torch_cuda, oracle, seed):
    torch = torch_cuda
    rng = np.random.default_rng(5000 + seed)
    n_rows, n_cols = int(rng.integers(1, 4000)), int(rng.integers(1, 4000))
    A = W.random_csr(n_rows, n_cols, seed=seed, max_len=int(rng.integers(1, min(n_cols, 80) + 1)),
                     empty_frac=float(rng.choice([0.0, 0.05, 0.3])), long_rows=int(rng.integers(0, 4)),
                     long_len=int(rng.integers(1, n_cols + 1)), dtype=np.float32)
    kw, vec = draw(rng)
    say("random layout", seed, n_rows, n_cols, A.nnz, kw, vec)
    try:
        M = rg.rgcsr_from_csr(A, **kw)
    except rg.RgcsrError as e:
        # refused only where documented: sliced ELLPACK / column-derived
        # lengths outside their geometry, or a load policy outside F32 / T = 1
        assert e.status == 6, str(e)
        assert kw["pad_loads"] in (2, 3) or kw["load_policy"] != 0, str(e)
        return
    G, T, sigma, tau = kw["G"], kw["T"], kw["sigma"], kw["tau"]
    exp = oracle.rgcsr_layout(A, G, T, sigma, tau)
    got = M.export()
    for k in INDEX_ARRAYS:
        np.testing.assert_array_equal(got[k], exp[k], err_msg=k)
    vd = kw["value_dtype"]
    if vd == "f32":
        for k in ("slot_val", "long_val"):
            np.testing.assert_array_equal(got[k].view(np.uint8), exp[k].view(np.uint8), err_msg=k)
    vals64 = storage_values(oracle, A, vd) if vd in ("bf16", "f16") else None
    B = A if vals64 is None else W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals64)
    tol = TOL_F64 if vec == "f64" else TOL_F32
    npdt = np.float64 if vec == "f64" else np.float32
    x = W.uniform_vector(A.n_cols, seed + 1, npdt)
    if kw["load_policy"] != 0 and vec == "f64":
        with pytest.raises(rg.RgcsrError) as e:
            M.spmv(dev(x))
        assert e.value.status == 6
        return
    y = host(M.spmv(dev(x)))
    assert oracle.scaled_error(y, oracle.csr_spmv(B, x), oracle.csr_absmv(B, x)) <= tol
    if kw["load_policy"] == 0:
        k = int(rng.choice([2, 4, 8, 16, 32]))
        X = W.uniform_matrix(A.n_cols, k, seed=seed + 2, dtype=npdt)
        Y = host(M.spmm(dev(X)))
        ref = oracle.csr_spmm(B, X)
        for c in range(k):
            assert oracle.scaled_error(Y[:, c], ref[:, c], oracle.csr_absmv(B, X[:, c])) <= tol, c
    M.close()
    del torch


@pytest.mark.parametrize("seed", range(16))
def test_random_batch_and_backward(torch_cuda, oracle, seed):
    """Seeded draws of small batches (per-matrix y within tolerance) and of
    the backward pass and value update on one matrix (dvals bit-exact to the
    rounded products, dx within tolerance, updated values bit-exact against
    a fresh conversion)."""
    torch = torch_cuda
    rng = np.random.default_rng(7000 + seed)
    kw, _ = draw(rng)
    kw["value_dtype"] = "f32"
    kw["load_policy"] = 0
    if kw["pad_loads"] in (2, 3):
        kw["pad_loads"] = -1
    mats = [W.random_csr(int(rng.integers(1, 900)), int(rng.integers(1, 900)), seed=100 * seed + m,
                         max_len=int(rng.integers(1, 40)), empty_frac=float(rng.choice([0.0, 0.2])),
                         long_rows=int(rng.integers(0, 3)), long_len=int(rng.integers(1, 600)), dtype=np.float32)
            for m in range(int(rng.integers(1, 9)))]
    say("random batch", seed, [(M.n_rows, M.n_cols, M.nnz) for M in mats], kw)
    B = rg.rgcsr_from_csr_batch(mats, **kw)
    ro, co = B.batch_offsets()
    x = W.uniform_vector(int(co[-1]), seed + 3, np.float32)
    y = host(B.spmv(dev(x)))
    for i, M in enumerate(mats):
        xi = x[co[i]:co[i + 1]]
        assert oracle.scaled_error(y[ro[i]:ro[i + 1]], oracle.csr_spmv(M, xi), oracle.csr_absmv(M, xi)) <= TOL_F32, i
    B.close()
    A = mats[0]
    transpose = bool(rng.random() < 0.5)
    say("random backward", seed, A.n_rows, A.n_cols, A.nnz, transpose)
    M = rg.rgcsr_from_csr(A, keep_csr_map=True, build_transpose=transpose, **kw)
    xa = W.normal_vector(A.n_cols, seed + 4, np.float32)
    dy = dev(W.normal_vector(A.n_rows, seed + 5, np.float32))
    dx = torch.empty(A.n_cols, device="cuda:0")
    dv = torch.empty(max(1, A.nnz), device="cuda:0")
    rg.rgcsr_spmv_transpose_grad(M, dev(xa), dy, dx, dv)
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    exact = (host(dy)[rows] * xa[A.col]).astype(np.float32)
    np.testing.assert_array_equal(host(dv)[:A.nnz].view(np.uint32), exact.view(np.uint32))
    AT = W.CSR(A.n_cols, A.n_rows, *oracle.csr_transpose(A))
    dyh = host(dy)
    assert oracle.scaled_error(host(dx), oracle.csr_spmv(AT, dyh), oracle.csr_absmv(AT, dyh)) <= TOL_F32
    theta = W.normal_vector(A.nnz, seed + 6, np.float32)
    if A.nnz:
        rg.rgcsr_set_values(M, dev(theta))
        exp = oracle.rgcsr_layout(W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, theta), kw["G"], kw["T"], kw["sigma"],
                                  kw["tau"])
        got = M.export()
        for k in ("slot_val", "long_val"):
            np.testing.assert_array_equal(got[k].view(np.uint32), exp[k].view(np.uint32), err_msg=k)
    M.close()


@pytest.mark.parametrize("seed", range(12))
def test_random_hybrid(torch_cuda, oracle, seed):
    """Seeded draws of the Hybrid comparison format: ELL width chosen by the
    rule or forced (0, 1, wider than every row), storage and vector dtype;
    arrays bit-exact against the oracle's Hybrid layout, SpMV within
    tolerance."""
    rng = np.random.default_rng(9000 + seed)
    n_rows, n_cols = int(rng.integers(1, 5000)), int(rng.integers(1, 5000))
    A = W.random_csr(n_rows, n_cols, seed=seed, max_len=int(rng.integers(1, min(n_cols, 60) + 1)),
                     empty_frac=float(rng.choice([0.0, 0.2])), long_rows=int(rng.integers(0, 4)),
                     long_len=int(rng.integers(1, n_cols + 1)), dtype=np.float32)
    width = int(rng.choice([-1, -1, 0, 1, 3, 200]))
    vd = str(rng.choice(["f32", "f64", "bf16"]))
    vec = "f64" if vd == "f64" else "f32"
    say("random hybrid", seed, n_rows, n_cols, A.nnz, width, vd)
    H = rg.hyb_from_csr(A, value_dtype=vd, ell_width=width)
    K1 = H.info["ell_width"]
    if width >= 0:
        assert K1 == width
    else:
        assert K1 == oracle.hyb_k1(A, {"f32": 4, "f64": 8, "bf16": 2}[vd])
    exp = oracle.hyb_layout(A, K1)
    got = rg.hyb_export(H)
    for k in ("ell_col", "coo_row", "coo_col"):
        np.testing.assert_array_equal(got[k], exp[k], err_msg=k)
    vals64 = storage_values(oracle, A, vd) if vd == "bf16" else None
    B = A if vals64 is None else W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals64)
    npdt = np.float64 if vec == "f64" else np.float32
    x = W.uniform_vector(A.n_cols, seed + 7, npdt)
    y = host(H.spmv(dev(x)))
    tol = TOL_F64 if vec == "f64" else TOL_F32
    assert oracle.scaled_error(y, oracle.csr_spmv(B, x), oracle.csr_absmv(B, x)) <= tol
    H.close()

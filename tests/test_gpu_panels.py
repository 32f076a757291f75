"""GPU parity of the column-panel copy (col_panels): the matrix split by
column into panels, each panel's pieces run on one XCD and the piece sums
added per row in panel order, against the FP64 oracle through the C ABI;
value updates, clones, the launches that stay on the layout itself, and the
degenerate splits (empty panels, empty rows, one column)."""
import numpy as np
import pytest

from gpu_util import TOL_F32, TOL_F64, check_spmv, dev, host, say, storage_values

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W

pytestmark = pytest.mark.gpu

LAY = dict(G=64, sigma=512, tau=16)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg._lib.load()
    return torch


@pytest.fixture(scope="module")
def zipf():
    A = W.zipf_matrix(60_000, seed=51)
    x = W.uniform_vector(A.n_cols, 52, np.float32)
    return A, x


def pieces(A, P, whole_max=LAY["tau"]):
    """Pieces of the panel split, counted on the host from the same rule
    (bounds at the columns where the running nonzero count reaches q*nnz/P;
    rows of at most whole_max nonzeros, empty ones included, stay whole, one
    piece each)."""
    # cnt[i]: nonzeros in the columns before column i
    cnt = np.concatenate([[0], np.bincount(A.col, minlength=A.n_cols).cumsum()])
    cb = [0]
    for q in range(1, P):
        t = (A.nnz * q + P - 1) // P
        cb.append(max(cb[-1], min(int(np.searchsorted(cnt, t)), A.n_cols)))
    cb.append(A.n_cols)
    L = np.diff(A.row_ptr)
    rows = np.repeat(np.arange(A.n_rows), L)
    pan = np.searchsorted(np.asarray(cb[1:]), A.col, side="right")
    split = np.repeat(L > whole_max, L)
    return int(np.unique(rows[split].astype(np.int64) * P + pan[split]).size) + int(np.sum(L <= whole_max))


def nan_out(torch, n, k=None, dtype=None):
    import torch as t
    shape = (n,) if k is None else (n, k)
    return t.full(shape, float("nan"), dtype=dtype or t.float32, device="cuda:0")


@pytest.mark.parametrize("P", [8, 16, 64])
@pytest.mark.parametrize("vdt", ["f32", "f64"])
def test_panel_spmm_parity_panels(torch_cuda, oracle, zipf, P, vdt):
    """Two right-hand sides on the copy, deterministic; one vector runs on the
    layout itself and gives the same bits as a handle without the copy."""
    torch = torch_cuda
    A, x = zipf
    say("panels", P, vdt)
    B = A if vdt == "f32" else W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.astype(np.float64))
    M = rg.rgcsr_from_csr(B, col_panels=P, value_dtype=vdt, **LAY)
    assert M.info["col_panels"] == P and M.info["panel_pieces"] == pieces(A, P)
    dt = torch.float32 if vdt == "f32" else torch.float64
    X = W.uniform_matrix(A.n_cols, 2, 62).astype(np.float32 if vdt == "f32" else np.float64)
    Y = nan_out(torch, A.n_rows, 2, dtype=dt)
    rg.rgcsr_spmv_batched(M, dev(X), Y)
    Yh = host(Y)
    B64 = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, B.val.astype(np.float64))
    ref = oracle.csr_spmm(B64, X.astype(np.float64))
    tol = TOL_F32 if vdt == "f32" else TOL_F64
    for c in range(2):
        assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(B64, X[:, c].astype(np.float64))) <= tol
    Y2 = nan_out(torch, A.n_rows, 2, dtype=dt)
    rg.rgcsr_spmv_batched(M, dev(X), Y2)
    np.testing.assert_array_equal(host(Y2), Yh)
    # one vector: the layout's own kernels
    M0 = rg.rgcsr_from_csr(B, value_dtype=vdt, **LAY)
    xv = x if vdt == "f32" else x.astype(np.float64)
    np.testing.assert_array_equal(host(M.spmv(dev(xv))), host(M0.spmv(dev(xv))))


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_panel_needs_f32_or_f64_values(torch_cuda, zipf, dt):
    A, _ = zipf
    say("panels refuse", dt)
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_from_csr(A, col_panels=8, value_dtype=dt, **LAY)
    assert e.value.status == 6


@pytest.mark.parametrize("tau", [-1, 0, 64])
def test_panel_whole_row_threshold(torch_cuda, oracle, zipf, tau):
    """Rows up to the long-row threshold stay whole (tau = -1: every row is
    split; tau = 0: every row with entries is split too)."""
    torch = torch_cuda
    A, x = zipf
    say("panels tau", tau)
    M = rg.rgcsr_from_csr(A, col_panels=8, G=64, sigma=512, tau=tau)
    assert M.info["panel_pieces"] == pieces(A, 8, whole_max=tau)
    y = nan_out(torch, A.n_rows)
    M.spmv(dev(x), y)
    check_spmv(oracle, A, x, host(y))
    X = W.uniform_matrix(A.n_cols, 4, 61)
    Y = nan_out(torch, A.n_rows, 4)
    rg.rgcsr_spmv_batched(M, dev(X), Y)
    Yh = host(Y)
    ref = oracle.csr_spmm(A, X)
    for c in range(4):
        assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32


@pytest.mark.parametrize("k", [2, 4, 8, 16, 5])
@pytest.mark.parametrize("persistent", [False, True])
def test_panel_spmm_parity(torch_cuda, oracle, zipf, k, persistent):
    torch = torch_cuda
    A, _ = zipf
    say("panels spmm", k, persistent)
    X = W.uniform_matrix(A.n_cols, k, 53)
    M = rg.rgcsr_from_csr(A, col_panels=8, **LAY)
    Y = nan_out(torch, A.n_rows, k)
    rg.rgcsr_spmv_batched(M, dev(X), Y, persistent=persistent)
    Yh = host(Y)
    ref = oracle.csr_spmm(A, X)
    for c in range(k):
        e = oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c]))
        assert e <= TOL_F32, (c, e)


@pytest.mark.parametrize("vdt", ["f32", "f64"])
@pytest.mark.parametrize("k", [1, 2, 4])
def test_panel_f64_vectors(torch_cuda, oracle, zipf, vdt, k):
    torch = torch_cuda
    A, _ = zipf
    say("panels f64", vdt, k)
    A64 = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.astype(np.float64))
    X = W.uniform_matrix(A.n_cols, k, 54).astype(np.float64)
    M = rg.rgcsr_from_csr(A64 if vdt == "f64" else A, col_panels=8, value_dtype=vdt, **LAY)
    Y = nan_out(torch, A.n_rows, k, dtype=torch.float64)
    rg.rgcsr_spmv_batched(M, dev(X), Y)
    Yh = host(Y)
    B = A64 if vdt == "f64" else W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val.astype(np.float64))
    ref = oracle.csr_spmm(B, X)
    for c in range(k):
        e = oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(B, X[:, c]))
        assert e <= TOL_F64, (c, e)


def test_panel_same_as_layout_within_rounding(torch_cuda, oracle, zipf):
    """The copy and the layout itself sum the split rows in different orders
    (the whole rows in the same one); both are within the FP32 bound of the
    oracle and of each other."""
    torch = torch_cuda
    A, _ = zipf
    say("panels vs layout")
    X = W.uniform_matrix(A.n_cols, 4, 63)
    M0 = rg.rgcsr_from_csr(A, **LAY)
    M1 = rg.rgcsr_from_csr(A, col_panels=8, **LAY)
    Y0, Y1 = nan_out(torch, A.n_rows, 4), nan_out(torch, A.n_rows, 4)
    rg.rgcsr_spmv_batched(M0, dev(X), Y0)
    rg.rgcsr_spmv_batched(M1, dev(X), Y1)
    Y0h, Y1h = host(Y0), host(Y1)
    L = np.diff(A.row_ptr)
    for c in range(4):
        s = oracle.csr_absmv(A, X[:, c])
        assert oracle.scaled_error(Y1h[:, c], Y0h[:, c].astype(np.float64), s) <= 2 * TOL_F32
    # a whole row is one piece summed by the same kernel path: same bits
    whole = L <= LAY["tau"]
    np.testing.assert_array_equal(Y1h[whole], Y0h[whole])


def test_panel_set_values_and_clone(torch_cuda, oracle, zipf):
    torch = torch_cuda
    A, x = zipf
    say("panels set_values clone")
    M = rg.rgcsr_from_csr(A, col_panels=8, keep_csr_map=True, **LAY)
    rng = np.random.default_rng(55)
    v2 = rng.standard_normal(A.nnz).astype(np.float32)
    B = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, v2)
    # device values (gather through the copy's CSR index map)
    rg.rgcsr_set_values(M, dev(v2))
    check_spmv(oracle, B, x, host(M.spmv(dev(x))))
    X = W.uniform_matrix(A.n_cols, 4, 56)
    Y = nan_out(torch, A.n_rows, 4)
    rg.rgcsr_spmv_batched(M, dev(X), Y)
    ref = oracle.csr_spmm(B, X)
    Yh = host(Y)
    for c in range(4):
        assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(B, X[:, c])) <= TOL_F32
    # host values in another dtype
    v3 = rng.standard_normal(A.nnz)
    C = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, v3.astype(np.float32).astype(np.float64))
    rg.rgcsr_set_values(M, v3)
    check_spmv(oracle, C, x, host(M.spmv(dev(x))))
    # a clone owns its copy: updating the original leaves the clone alone
    K = M.clone()
    assert K.info["col_panels"] == 8 and K.info["panel_pieces"] == M.info["panel_pieces"]
    yk = host(K.spmv(dev(x)))
    rg.rgcsr_set_values(M, dev(v2))
    np.testing.assert_array_equal(host(K.spmv(dev(x))).view(np.uint32), yk.view(np.uint32))
    check_spmv(oracle, C, x, yk)
    check_spmv(oracle, B, x, host(M.spmv(dev(x))))


def test_panel_launches_on_the_layout(torch_cuda, oracle):
    """X rows too wide for the slice budget (3 MiB of x per panel) run on the
    layout itself (with its column tiles); the result is the same product."""
    torch = torch_cuda
    A = W.zipf_matrix(400_000, seed=57)
    say("panels fallback", A.nnz)
    M = rg.rgcsr_from_csr(A, col_panels=8, **LAY)
    # 8 columns of X: 50,000 columns per panel * 8 * 4 bytes = 1.6 MB -> copy
    # 32 columns: 6.4 MB per panel -> layout, column blocks of up to 32
    for k in (8, 32):
        X = W.uniform_matrix(A.n_cols, k, 58)
        Y = nan_out(torch, A.n_rows, k)
        rg.rgcsr_spmv_batched(M, dev(X), Y)
        Yh = host(Y)
        ref = oracle.csr_spmm(A, X)
        for c in (0, k // 2, k - 1):
            assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32, (k, c)


def test_panel_degenerate_splits(torch_cuda, oracle):
    torch = torch_cuda
    rng = np.random.default_rng(59)
    cases = []
    # one column (every panel but one is empty)
    n = 2500
    rp = np.arange(n + 1, dtype=np.int64)
    cases.append(W.CSR(n, 1, rp, np.zeros(n, np.int32), rng.standard_normal(n).astype(np.float32)))
    # fewer columns than panels, rows of 0..5 entries
    lens = rng.integers(0, 6, size=n)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    col = np.concatenate([np.sort(rng.choice(5, size=l, replace=False)) for l in lens]).astype(np.int32)
    cases.append(W.CSR(n, 5, rp, col, rng.standard_normal(int(rp[-1])).astype(np.float32)))
    # every other row empty, one row with entries in every panel and one
    # row long enough for chunk partial sums inside each panel
    n, m = 4000, 300_000
    lens = np.where(np.arange(n) % 2 == 0, 0, rng.integers(1, 4, size=n))
    lens[1] = m
    lens[3] = 2000
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    col = np.concatenate([np.arange(m) if l == m else np.sort(rng.choice(m, size=l, replace=False))
                          for l in lens]).astype(np.int32)
    cases.append(W.CSR(n, m, rp, col, rng.standard_normal(int(rp[-1])).astype(np.float32)))
    # no nonzeros at all
    cases.append(W.CSR(100, 50, np.zeros(101, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)))
    for i, A in enumerate(cases):
        say("panels degenerate", i, A.n_rows, A.n_cols, A.nnz)
        x = W.uniform_vector(A.n_cols, 60 + i, np.float32)
        for P in (8, 16):
            M = rg.rgcsr_from_csr(A, col_panels=P, **LAY)
            assert M.info["panel_pieces"] == pieces(A, P)
            y = nan_out(torch, A.n_rows)
            M.spmv(dev(x), y)
            check_spmv(oracle, A, x, host(y))
            X = W.uniform_matrix(A.n_cols, 4, 70 + i)
            Y = nan_out(torch, A.n_rows, 4)
            rg.rgcsr_spmv_batched(M, dev(X), Y)
            Yh = host(Y)
            ref = oracle.csr_spmm(A, X)
            for c in range(4):
                assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32


def test_panel_rejections(torch_cuda, zipf):
    A, _ = zipf
    say("panels rejections")
    for P in (-8, 4, 12, 72):
        with pytest.raises(rg.RgcsrError) as e:
            rg.rgcsr_from_csr(A, col_panels=P, **LAY)
        assert e.value.status == 1
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_from_csr_batch([A, A], col_panels=8, **LAY)
    assert e.value.status == 6
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_plan_from_csr(A, col_panels=8, **LAY)
    assert e.value.status == 6


def test_panel_full_size_zipf_spmm(torch_cuda, oracle):
    """The Zipf matrix of 10^6 rows, four right-hand sides, every entry
    against the oracle (FP64 SpMM in C)."""
    torch = torch_cuda
    A, _ = W.workload_zipf(1_000_000)
    say("panels full-size spmm", A.nnz)
    X = W.uniform_matrix(A.n_cols, 4, W.SEEDS["spmm_X"])
    M = rg.rgcsr_from_csr(A, col_panels=8, G=64, sigma=512, tau=16)
    Y = nan_out(torch, A.n_rows, 4)
    rg.rgcsr_spmv_batched(M, dev(X), Y)
    Yh = host(Y)
    ref = oracle.csr_spmm(A, X)
    for c in range(4):
        assert oracle.scaled_error(Yh[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32


def test_panel_device_inputs_and_host_sizes(torch_cuda, oracle, zipf):
    """Device CSR inputs with col_panels go through the host conversion and
    give the same bits as host inputs; the host-only rgcsr_panel_sizes counts
    the pieces the handle holds."""
    torch = torch_cuda
    A, _ = zipf
    say("panels device inputs")
    X = W.uniform_matrix(A.n_cols, 4, 64)
    Mh = rg.rgcsr_from_csr(A, col_panels=8, **LAY)
    Md = rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(A.row_ptr, np.int64)),
                                  dev(np.ascontiguousarray(A.col, np.int32)), dev(A.val),
                                  rg.make_opts(col_panels=8, **LAY))
    s = rg.rgcsr_panel_sizes(A, rg.make_opts(col_panels=8, **LAY))
    assert Mh.info["panel_pieces"] == Md.info["panel_pieces"] == s["pieces"]
    Yh, Yd = nan_out(torch, A.n_rows, 4), nan_out(torch, A.n_rows, 4)
    rg.rgcsr_spmv_batched(Mh, dev(X), Yh)
    rg.rgcsr_spmv_batched(Md, dev(X), Yd)
    np.testing.assert_array_equal(host(Yd), host(Yh))

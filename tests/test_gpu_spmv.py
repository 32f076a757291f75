"""GPU parity of the RgCSR converter and SpMV against the FP64 CPU oracle,
called through the C ABI (ctypes binding)."""
import numpy as np
import pytest

from gpu_util import TOL_F32, TOL_F64, check_spmv, dev, host, say, storage_values

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg._lib.load()
    return torch


def layout_equal(got, exp):
    for k in ("gp", "short_len", "short_row", "slot_col", "long_row", "long_ptr", "long_col"):
        np.testing.assert_array_equal(got[k], exp[k], err_msg=k)
    for k in ("slot_val", "long_val"):
        np.testing.assert_array_equal(got[k].view(np.uint8), exp[k].view(np.uint8), err_msg=k)


def test_laplace2d_fp64_paper_layout(torch_cuda, oracle):
    """2D 5-point 64x64, float64, G = 64, paper layout."""
    torch = torch_cuda
    A, x = W.workload_laplace2d()
    say("laplace2d f64 G=64")
    M = rg.rgcsr_from_csr(A, G=64, value_dtype="f64")
    layout_equal(M.export(), oracle.rgcsr_layout(A, 64))
    rp, col, val = M.to_csr()
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(col, A.col)
    np.testing.assert_array_equal(val.view(np.uint64), A.val.view(np.uint64))
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, tol=TOL_F64)
    # A * 1: 4 - number of neighbours, exact
    ones = torch.ones(A.n_cols, dtype=torch.float64, device="cuda:0")
    np.testing.assert_array_equal(host(M.spmv(ones)), oracle.csr_spmv(A, np.ones(A.n_cols)))
    M.close()


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_identity_and_diagonal_bit_exact(torch_cuda, oracle, dt):
    torch = torch_cuda
    npdt = np.float64 if dt == "f64" else np.float32
    n = 100_003
    x = W.uniform_vector(n, 1, npdt)
    say("identity/diagonal", dt)
    M = rg.rgcsr_from_csr(W.identity(n, npdt), value_dtype=dt)
    np.testing.assert_array_equal(host(M.spmv(dev(x))), x)
    d = W.normal_vector(n, 2, npdt)
    M = rg.rgcsr_from_csr(W.diagonal(d), value_dtype=dt)
    np.testing.assert_array_equal(host(M.spmv(dev(x))), d * x)
    del torch


PARAMS = [(64, 1, 1, -1), (128, 1, 1, -1), (256, 1, 1, -1), (32, 1, 1, -1), (16, 2, 1, -1),
          (64, 2, 1, -1), (64, 4, 1, -1), (8, 8, 1, -1), (64, 1, 1 << 40, 16), (64, 1, 1 << 40, 0),
          (64, 1, 512, 24), (128, 2, 1 << 40, 64), (64, 8, 1 << 40, 100), (1, 1, 1, -1), (4, 1, 1, 3)]


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS)
def test_random_matrix_fp32_all_layouts(torch_cuda, oracle, G, T, sigma, tau):
    """Several groups, a ragged last group, empty rows, long rows of several
    wavefront chunks; converter bit-exact and SpMV within tolerance."""
    A = W.random_csr(3001, 2500, seed=G + 3 * T, max_len=70, empty_frac=0.2, long_rows=5,
                     long_len=2300, dtype=np.float32)
    x = W.uniform_vector(A.n_cols, 11, np.float32)
    say("random fp32", G, T, sigma, tau)
    M = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau)
    layout_equal(M.export(), oracle.rgcsr_layout(A, G, T, sigma, tau))
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y)
    M.close()


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS[:6] + PARAMS[8:10])
def test_random_matrix_fp64(torch_cuda, oracle, G, T, sigma, tau):
    A = W.random_csr(1500, 1200, seed=G + T, max_len=50, long_rows=3, long_len=1100)
    x = W.uniform_vector(A.n_cols, 12, np.float64)
    say("random fp64", G, T, sigma, tau)
    M = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau, value_dtype="f64")
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, tol=TOL_F64)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_low_precision_values(torch_cuda, oracle, dt):
    A = W.random_csr(4000, 3000, seed=7, max_len=40, long_rows=2, long_len=2000, dtype=np.float32)
    x = W.uniform_vector(A.n_cols, 13, np.float32)
    say("low precision", dt)
    M = rg.rgcsr_from_csr(A, G=64, sigma=4000, tau=32, value_dtype=dt)
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, vals64=storage_values(oracle, A, dt))


def test_fp32_values_fp64_vectors(torch_cuda, oracle):
    A = W.random_csr(5000, 5000, seed=8, max_len=30, long_rows=2, long_len=3000, dtype=np.float32)
    x = W.uniform_vector(A.n_cols, 14, np.float64)
    say("f32 values f64 vectors")
    M = rg.rgcsr_from_csr(A, G=64, sigma=5000, tau=20, value_dtype="f32")
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, tol=TOL_F64)


def test_zipf_sorted_with_long_rows(torch_cuda, oracle):
    A = W.zipf_matrix(200_000, seed=3)
    x = W.uniform_vector(A.n_cols, 15, np.float32)
    for (G, T, sigma, tau) in [(64, 1, 200_000, 16), (64, 1, 200_000, 64), (64, 2, 4096, 32), (64, 1, 1, -1)]:
        say("zipf 200k", G, T, sigma, tau)
        M = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau)
        check_spmv(oracle, A, x, host(M.spmv(dev(x))))
        M.close()


def test_zipf_fp64_long_rows(torch_cuda, oracle):
    """Double values, vectors and accumulation through every long-row path
    (LDS-staged wavefront items and workgroup items) on a power-law matrix."""
    A = W.zipf_matrix(200_000, seed=6).astype(np.float64)
    x = W.uniform_vector(A.n_cols, 16, np.float64)
    for (G, T, sigma, tau) in [(64, 1, 512, 16), (64, 1, 200_000, 40), (64, 2, 4096, 32)]:
        say("zipf 200k fp64", G, T, sigma, tau)
        M = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau, value_dtype="f64")
        assert M.info["long_work"] > 0
        check_spmv(oracle, A, x, host(M.spmv(dev(x))), tol=TOL_F64)
        M.close()


@pytest.mark.parametrize("sigma,tau", [(4096, 32), (512, 16), (1, -1), (1 << 40, 24)])
def test_rows_per_lane_schedules_agree(torch_cuda, oracle, sigma, tau):
    """Every kernel schedule (rows per lane fixed at 1, 2, 4, 8 or chosen per
    wavefront; loads over the group width or the row length; sliced ELLPACK,
    which multiplies the padding) multiplies each row in the same serial
    order, so all give the same values (padding adds only zeros for finite x),
    within tolerance of the oracle."""
    A = W.zipf_matrix(150_001, seed=9)
    x = W.uniform_vector(A.n_cols, 16, np.float32)
    ref = None
    for R in (0, 1, 2, 4, 8):
        for pad in (0, 1, 2, 3):
            say("schedules zipf 150001", sigma, tau, R, pad)
            M = rg.rgcsr_from_csr(A, G=64, sigma=sigma, tau=tau, rows_per_lane=R, pad_loads=pad)
            assert (M.info["rows_per_lane"] == R or R == 0) and M.info["pad_loads"] == pad
            y = host(M.spmv(dev(x)))
            M.close()
            if ref is None:
                check_spmv(oracle, A, x, y)
                ref = y
            elif pad == 2:   # padding multiplied: same values, zeros may differ in sign
                np.testing.assert_array_equal(y, ref)
            else:
                np.testing.assert_array_equal(y.view(np.uint32), ref.view(np.uint32))


def test_row_lengths_from_columns_mode(torch_cuda, oracle):
    """pad_loads = 3 reads no row lengths; it is chosen by default when a lane
    owns a whole row and no grouped row is empty, and refused otherwise."""
    S = W.laplacian_3d_7pt(20, dtype=np.float32)
    x = W.uniform_vector(S.n_cols, 20, np.float32)
    M = rg.rgcsr_from_csr(S, G=64)
    assert M.info["pad_loads"] == 3
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, S, x, y)
    M0 = rg.rgcsr_from_csr(S, G=64, pad_loads=0)
    np.testing.assert_array_equal(y.view(np.uint32), host(M0.spmv(dev(x))).view(np.uint32))
    A = W.random_csr(2000, 2000, seed=3, max_len=20, empty_frac=0.1, dtype=np.float32)
    assert rg.rgcsr_from_csr(A, G=64).info["pad_loads"] in (0, 1)
    for kw in (dict(G=64), dict(G=32, T=2)):
        with pytest.raises(rg.RgcsrError) as e:
            rg.rgcsr_from_csr(A if kw["G"] == 64 else S, pad_loads=3, **kw)
        assert e.value.status == 6


@pytest.mark.parametrize("G,T,sigma,tau", [(64, 1, 1, -1), (128, 1, 1 << 40, 32), (64, 2, 1, -1), (32, 2, 4096, 8)])
def test_sliced_ellpack_mode(torch_cuda, oracle, G, T, sigma, tau):
    """Sliced ELLPACK over the same layout (no row lengths, padding
    multiplied) equals RgCSR for finite x, including lanes_per_row > 1."""
    A = W.random_csr(3001, 2500, seed=21, max_len=70, empty_frac=0.2, long_rows=5, long_len=2300,
                     dtype=np.float32)
    x = W.uniform_vector(A.n_cols, 17, np.float32)
    say("sliced ELLPACK", G, T, sigma, tau)
    M = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau, pad_loads=1)
    E = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau, pad_loads=2)
    assert E.info["pad_loads"] == 2
    y, ye = host(M.spmv(dev(x))), host(E.spmv(dev(x)))
    check_spmv(oracle, A, x, ye)
    np.testing.assert_array_equal(ye, y)
    with pytest.raises(rg.RgcsrError) as e:   # groups narrower than a wavefront
        rg.rgcsr_from_csr(A, G=16, T=1, pad_loads=2)
    assert e.value.status == 6


def test_load_policies_same_result(torch_cuda, oracle):
    """Cached streams (1) and nontemporal x (2) change only cache hints: the
    bits equal the default policy's; unsupported combinations are errors.
    (The column-tiled long rows run with policy 0 only, so they are off here:
    with them the default policy sums those rows in another order.)"""
    torch = torch_cuda
    A = W.zipf_matrix(120_000, seed=10)
    x = W.uniform_vector(A.n_cols, 18, np.float32)
    ref = None
    for lay in (dict(sigma=1, tau=-1), dict(sigma=512, tau=16)):
        for lp in (0, 1, 2):
            say("load policy", lay, lp)
            M = rg.rgcsr_from_csr(A, G=64, load_policy=lp, tile_min_len=0, **lay)
            assert M.info["load_policy"] == lp
            y = host(M.spmv(dev(x)))
            M.close()
            if lp == 0:
                check_spmv(oracle, A, x, y)
                ref = y
            else:
                np.testing.assert_array_equal(y.view(np.uint32), ref.view(np.uint32))
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_from_csr(A, G=64, load_policy=1, value_dtype="f64")
    assert e.value.status == 6
    M = rg.rgcsr_from_csr(A, G=64, load_policy=2)
    with pytest.raises(rg.RgcsrError) as e:
        M.spmv(torch.zeros(A.n_cols, dtype=torch.float64, device="cuda:0"))
    assert e.value.status == 6


def test_rcm_reordered_spmv(torch_cuda, oracle):
    """SpMV of P A P^T on P x is P (A x): the ordering only renumbers."""
    A = W.zipf_matrix(40_000, seed=5, max_len=500)
    S, _ = W.scrambled(W.laplacian_3d_7pt(24, dtype=np.float32), 3)
    for M0 in (A, S):
        x = W.uniform_vector(M0.n_cols, 19, np.float32)
        perm = rg.rgcsr_rcm_order(M0)
        B = W.permute_symmetric(M0, perm)
        say("rcm reordered", M0.n_rows)
        M = rg.rgcsr_from_csr(B, G=64, sigma=512, tau=16)
        y = host(M.spmv(dev(np.ascontiguousarray(x[perm]))))
        check_spmv(oracle, B, x[perm], y)
        yo = oracle.csr_spmv(M0, x)[perm]
        assert np.max(np.abs(y - yo)) <= 1e-5 * max(1.0, float(np.max(oracle.csr_absmv(M0, x))))
        M.close()


def test_hip_graph_capture_and_replay(torch_cuda, oracle):
    """The SpMV (including the chunk-combine launch of a row over 16,384
    nonzeros) can be captured in a HIP graph: every replay, with eager work
    and host syncs between replays, equals an eager launch on the same x."""
    torch = torch_cuda
    A = W.random_csr(5000, 30000, seed=12, max_len=40, long_rows=3, long_len=20000, dtype=np.float32)
    M = rg.rgcsr_from_csr(A, G=64, sigma=512, tau=16)
    assert M.info["partials"] > 0
    x = torch.from_numpy(W.uniform_vector(A.n_cols, 22, np.float32)).cuda()
    y = torch.empty(A.n_rows, device="cuda:0")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            rg.rgcsr_spmv(M, x, y)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rg.rgcsr_spmv(M, x, y)
    ref = torch.empty_like(y)
    for rep in range(4):
        say("graph replay", rep)
        x.mul_(-1.5).add_(0.25)          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = y.clone()
        rg.rgcsr_spmv(M, x, ref)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(got).view(np.uint32), host(ref).view(np.uint32))
        check_spmv(oracle, A, host(x), host(got))


def test_deterministic_repeat(torch_cuda, oracle):
    """No atomics in RgCSR SpMV: repeated launches give identical bits, also
    for rows split over several wavefronts."""
    torch = torch_cuda
    A = W.zipf_matrix(100_000, seed=4)
    x = dev(W.uniform_vector(A.n_cols, 16, np.float32))
    say("determinism")
    M = rg.rgcsr_from_csr(A, G=64, sigma=100_000, tau=16)
    y0 = host(M.spmv(x))
    for _ in range(5):
        np.testing.assert_array_equal(host(M.spmv(x)), y0)
    say("determinism with rows split over several workgroups")
    B = W.random_csr(300, 100_000, seed=5, max_len=30, long_rows=4, long_len=70_000, dtype=np.float32)
    M = rg.rgcsr_from_csr(B, G=64, sigma=300, tau=16)
    assert M.info["partials"] > 0
    y0 = host(M.spmv(x))
    check_spmv(oracle, B, host(x), y0)
    for _ in range(5):
        np.testing.assert_array_equal(host(M.spmv(x)), y0)
    del torch


def test_edge_cases(torch_cuda, oracle):
    torch = torch_cuda
    say("edge: empty rows only")
    A = W.CSR(130, 50, np.zeros(131, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    M = rg.rgcsr_from_csr(A)
    y = torch.full((130,), 7.0, device="cuda:0")
    M.spmv(dev(np.ones(50, np.float32)), y)
    assert (host(y) == 0).all()
    say("edge: n < 64, one row")
    A = W.random_csr(1, 9, seed=1, max_len=9, empty_frac=0.0, dtype=np.float32)
    x = W.uniform_vector(9, 1, np.float32)
    check_spmv(oracle, A, x, host(rg.rgcsr_from_csr(A).spmv(dev(x))))
    say("edge: one very long row split over many chunks")
    n = 40_000
    A = W.CSR(2, n, np.array([0, n, n + 3], np.int64),
              np.concatenate([np.arange(n), [0, 5, 9]]).astype(np.int32),
              W.normal_vector(n + 3, 3, np.float32))
    x = W.uniform_vector(n, 2, np.float32)
    for tau in (-1, 8):
        check_spmv(oracle, A, x, host(rg.rgcsr_from_csr(A, sigma=2, tau=tau).spmv(dev(x))))
    say("edge: zero rows")
    A = W.CSR(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    M = rg.rgcsr_from_csr(A)
    M.spmv(dev(np.ones(5, np.float32)), torch.empty(0, device="cuda:0"))


def test_unaligned_multi_rhs_falls_back(torch_cuda, oracle):
    torch = torch_cuda
    A = W.random_csr(3000, 2000, seed=10, max_len=20, long_rows=2, long_len=1500, dtype=np.float32)
    M = rg.rgcsr_from_csr(A, sigma=3000, tau=16)
    X = W.uniform_matrix(A.n_cols, 4, seed=6)
    Xd = torch.zeros(A.n_cols * 4 + 1, device="cuda:0")[1:].view(A.n_cols, 4)  # 4 bytes off alignment
    Xd.copy_(dev(X))
    say("unaligned k=4")
    Y = host(M.spmm(Xd))
    ref = oracle.csr_spmm(A, X)
    for c in range(4):
        assert oracle.scaled_error(Y[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32


def test_device_resident_csr_input(torch_cuda, oracle):
    torch = torch_cuda
    A = W.random_csr(2000, 1500, seed=9, max_len=20, dtype=np.float32)
    say("device csr input")
    M = rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(A.row_ptr), dev(A.col), dev(A.val),
                                 rg.make_opts(G=64, sigma=2000, tau=10))
    layout_equal(M.export(), oracle.rgcsr_layout(A, 64, 1, 2000, 10))
    del torch


def test_errors_surface_as_status(torch_cuda):
    torch = torch_cuda
    A = W.random_csr(100, 100, seed=1, dtype=np.float32)
    M = rg.rgcsr_from_csr(A)
    X = torch.zeros((100, 4), device="cuda:0")
    Y = torch.zeros((100, 4), device="cuda:0")
    with pytest.raises(rg.RgcsrError) as e:   # leading dimension smaller than k
        rg._lib.call("rgcsr_spmv_batched", M.handle, 4, X.data_ptr(), 2, Y.data_ptr(), 4, rg.RGCSR_F32, 0, 0)
    assert e.value.status == 1
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_from_csr(A, G=48)
    assert e.value.status == 6
    Md = rg.rgcsr_from_csr(A, value_dtype="f64")
    with pytest.raises(rg.RgcsrError):
        Md.spmv(torch.zeros(100, device="cuda:0"))


def test_stream_read_helper(torch_cuda):
    """The bandwidth probe reads any 16-byte multiple and rejects bad sizes."""
    torch = torch_cuda
    buf = torch.zeros(1 << 22, dtype=torch.uint8, device="cuda:0")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rg.rgcsr_stream_read(buf, sink)
    rg.rgcsr_stream_read(buf[:16], sink)
    torch.cuda.synchronize()
    assert int(sink.item()) == 0  # all-zero data never reaches the store
    with pytest.raises(rg.RgcsrError) as e:
        rg._lib.call("rgcsr_stream_read", buf.data_ptr(), 17, sink.data_ptr(), 0)
    assert e.value.status == 1
    with pytest.raises(rg.RgcsrError) as e:
        rg._lib.call("rgcsr_stream_read", buf.data_ptr() + 4, 16, sink.data_ptr(), 0)
    assert e.value.status == 1


def test_gather_floor_helper(torch_cuda):
    """The gather-floor probe visits every entry once: lane l sums entries
    l, l + S, ..., l + 7S (S = lanes rounded up to whole workgroups)."""
    torch = torch_cuda
    n, ncols = 100_003, 5000
    rng = np.random.default_rng(3)
    col = rng.integers(0, ncols, n).astype(np.int32)
    val = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(ncols).astype(np.float32)
    lanes = (n + 7) // 8
    S = (lanes + 255) // 256 * 256
    out = torch.empty(lanes, device="cuda:0")
    rg.rgcsr_gather_floor(dev(col), dev(val), dev(x), out)
    got = host(out)
    prod = np.zeros(S * 8)
    prod[:n] = val.astype(np.float64) * x[col].astype(np.float64)
    ref = prod.reshape(8, S).sum(axis=0)[:lanes]
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, float(np.max(np.abs(ref))))
    with pytest.raises(ValueError):
        rg.rgcsr_gather_floor(dev(col), dev(val[:-1]), dev(x), out)


@pytest.mark.slow
def test_full_size_laplace3d_and_zipf(torch_cuda, oracle):
    """The benchmark matrices at full size, in the benchmark's layouts."""
    from bench import LAYOUT_STENCIL, LAYOUT_ZIPF
    for name, mk, lay in (("laplace3d 128^3", W.workload_laplace3d, LAYOUT_STENCIL),
                          ("zipf 1e6", W.workload_zipf, LAYOUT_ZIPF)):
        A, x = mk()
        say("full size", name, lay)
        M = rg.rgcsr_from_csr(A, **lay)
        y = host(M.spmv(dev(x)))
        e = check_spmv(oracle, A, x, y, tol=TOL_F32)
        say("  scaled error", e)
        M.close()


@pytest.mark.slow
def test_full_size_27pt_every_storage_dtype(torch_cuda, oracle):
    """27-point 160^3 (n = 4,096,000, 109M nonzeros) at full size: A*1 equals
    28 - prod(m_d) exactly in every storage dtype (27 and -1 are exact in
    BF16/FP16, the sums are small integers), and random x matches the oracle
    on every row."""
    torch = torch_cuda
    N = 160
    A = W.stencil_3d_27pt(N, dtype=np.float32)
    ones = torch.ones(A.n_cols, device="cuda:0")
    i = np.arange(N)
    m = np.where((i == 0) | (i == N - 1), 2, 3)
    expect = (28 - m[:, None, None] * m[None, :, None] * m[None, None, :]).reshape(-1).astype(np.float32)
    x = W.uniform_vector(A.n_cols, 28, np.float32)
    for dt in ("f32", "bf16", "f16"):
        say("full size 27pt", dt)
        M = rg.rgcsr_from_csr(A, G=64, value_dtype=dt)
        np.testing.assert_array_equal(host(M.spmv(ones)), expect)
        y = host(M.spmv(dev(x)))
        e = check_spmv(oracle, A, x, y, vals64=None if dt == "f32" else storage_values(oracle, A, dt))
        say("  scaled error, all rows", e)
        M.close()
        del M


@pytest.mark.slow
def test_full_size_batched_set(torch_cuda, oracle):
    """The 4,096-matrix batch at full size in one launch (the layout the
    batched benchmark's autotuner picks, and the paper layout); every matrix
    against the oracle, per-matrix tolerance."""
    torch = torch_cuda
    mats = W.batched_set(count=4096, seed=W.SEEDS["batched"])
    xh = W.uniform_vector(sum(M.n_cols for M in mats), 30, np.float32)
    x = dev(xh)
    pick = range(len(mats))
    for kw in (dict(G=64, sigma=256, pad_loads=0), dict(G=64)):
        say("full size batch", kw)
        B = rg.rgcsr_from_csr_batch(mats, **kw)
        ro, co = B.batch_offsets()
        y = torch.empty(int(ro[-1]), device="cuda:0")
        rg.rgcsr_spmv_batched(B, x.view(-1, 1), y.view(-1, 1), True)
        yh = host(y)
        for i in pick:
            check_spmv(oracle, mats[i], xh[co[i]:co[i + 1]], yh[ro[i]:ro[i + 1]])
        B.close()


def test_autotune_picks_a_timed_candidate_and_caches(torch_cuda, oracle, tmp_path):
    torch = torch_cuda
    A = W.zipf_matrix(60_000, seed=8)
    x = dev(W.uniform_vector(A.n_cols, 17, np.float32))
    y = torch.empty(A.n_rows, device="cuda:0")
    cache = str(tmp_path / "tune.json")
    say("autotune")
    best, tried = rg.rgcsr_autotune(A, x, y, max_candidates=8, reps=3, cache_path=cache)
    assert 2 <= len(tried) <= 8
    assert all(t["us"] > 0 for t in tried)
    assert min(t["us"] for t in tried) == [t["us"] for t in tried if t["opts"] == rg.opts_dict(best)][0]
    M = rg.rgcsr_from_csr(A, opts=best)
    check_spmv(oracle, A, host(x), host(M.spmv(x)))
    best2, tried2 = rg.rgcsr_autotune(A, x, y, cache_path=cache)   # served from the cache
    assert rg.opts_dict(best2) == rg.opts_dict(best) and tried2 == tried


def test_autotune_covers_group_size_and_lanes(torch_cuda, oracle):
    """The cost model proposes group sizes and lanes per row beyond (64, 1)
    where they move fewer bytes (long uniform rows), always keeps the paper
    layout, and every timed candidate is correct."""
    torch = torch_cuda
    A = W.banded_poisson_matrix(30_000, 120.0, 400, np.random.default_rng(31), np.float32)
    x = dev(W.uniform_vector(A.n_cols, 23, np.float32))
    y = torch.empty(A.n_rows, device="cuda:0")
    say("autotune G and T")
    best, tried = rg.rgcsr_autotune(A, x, y, max_candidates=6, reps=2)
    pairs = {(t["opts"]["group_size"], t["opts"]["lanes_per_row"]) for t in tried}
    assert (64, 1) in pairs
    for t in tried:
        M = rg.rgcsr_from_csr(A, opts=rg.opts_from_dict(t["opts"]))
        check_spmv(oracle, A, host(x), host(M.spmv(x)))
        M.close()


def test_autotune_batch(torch_cuda, oracle, tmp_path):
    torch = torch_cuda
    mats = W.batched_set(count=48, n_lo=50, n_hi=3000, seed=32)
    ncols = sum(M.n_cols for M in mats)
    nrows = sum(M.n_rows for M in mats)
    xh = W.uniform_vector(ncols, 24, np.float32)
    x, y = dev(xh), torch.empty(nrows, device="cuda:0")
    cache = str(tmp_path / "tune_batch.json")
    say("autotune batch")
    best, tried = rg.rgcsr_autotune_batch(mats, x, y, max_candidates=5, reps=2, cache_path=cache)
    assert 1 <= len(tried) <= 5
    assert rg.opts_dict(best) in [t["opts"] for t in tried]
    B = rg.rgcsr_from_csr_batch(mats, opts=best)
    yh = host(B.spmv(x))
    ro, co = B.batch_offsets()
    for i in range(0, len(mats), 7):
        M = mats[i]
        check_spmv(oracle, M, xh[co[i]:co[i + 1]], yh[ro[i]:ro[i + 1]])
    best2, tried2 = rg.rgcsr_autotune_batch(mats, x, y, cache_path=cache)
    assert rg.opts_dict(best2) == rg.opts_dict(best) and tried2 == tried


@pytest.mark.parametrize("empty,lay", [(0.1, dict(G=64)), (0.1, dict(G=64, sigma=1 << 40, tau=16)),
                                       (0.1, dict(G=64, pad_loads=0)), (0.1, dict(G=64, pad_loads=1)),
                                       (0.1, dict(G=32, T=2, tau=24)), (0.0, dict(G=64, pad_loads=3)),
                                       (0.0, dict(G=64, sigma=512, tau=8, pad_loads=3))])
def test_non_finite_x_reaches_only_rows_that_use_it(torch_cuda, oracle, empty, lay):
    """y_i sums the stored nonzeros of row i only (§3.4): a NaN or infinity in
    x reaches exactly the rows with a nonzero in that column, also x[0], which
    padding and out-of-range steps gather but never multiply."""
    if empty:
        A = W.random_csr(3000, 2500, seed=41, max_len=40, empty_frac=empty, long_rows=4, long_len=2200,
                         dtype=np.float32)
    else:  # no empty row: every Zipf row has at least one nonzero
        A = W.zipf_matrix(20_000, seed=41, max_len=3000)
    x = W.uniform_vector(A.n_cols, 42, np.float32)
    bad = {0: np.nan, 5: np.inf, 17: -np.inf, 1234: np.nan}
    for c, v in bad.items():
        x[c] = v
    say("non-finite x", lay)
    ref = oracle.csr_spmv(A, x)
    xf = x.copy()
    xf[list(bad)] = 0.0
    s = oracle.csr_absmv(A, xf)
    M = rg.rgcsr_from_csr(A, **lay)
    assert M.info["pad_loads"] == lay.get("pad_loads", M.info["pad_loads"])
    ys = {"rgcsr": host(M.spmv(dev(x)))}
    if "tau" not in lay and "T" not in lay and "pad_loads" not in lay:
        ys["hybrid"] = host(rg.hyb_from_csr(A).spmv(dev(x)))
    for name, y in ys.items():
        np.testing.assert_array_equal(np.isnan(y), np.isnan(ref), err_msg=name)
        np.testing.assert_array_equal(np.isposinf(y), np.isposinf(ref), err_msg=name)
        np.testing.assert_array_equal(np.isneginf(y), np.isneginf(ref), err_msg=name)
        fin = np.isfinite(ref)
        assert np.any(~fin) and np.any(fin)
        assert oracle.scaled_error(y[fin], ref[fin], s[fin]) <= TOL_F32, name

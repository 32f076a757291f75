"""GPU parity of the column-tiled long rows (x staged in LDS per tile of
8,192 columns, 4,096 for F64 storage, partial sums added in a fixed order)
against the FP64 oracle,
through the C ABI, and the paths that must fall back to the long-row kernel
(FP64 vectors, several right-hand sides, strided x, other load policies)."""
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


@pytest.fixture(scope="module")
def zipf():
    # 200,000 columns: 25 tiles, the last one partial (3,392 columns)
    A = W.zipf_matrix(200_000, seed=41)
    x = W.uniform_vector(A.n_cols, 42, np.float32)
    return A, x


LAY = dict(G=64, sigma=512, tau=16)


def tiled(A, **kw):
    o = dict(LAY)
    o.update(kw)
    M = rg.rgcsr_from_csr(A, **o)
    return M


@pytest.mark.parametrize("min_len", [64, 300, 2000])
@pytest.mark.parametrize("dt", ["f32", "bf16", "f16"])
def test_tiled_parity(torch_cuda, oracle, zipf, min_len, dt):
    A, x = zipf
    say("tiles", min_len, dt)
    M = tiled(A, tile_min_len=min_len, value_dtype=dt)
    assert M.info["tiled_rows"] > 0 and M.info["n_tiles"] == 25
    L = np.diff(A.row_ptr)
    assert M.info["tiled_rows"] == int(np.sum(L >= min_len))
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, vals64=None if dt == "f32" else storage_values(oracle, A, dt))
    # deterministic: the same bits again
    np.testing.assert_array_equal(host(M.spmv(dev(x))).view(np.uint32), y.view(np.uint32))


def test_tiles_off_and_fallbacks(torch_cuda, oracle, zipf):
    torch = torch_cuda
    A, x = zipf
    M = tiled(A, tile_min_len=64)
    M0 = tiled(A, tile_min_len=0)
    assert M.info["tiled_rows"] > 0 and M0.info["tiled_rows"] == 0
    say("tiles off")
    check_spmv(oracle, A, x, host(M0.spmv(dev(x))))
    # x that is not 16-byte aligned: the tile is staged element by element
    say("tiles, x at a 4-byte offset")
    buf = torch.empty(A.n_cols + 1, device="cuda:0")
    buf[1:] = dev(x)
    xs = buf[1:]
    assert xs.data_ptr() % 16 != 0
    y = host(M.spmv(xs))
    check_spmv(oracle, A, x, y)
    np.testing.assert_array_equal(y.view(np.uint32), host(M.spmv(dev(x))).view(np.uint32))
    # FP64 vectors: the long-row kernel runs the tiled rows
    say("tiles, FP64 vectors")
    x64 = x.astype(np.float64)
    check_spmv(oracle, A, x64, host(M.spmv(dev(x64))), tol=TOL_F32)
    # several right-hand sides: long-row kernel, per column against the oracle
    say("tiles, k = 4")
    X = W.uniform_matrix(A.n_cols, 4, 43)
    Y = host(M.spmm(dev(X)))
    ref = oracle.csr_spmm(A, X)
    for c in range(4):
        assert oracle.scaled_error(Y[:, c], ref[:, c], oracle.csr_absmv(A, X[:, c])) <= TOL_F32
    # other load policies take the long-row kernel
    say("tiles, load policy 1")
    M1 = tiled(A, tile_min_len=64, load_policy=1)
    check_spmv(oracle, A, x, host(M1.spmv(dev(x))))


def test_tiles_follow_value_updates_clone_and_transpose(torch_cuda, oracle, zipf):
    torch = torch_cuda
    A, x = zipf
    say("tiles, set_values, clone, transpose")
    M = tiled(A, tile_min_len=64, keep_csr_map=True, build_transpose=True)
    assert M.info["tiled_rows"] > 0
    theta = W.normal_vector(A.nnz, 44, np.float32)
    rg.rgcsr_set_values(M, dev(theta))
    A2 = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, theta)
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A2, x, y)
    C = M.clone()
    np.testing.assert_array_equal(host(C.spmv(dev(x))).view(np.uint32), y.view(np.uint32))
    # dx = A^T dy on the transposed handle (its own tiled rows, if any)
    dy = W.normal_vector(A.n_rows, 45, np.float32)
    dx = torch.empty(A.n_cols, device="cuda:0")
    rg.rgcsr_spmv_transpose_grad(M, None, dev(dy), dx, None)
    AT = W.CSR(A.n_cols, A.n_rows, *oracle.csr_transpose(A2))
    check_spmv(oracle, AT, dy, host(dx))


def test_tiles_built_on_device_and_into_torch_memory(torch_cuda, oracle, zipf):
    torch = torch_cuda
    A, x = zipf
    M = tiled(A, tile_min_len=64)
    y = host(M.spmv(dev(x)))
    say("tiles, device conversion")
    D = rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(A.row_ptr, np.int64)),
                                 dev(A.col), dev(A.val), rg.make_opts(**LAY, tile_min_len=64))
    assert D.info["tiled_rows"] == M.info["tiled_rows"]
    np.testing.assert_array_equal(host(D.spmv(dev(x))).view(np.uint32), y.view(np.uint32))
    np.testing.assert_array_equal(host(D.clone().spmv(dev(x))).view(np.uint32), y.view(np.uint32))
    say("tiles, plan and build into torch memory")
    P = rg.rgcsr_plan_from_csr(A, **LAY, tile_min_len=64)
    B = P.build()
    assert B.info["tiled_rows"] == M.info["tiled_rows"]
    np.testing.assert_array_equal(host(B.spmv(dev(x))).view(np.uint32), y.view(np.uint32))


def test_tiles_with_a_dense_tile_segment(torch_cuda, oracle):
    """A row holding 4,096 consecutive columns of one tile (one segment of
    4,096 entries, a whole unit: 64 lanes per row, 64 products per lane) next
    to sparse long rows, and a row with 5,000 entries in one tile, more than a
    unit holds, which stays on the long-row path."""
    A = W.random_csr(3000, 70_000, seed=46, max_len=8, long_rows=6, long_len=9000)
    L = np.diff(A.row_ptr).copy()
    cols, vals = [], []
    rng = np.random.default_rng(47)
    for r in range(A.n_rows):
        c = A.col[A.row_ptr[r]:A.row_ptr[r + 1]]
        v = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
        if r == 0:
            c = np.concatenate([np.arange(4096), 8192 + np.sort(rng.choice(60_000, 3000, replace=False))])
            c = c.astype(np.int32)
            v = rng.standard_normal(len(c))
        if r == 1:
            c = np.concatenate([np.sort(rng.choice(16_384, 1500, replace=False)), 16_384 + np.arange(5000)])
            c = c.astype(np.int32)
            v = rng.standard_normal(len(c))
        cols.append(c)
        vals.append(v)
        L[r] = len(c)
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    A = W.CSR(A.n_rows, A.n_cols, rp, np.concatenate(cols).astype(np.int32),
              np.concatenate(vals).astype(np.float32))
    x = W.uniform_vector(A.n_cols, 48, np.float32)
    say("tiles, dense tile segment")
    M = rg.rgcsr_from_csr(A, G=64, tau=16, tile_min_len=1000)
    assert M.info["tiled_rows"] == int(np.sum(L >= 1000)) - 1
    check_spmv(oracle, A, x, host(M.spmv(dev(x))))


@pytest.mark.parametrize("vdt", ["f32", "f64"])
def test_tiles_in_a_batch(torch_cuda, oracle, vdt):
    torch = torch_cuda
    mats = [W.zipf_matrix(60_000, seed=50 + i) for i in range(3)]
    say("tiles, batch", vdt)
    B = rg.rgcsr_from_csr_batch(mats, G=64, sigma=512, tau=16, tile_min_len=64, value_dtype=vdt)
    assert B.info["tiled_rows"] > 0
    ro, co = B.batch_offsets()
    ft = np.float64 if vdt == "f64" else np.float32
    xh = W.uniform_vector(int(co[-1]), 51, ft)
    y = torch.empty(int(ro[-1]), dtype=torch.float64 if vdt == "f64" else torch.float32, device="cuda:0")
    rg.rgcsr_spmv(B, dev(xh), y)
    yh = host(y)
    for i, Mi in enumerate(mats):
        check_spmv(oracle, Mi, xh[co[i]:co[i + 1]], yh[ro[i]:ro[i + 1]], tol=TOL_F64 if vdt == "f64" else TOL_F32)


def test_full_size_zipf_tiles_auto(torch_cuda, oracle):
    """The benchmark's Zipf layout picks the column tiles by itself."""
    from bench import LAYOUT_ZIPF
    A, x = W.workload_zipf()
    M = rg.rgcsr_from_csr(A, **LAYOUT_ZIPF)
    say("full-size Zipf, automatic tiles", M.info["tiled_rows"], M.info["tile_entries"])
    assert M.info["tiled_rows"] > 0
    check_spmv(oracle, A, x, host(M.spmv(dev(x))))


# F64 storage: tiles of 4,096 columns and units of 2,048 entries with x, the
# products and the partial sums in FP64.  200,000 columns make 49 tiles, the last one partial (3,392
# columns); rows need at least max(min_len, 25) nonzeros.
@pytest.mark.parametrize("min_len", [16, 300, 2000])
def test_tiled_parity_f64(torch_cuda, oracle, zipf, min_len):
    A, _ = zipf
    x = W.uniform_vector(A.n_cols, 52, np.float64)
    say("tiles, F64 storage", min_len)
    M = tiled(A, tile_min_len=min_len, value_dtype="f64")
    assert M.info["n_tiles"] == 49
    L = np.diff(A.row_ptr)
    assert M.info["tiled_rows"] == int(np.sum(L >= max(min_len, 25)))
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A, x, y, tol=TOL_F64)
    np.testing.assert_array_equal(host(M.spmv(dev(x))).view(np.uint64), y.view(np.uint64))
    M0 = tiled(A, tile_min_len=0, value_dtype="f64")
    assert M0.info["tiled_rows"] == 0
    check_spmv(oracle, A, x, host(M0.spmv(dev(x))), tol=TOL_F64)


def test_tiles_f64_updates_clone_device_and_torch_memory(torch_cuda, oracle, zipf):
    """F64 tiles follow value updates (both value paths), clones, device
    conversion and plan/build, bit for bit; x at an 8-byte offset (not
    16-byte aligned) stages the tile element by element; two right-hand
    sides take the long-row kernel."""
    torch = torch_cuda
    A, _ = zipf
    x = W.uniform_vector(A.n_cols, 53, np.float64)
    lay = dict(LAY, tile_min_len=64, value_dtype="f64")
    say("tiles, F64 set_values and clone")
    M = tiled(A, keep_csr_map=True, build_transpose=True, **lay)
    assert M.info["tiled_rows"] > 0
    theta = W.normal_vector(A.nnz, 54, np.float64)
    rg.rgcsr_set_values(M, dev(theta))
    A2 = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, theta)
    y = host(M.spmv(dev(x)))
    check_spmv(oracle, A2, x, y, tol=TOL_F64)
    np.testing.assert_array_equal(host(M.clone().spmv(dev(x))).view(np.uint64), y.view(np.uint64))
    rg.rgcsr_set_values(M, theta)  # host values: the other update path
    np.testing.assert_array_equal(host(M.spmv(dev(x))).view(np.uint64), y.view(np.uint64))
    say("tiles, F64 x at an 8-byte offset")
    buf = torch.empty(A.n_cols + 1, dtype=torch.float64, device="cuda:0")
    buf[1:] = dev(x)
    assert buf[1:].data_ptr() % 16 != 0
    np.testing.assert_array_equal(host(M.spmv(buf[1:])).view(np.uint64), y.view(np.uint64))
    say("tiles, F64 k = 2 and strided x")
    X = W.uniform_matrix(A.n_cols, 2, 55).astype(np.float64)
    Y = host(M.spmm(dev(X)))
    ref = oracle.csr_spmm(A2, X)
    for c in range(2):
        assert oracle.scaled_error(Y[:, c], ref[:, c], oracle.csr_absmv(A2, X[:, c])) <= TOL_F64
    say("tiles, F64 device conversion")
    y1 = host(tiled(A, **lay).spmv(dev(x)))
    D = rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(A.row_ptr, np.int64)),
                                 dev(A.col), dev(A.val), rg.make_opts(**lay))
    assert D.info["tiled_rows"] == M.info["tiled_rows"]
    np.testing.assert_array_equal(host(D.spmv(dev(x))).view(np.uint64), y1.view(np.uint64))
    say("tiles, F64 plan and build into torch memory")
    B = rg.rgcsr_plan_from_csr(A, **lay).build()
    np.testing.assert_array_equal(host(B.spmv(dev(x))).view(np.uint64), y1.view(np.uint64))
    check_spmv(oracle, A, x, y1, tol=TOL_F64)


def test_tiles_f64_with_a_whole_unit_segment(torch_cuda, oracle):
    """F64 tiles of 4,096 columns and units of 2,048 entries: a row holding
    2,048 consecutive columns of tile 1 (one segment that fills a unit) next
    to sparse long rows, and a row with 3,000 entries in tile 3, more than a
    unit holds, which stays on the long-row path."""
    A = W.random_csr(2000, 40_000, seed=56, max_len=8, long_rows=5, long_len=6000)
    L = np.diff(A.row_ptr).copy()
    cols, vals = [], []
    rng = np.random.default_rng(57)
    for r in range(A.n_rows):
        c = A.col[A.row_ptr[r]:A.row_ptr[r + 1]]
        v = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
        if r == 3:
            c = np.concatenate([np.sort(rng.choice(4096, 700, replace=False)), 4096 + np.arange(2048),
                                8192 + np.sort(rng.choice(30_000, 900, replace=False))]).astype(np.int32)
            v = rng.standard_normal(len(c))
        if r == 4:
            c = np.concatenate([np.sort(rng.choice(4096, 500, replace=False)),
                                12_288 + np.arange(3000)]).astype(np.int32)
            v = rng.standard_normal(len(c))
        cols.append(c)
        vals.append(v)
        L[r] = len(c)
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    A = W.CSR(A.n_rows, A.n_cols, rp, np.concatenate(cols).astype(np.int32), np.concatenate(vals))
    x = W.uniform_vector(A.n_cols, 58, np.float64)
    say("tiles, F64 whole-unit segment")
    M = rg.rgcsr_from_csr(A, G=64, tau=16, tile_min_len=1000, value_dtype="f64")
    assert M.info["tiled_rows"] == int(np.sum(L >= 1000)) - 1
    check_spmv(oracle, A, x, host(M.spmv(dev(x))), tol=TOL_F64)


def test_full_size_zipf_tiles_auto_f64(torch_cuda, oracle):
    """The benchmark's Zipf layout in F64 storage picks the column tiles by
    itself (4,096 columns each)."""
    from bench import LAYOUT_ZIPF
    A, x = W.workload_zipf()
    x = x.astype(np.float64)
    M = rg.rgcsr_from_csr(A, value_dtype="f64", **LAYOUT_ZIPF)
    say("full-size Zipf F64, automatic tiles", M.info["tiled_rows"], M.info["tile_entries"])
    assert M.info["tiled_rows"] > 0 and M.info["n_tiles"] == -(-A.n_cols // 4096)
    check_spmv(oracle, A, x, host(M.spmv(dev(x))), tol=TOL_F64)


@pytest.mark.parametrize("vdt", ["f32", "f64"])
def test_handle_tiles_match_host_tile_sizes(torch_cuda, zipf, vdt):
    """A handle built on the host or on the device tiles the rows that
    rgcsr_tile_sizes selects without a GPU."""
    A, _ = zipf
    o = dict(LAY, tile_min_len=64, value_dtype=vdt)
    s = rg.rgcsr_tile_sizes(A, rg.make_opts(**o))
    assert s["tiled_rows"] > 0
    say("tiles, host sizes against handles", vdt)
    M = rg.rgcsr_from_csr(A, **o)
    D = rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(A.row_ptr, np.int64)),
                                 dev(A.col), dev(A.val), rg.make_opts(**o))
    for H in (M, D):
        assert (H.info["n_tiles"], H.info["tiled_rows"], H.info["tile_entries"]) == \
            (s["n_tiles"], s["tiled_rows"], s["tile_entries"])

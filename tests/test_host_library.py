"""CPU tests of librgcsr's host logic: exported symbols, the host layout
against the oracle (bit for bit), value rounding against torch, the Hybrid
width rule against the oracle, and the error codes of malformed input."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import _lib
from paper_1012_2270_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1012_2270_amd import build
        build.build()
    return _lib.load()


def header_functions():
    with open(os.path.join(ROOT, "include", "rgcsr.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:rgcsr|hyb)_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"
    assert rg.version().startswith("rgcsr")


def test_status_strings(lib):
    for code in range(7):
        assert lib.rgcsr_status_string(code)


def same_layout(L, O, check_values=True):
    for k in ("gp", "short_len", "short_row", "slot_col", "long_row", "long_ptr", "long_col"):
        np.testing.assert_array_equal(L[k], O[k], err_msg=k)
    if check_values:
        for k in ("slot_val", "long_val"):
            np.testing.assert_array_equal(L[k].view(np.uint8), O[k].view(np.uint8), err_msg=k)


PARAMS = [(64, 1, 1, -1), (4, 1, 1, -1), (128, 1, 1, -1), (32, 2, 1, -1), (64, 4, 1 << 40, 16),
          (16, 8, 300, 5), (64, 1, 4096, 0), (256, 1, 1, 200), (1, 1, 1, -1), (7, 2, 9, 3)]


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS)
def test_layout_matches_oracle_bit_exact(lib, oracle, G, T, sigma, tau):
    A = W.random_csr(777, 400, seed=G * 7 + T, max_len=40, long_rows=6, long_len=390, empty_frac=0.15)
    opts = rg.make_opts(G=G, T=T, sigma=sigma, tau=tau, value_dtype="f64")
    L = rg.rgcsr_layout_host(A, opts)
    O = oracle.rgcsr_layout(A, G, T, sigma, tau)
    same_layout(L, O)
    assert L["slots"] == O["slots"] and L["n_groups"] == O["groups"]


def test_layout_zipf_sorted_long_rows(lib, oracle):
    A = W.zipf_matrix(30_000, seed=9)
    for (G, T, sigma, tau) in [(64, 1, 30_000, 16), (64, 1, 1, -1), (64, 2, 4096, 64)]:
        L = rg.rgcsr_layout_host(A, rg.make_opts(G=G, T=T, sigma=sigma, tau=tau))
        O = oracle.rgcsr_layout(A, G, T, sigma, tau)
        same_layout(L, O)


@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_value_rounding_matches_torch(lib, oracle, dt):
    """Stored values are rounded to nearest even from float32; torch's CPU
    conversion pins the finite and infinite cases bit for bit."""
    A = W.random_csr(300, 200, seed=5, max_len=30)
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2 ** 32, A.nnz, dtype=np.uint64).astype(np.uint32)
    # bias towards the interesting exponent range of the 16-bit types
    bits[::3] = (bits[::3] & 0x807fffff) | (rng.integers(95, 150, bits[::3].size).astype(np.uint32) << 23)
    bits[:8] = [0x33000000, 0x33000001, 0x477ff000, 0x477fefff, 0x387fffff, 0x80000000, 0x7f800000, 0x00000001]
    vals = bits.view(np.float32)
    A = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals)
    L = rg.rgcsr_layout_host(A, rg.make_opts(G=64, value_dtype=dt))
    want = oracle.round_values(vals, dt)
    O = oracle.rgcsr_layout(A, 64, values=want)
    got, exp = L["slot_val"], O["slot_val"]
    if dt == "f32":
        np.testing.assert_array_equal(got.view(np.uint32), exp.view(np.uint32))
        return
    g16, e16 = got.view(np.uint16), exp.view(np.uint16)
    expo = 0x7c00 if dt == "f16" else 0x7f80
    man = 0x03ff if dt == "f16" else 0x007f
    e_nan = ((e16 & expo) == expo) & ((e16 & man) != 0)
    g_nan = ((g16 & expo) == expo) & ((g16 & man) != 0)
    np.testing.assert_array_equal(g_nan, e_nan)
    np.testing.assert_array_equal(g16[~e_nan], e16[~e_nan])


def test_float64_to_bf16_goes_through_float32(lib, oracle):
    v = np.random.default_rng(1).standard_normal(5000)
    A = W.CSR(1, 5000, np.array([0, 5000]), np.arange(5000, dtype=np.int32), v)
    L = rg.rgcsr_layout_host(A, rg.make_opts(G=64, value_dtype="bf16"))
    want = oracle.round_values(v.astype(np.float32), "bf16")
    np.testing.assert_array_equal(L["slot_val"].view(np.uint16), want)


def test_layout_sizes_match_oracle(lib, oracle):
    A = W.random_csr(2000, 900, seed=3, max_len=60, long_rows=20, long_len=800)
    for G, T, s, t in PARAMS:
        got = rg.rgcsr_layout_sizes(A, rg.make_opts(G=G, T=T, sigma=s, tau=t))
        exp = oracle.rgcsr_sizes(A, G, T, s, t)
        assert (got["n_groups"], got["n_short"], got["n_long"], got["slots"], got["long_nnz"]) == \
            (exp["groups"], exp["n_short"], exp["n_long"], exp["slots"], exp["long_nnz"])


def test_long_work_items_cover_long_rows(lib):
    """Rows longer than 1024 go to whole-workgroup items of 16384 nonzeros; a
    row needing several items gets one partial-sum slot per item."""
    A = W.zipf_matrix(50_000, seed=2)
    extra = W.random_csr(20, 50_000, seed=3, max_len=5, long_rows=3, long_len=40_000)
    for M in (A, extra):
        for tau in (0, 8, 64, 700):
            info = rg.rgcsr_layout_sizes(M, rg.make_opts(G=64, sigma=M.n_rows, tau=tau))
            lens = np.diff(M.row_ptr)
            lens = lens[lens > tau]
            nch = (lens[lens > 1024] + 16383) // 16384
            assert info["partials"] == int(nch[nch > 1].sum())
            assert info["long_nnz"] == int(lens.sum())


@pytest.mark.parametrize("s_v,dt", [(4, "f32"), (8, "f64"), (2, "bf16")])
def test_hybrid_width_rule_matches_oracle(lib, oracle, s_v, dt):
    for A in (W.laplacian_3d_7pt(20), W.zipf_matrix(40_000, seed=4),
              W.random_csr(3000, 3000, seed=1, max_len=50, long_rows=4, long_len=2000)):
        assert rg.hyb_choose_width(A, dt) == oracle.hyb_k1(A, s_v)


def _status(fn, *args):
    try:
        fn(*args)
    except _lib.RgcsrError as e:
        return e.status
    return 0


def test_malformed_csr_is_rejected(lib):
    good = W.random_csr(20, 10, seed=0, max_len=5)
    opts = rg.make_opts()
    assert _status(rg.rgcsr_layout_host, good, opts) == 0

    def mk(rp, col):
        return W.CSR(3, 4, np.array(rp, np.int64), np.array(col, np.int32), np.ones(len(col)))
    bad = [mk([1, 2, 3, 4], [0, 1, 2, 3]),      # rp[0] != 0
           mk([0, 2, 1, 3], [0, 1, 2]),         # decreasing
           mk([0, 1, 2, 3], [0, 5, 1]),         # column out of range
           mk([0, 2, 2, 3], [2, 1, 0]),         # not ascending
           mk([0, 2, 2, 3], [1, 1, 0])]         # duplicate
    for A in bad:
        assert _status(rg.rgcsr_layout_host, A, opts) == 2  # RGCSR_ECSR
    assert "row" in _lib.load().rgcsr_last_error().decode()


def test_bad_options_rejected(lib):
    A = W.random_csr(20, 10, seed=0, max_len=5)
    assert _status(rg.rgcsr_layout_host, A, rg.make_opts(T=3)) == 1
    assert _status(rg.rgcsr_layout_host, A, rg.make_opts(G=-2)) == 1
    # a dtype code the library does not know, passed straight through the ABI
    rp, col = A.row_ptr.astype(np.int64), A.col.astype(np.int32)
    val = A.val.astype(np.float64)
    assert _status(_lib.call, "rgcsr_layout_host", A.n_rows, A.n_cols, A.nnz, rp.ctypes.data,
                   col.ctypes.data, val.ctypes.data, 9, ctypes.byref(rg.make_opts()),
                   *([None] * 9)) == 1


def test_empty_matrix_layout(lib, oracle):
    A = W.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    L = rg.rgcsr_layout_host(A, rg.make_opts(value_dtype="f64"))
    assert L["slots"] == 0 and L["n_groups"] == 0
    A = W.CSR(5, 3, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0))
    L = rg.rgcsr_layout_host(A, rg.make_opts(G=4, value_dtype="f64"))
    same_layout(L, oracle.rgcsr_layout(A, 4))


def test_plan_needs_no_gpu_and_sizes_the_device_block(lib):
    """rgcsr_plan_from_csr converts on the host only; the device bytes cover
    every layout array (each 256-byte aligned inside one block)."""
    A = W.random_csr(3000, 2500, seed=9, max_len=60, empty_frac=0.1, long_rows=4, long_len=2000)
    for kw in (dict(G=64), dict(G=64, sigma=512, tau=24), dict(G=128, T=2, value_dtype="bf16")):
        P = rg.rgcsr_plan_from_csr(A, **kw)
        s = rg.rgcsr_layout_sizes(A, rg.make_opts(**kw))
        esz = {"f32": 4, "bf16": 2}[kw.get("value_dtype", "f32")]
        arrays = (s["slots"] + s["long_nnz"]) * (esz + 4) + (s["n_groups"] + 1) * 8 + s["n_short"] * 4
        assert arrays <= P.device_bytes <= arrays + 64 * 1024 + 16 * A.n_rows
        assert P.device_bytes % 256 == 0
        PT = rg.rgcsr_plan_from_csr(A, build_transpose=True, **kw)
        assert PT.device_bytes > P.device_bytes + A.nnz * (esz + 4)
        P.close()
        PT.close()


def test_plan_sizes_the_column_tiles(lib):
    """The plan's device block holds the column-tiled copy of the long rows:
    8,192-column tiles with FP32 partial sums for F32 storage, 4,096-column
    tiles with FP64 partial sums for F64 storage.  Rows of at least
    max(min_len, tiles / 2) nonzeros are tiled; the extra bytes cover their
    16-bit columns and values, one partial sum per (tile, row), the
    tile-major row pointers and the source map (sizes from an independent
    count)."""
    A = W.random_csr(2000, 1_000_000, seed=12, max_len=8, long_rows=400, long_len=1200)
    L = np.diff(A.row_ptr)
    for vt, cols, esz in (("f32", 8192, 4), ("f64", 4096, 8)):
        n_tiles = -(-A.n_cols // cols)
        rows = L >= max(300, (n_tiles + 1) // 2)
        n_trows, n_ent = int(rows.sum()), int(L[rows].sum())
        long_nnz = int(L[L > 16].sum())
        assert n_trows == 400 and long_nnz == n_ent
        base = rg.rgcsr_plan_from_csr(A, G=64, tau=16, tile_min_len=0, value_dtype=vt)
        tiled = rg.rgcsr_plan_from_csr(A, G=64, tau=16, tile_min_len=300, value_dtype=vt)
        d = tiled.device_bytes - base.device_bytes
        low = (n_ent * (2 + esz) + n_tiles * n_trows * esz + long_nnz * 4 + n_tiles * (n_trows + 1) * 4
               + n_trows * 4)
        assert low <= d <= low + 64 * 1024, (vt, d, low)
        base.close()
        tiled.close()


def test_batch_plan_needs_no_gpu(lib):
    """rgcsr_plan_from_csr_batch converts a block-diagonal batch on the host:
    a batch of one matrix needs the same device block as the single-matrix
    plan, a larger batch more than its largest member; empty batches, mixed
    value types, malformed members and column panels are refused."""
    mats = [W.random_csr(700 + 100 * i, 500 + 50 * i, seed=20 + i, max_len=30, long_rows=2, long_len=400,
                         dtype=np.float32) for i in range(3)]
    kw = dict(G=64, sigma=256, tau=24)
    one = rg.rgcsr_plan_from_csr_batch(mats[:1], **kw)
    single = rg.rgcsr_plan_from_csr(mats[0], **kw)
    assert one.device_bytes == single.device_bytes
    three = rg.rgcsr_plan_from_csr_batch(mats, **kw)
    assert three.device_bytes > max(rg.rgcsr_plan_from_csr(A, **kw).device_bytes for A in mats)
    assert three.device_bytes % 256 == 0
    for P in (one, single, three):
        P.close()
    with pytest.raises(ValueError):
        rg.rgcsr_plan_from_csr_batch([mats[0], W.CSR(mats[1].n_rows, mats[1].n_cols, mats[1].row_ptr,
                                                     mats[1].col, mats[1].val.astype(np.float64))], **kw)
    p = ctypes.c_void_p()
    o = rg.make_opts(**kw)
    with pytest.raises(rg.RgcsrError) as e:
        _lib.call("rgcsr_plan_from_csr_batch", 0, None, None, None, None, None, 1, ctypes.byref(o), ctypes.byref(p))
    assert e.value.status == 1
    bad = W.CSR(mats[1].n_rows, mats[1].n_cols, mats[1].row_ptr.copy(), mats[1].col.copy(), mats[1].val)
    bad.col[0] = bad.n_cols
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_plan_from_csr_batch([mats[0], bad], **kw)
    assert e.value.status == 2
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_plan_from_csr_batch(mats, col_panels=8, **kw)
    assert e.value.status == 6


def test_plan_build_argument_errors(lib):
    """A buffer below the plan's size or off 256-byte alignment is refused
    before any device work, and the plan stays buildable; bad CSR is refused
    by the plan step."""
    A = W.random_csr(500, 400, seed=2, max_len=20)
    P = rg.rgcsr_plan_from_csr(A)
    h = ctypes.c_void_p()
    with pytest.raises(rg.RgcsrError) as e:
        _lib.call("rgcsr_build", P._p, 1 << 20, P.device_bytes - 1, None, ctypes.byref(h))
    assert e.value.status == 1 and "smaller" in str(e.value)
    with pytest.raises(rg.RgcsrError) as e:
        _lib.call("rgcsr_build", P._p, (1 << 20) + 64, P.device_bytes, None, ctypes.byref(h))
    assert e.value.status == 1 and "aligned" in str(e.value)
    b = ctypes.c_int64()
    _lib.call("rgcsr_plan_device_bytes", P._p, ctypes.byref(b))
    assert b.value == P.device_bytes
    P.close()
    bad = W.CSR(3, 4, np.array([0, 2, 1, 3], np.int64), np.array([0, 1, 2], np.int32), np.ones(3))
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_plan_from_csr(bad)
    assert e.value.status == 2
    assert lib.rgcsr_plan_destroy(None) == 0

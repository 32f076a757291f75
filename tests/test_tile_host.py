"""Host logic of the column-tiled copy (rgcsr_tile_sizes, no GPU): the tile
width by value type, the row-length threshold, the unit limit on a row's
entries in one tile and the automatic minimum, against an independent count
in numpy; argument and CSR errors."""
import numpy as np
import pytest

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W


def expected(A, tau, min_len, vdt):
    """Tiles of 8,192 columns (4,096 for F64 storage); candidates are the
    long rows (more than tau nonzeros, none when tau < 0) of at least
    max(min_len or 256, ceil(tiles / 2)) nonzeros whose entries in any one
    tile fit a unit (4,096; 2,048 for F64); the automatic choice
    (min_len < 0) keeps them only when they hold 262,144 nonzeros or more."""
    cols = 4096 if vdt == "f64" else 8192
    unit = 2048 if vdt == "f64" else 4096
    L = np.diff(A.row_ptr)
    none = (dict(n_tiles=0, tiled_rows=0, tile_entries=0), 0)
    if min_len == 0 or tau < 0 or A.n_cols == 0 or not np.any(L > tau):
        return none
    n_tiles = -(-A.n_cols // cols)
    thr = max(256 if min_len < 0 else min_len, (n_tiles + 1) // 2)
    rows = []
    for r in np.nonzero((L > tau) & (L >= thr))[0]:
        t = A.col[A.row_ptr[r]:A.row_ptr[r + 1]] // cols
        # columns ascend within a row, so a tile's entries are one run
        if np.bincount(t).max() > unit:
            continue
        rows.append(r)
    ent = int(L[rows].sum()) if rows else 0
    if not rows or (min_len < 0 and ent < 262_144):
        return none
    return dict(n_tiles=n_tiles, tiled_rows=len(rows), tile_entries=ent), thr


def with_dense_rows(seed):
    """Random rows plus two long rows with 3,000 and 5,000 consecutive columns
    in one tile of each width, over 60,000 columns."""
    A = W.random_csr(1500, 60_000, seed=seed, max_len=10, long_rows=6, long_len=7000, dtype=np.float32)
    rng = np.random.default_rng(seed)
    L = np.diff(A.row_ptr).copy()
    cols = [A.col[A.row_ptr[r]:A.row_ptr[r + 1]] for r in range(A.n_rows)]
    cols[0] = np.concatenate([np.sort(rng.choice(8192, 400, replace=False)), 8192 + np.arange(3000)])
    cols[1] = np.concatenate([np.sort(rng.choice(16_384, 900, replace=False)), 16_384 + np.arange(5000)])
    for r in (0, 1):
        L[r] = len(cols[r])
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    c = np.concatenate(cols).astype(np.int32)
    return W.CSR(A.n_rows, A.n_cols, rp, c, np.ones(len(c), np.float32))


CASES = [
    ("zipf 20k", lambda: W.zipf_matrix(20_000, seed=81)),
    ("zipf 200k", lambda: W.zipf_matrix(200_000, seed=82)),
    ("dense segments", lambda: with_dense_rows(83)),
    ("random, empty rows", lambda: W.random_csr(3_000, 30_000, seed=84, max_len=40, empty_frac=0.3,
                                                long_rows=20, long_len=1500)),
    ("one column", lambda: W.CSR(500, 1, np.arange(501, dtype=np.int64), np.zeros(500, np.int32),
                                 np.ones(500, np.float32))),
    ("no nonzeros", lambda: W.CSR(40, 30, np.zeros(41, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("vdt", ["f32", "f64", "bf16"])
@pytest.mark.parametrize("tau,min_len", [(-1, 64), (0, 64), (6, -1), (16, 0), (16, 300), (16, 1000)])
def test_tile_sizes_match_the_rule(name, make, vdt, tau, min_len):
    A = make()
    s = rg.rgcsr_tile_sizes(A, rg.make_opts(G=64, sigma=512, tau=tau, tile_min_len=min_len, value_dtype=vdt))
    want, thr = expected(A, tau, min_len, vdt)
    assert {k: s[k] for k in want} == want
    assert s["min_len"] == thr
    unit = 2048 if vdt == "f64" else 4096
    if want["tiled_rows"]:
        # every unit holds at most a unit's entries of one tile; the XCD
        # queues add at most seven empty units per round of eight
        assert -(-want["tile_entries"] // unit) <= s["units"] <= 8 * want["n_tiles"] * want["tiled_rows"]
    else:
        assert s["units"] == 0


def test_dense_segments_are_left_to_the_long_row_path():
    """The 3,000-entry segment fits an F32 unit but not an F64 one; the
    5,000-entry segment fits neither."""
    A = with_dense_rows(83)
    L = np.diff(A.row_ptr)
    n_candidates = int(np.sum(L >= 1000))
    f32 = rg.rgcsr_tile_sizes(A, rg.make_opts(tau=16, tile_min_len=1000))
    f64 = rg.rgcsr_tile_sizes(A, rg.make_opts(tau=16, tile_min_len=1000, value_dtype="f64"))
    assert f32["tiled_rows"] == n_candidates - 1
    assert f64["tiled_rows"] == n_candidates - 2
    assert (f32["n_tiles"], f64["n_tiles"]) == (8, 15)


def test_tile_sizes_refusals():
    A = W.zipf_matrix(2_000, seed=85)
    with pytest.raises(rg.RgcsrError) as e:
        rg._lib.call("rgcsr_tile_sizes", A.n_rows, A.n_cols, A.nnz, 0, 0, None, None, None, None, None, None)
    assert e.value.status == 1
    B = W.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col.copy(), A.val)
    B.col[0] = A.n_cols  # column out of range
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_tile_sizes(B, rg.make_opts(tau=16, tile_min_len=64))
    assert e.value.status == 2
    o = rg.make_opts(tau=16, tile_min_len=64)
    o.value_dtype = 9  # not a dtype code
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_tile_sizes(A, o)
    assert e.value.status == 1

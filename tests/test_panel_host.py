"""Host logic of the column-panel copy (rgcsr_panel_sizes, no GPU): the panel
column bounds, the rows kept whole and split, and the piece counts, against
an independent count in numpy; argument and CSR errors."""
import numpy as np
import pytest

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W


def expected(A, P, tau):
    """Bounds: the first column at which the nonzeros of the columns before it
    reach ceil(q * nnz / P), nondecreasing; rows of at most tau nonzeros (all
    of them kept whole when tau >= 0, none when tau < 0) are one piece each,
    the others one piece per panel holding some of their entries."""
    L = np.diff(A.row_ptr)
    before = np.concatenate([[0], np.cumsum(np.bincount(A.col, minlength=A.n_cols))])
    cb = [0]
    for q in range(1, P):
        t = -(-A.nnz * q // P)
        cb.append(max(cb[-1], min(int(np.searchsorted(before, t)), A.n_cols)))
    cb.append(A.n_cols)
    split = L > tau
    rows = np.repeat(np.arange(A.n_rows), L)
    pan = np.searchsorted(np.asarray(cb[1:]), A.col, side="right")
    es = np.repeat(split, L)
    split_pieces = int(np.unique(rows[es].astype(np.int64) * P + pan[es]).size)
    whole = int(np.sum(~split))
    return np.asarray(cb), int(split.sum()), split_pieces, whole + split_pieces


CASES = [
    ("zipf", lambda: W.zipf_matrix(20_000, seed=71)),
    ("banded", lambda: W.banded_poisson_matrix(5_000, 12.0, 200, np.random.default_rng(72))),
    ("random, empty rows", lambda: W.random_csr(3_000, 900, seed=73, max_len=40, empty_frac=0.3,
                                                long_rows=4, long_len=700)),
    ("one column", lambda: W.CSR(500, 1, np.arange(501, dtype=np.int64), np.zeros(500, np.int32),
                                 np.ones(500, np.float32))),
    ("no nonzeros", lambda: W.CSR(40, 30, np.zeros(41, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("P", [8, 16, 64])
@pytest.mark.parametrize("tau", [-1, 0, 6, 16])
def test_panel_sizes_match_the_rule(name, make, P, tau):
    A = make()
    s = rg.rgcsr_panel_sizes(A, rg.make_opts(G=64, sigma=512, tau=tau, col_panels=P))
    cb, split_rows, split_pieces, pieces = expected(A, P, tau)
    np.testing.assert_array_equal(s["col_bounds"], cb)
    assert s["split_rows"] == split_rows
    assert s["split_pieces"] == split_pieces
    assert s["pieces"] == pieces
    # every nonzero lands in the copy once: grouped nonzeros (slots include
    # padding) plus long-row nonzeros cover nnz
    assert s["long_nnz"] <= A.nnz and s["slots"] + s["long_nnz"] >= A.nnz


def test_panel_bounds_balance_the_nonzeros():
    """Each panel holds at most its share of the nonzeros plus one column's."""
    A = W.zipf_matrix(50_000, seed=74)
    P = 8
    cb = rg.rgcsr_panel_sizes(A, rg.make_opts(tau=16, col_panels=P))["col_bounds"]
    per = np.array([np.sum((A.col >= cb[q]) & (A.col < cb[q + 1])) for q in range(P)])
    assert per.sum() == A.nnz
    colmax = np.bincount(A.col, minlength=A.n_cols).max()
    assert per.max() <= -(-A.nnz // P) + colmax


def test_panel_sizes_refusals():
    A = W.zipf_matrix(2_000, seed=75)
    for P in (0, 4, 12, 72, -8):
        with pytest.raises(rg.RgcsrError) as e:
            rg.rgcsr_panel_sizes(A, rg.make_opts(col_panels=P))
        assert e.value.status == 1
    B = W.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col.copy(), A.val)
    B.col[0] = A.n_cols  # column out of range
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_panel_sizes(B, rg.make_opts(col_panels=8))
    assert e.value.status == 2

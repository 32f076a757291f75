"""Pins for the oracle's RgCSR layout against the paper's worked example
(Section 3.4), hand-derived layouts, brute force and grid closed forms."""
import itertools
import json
import os

import numpy as np
import pytest

from paper_1012_2270_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def worked_example():
    with open(GOLDEN) as f:
        ex = json.load(f)
    cols = ex["columns_by_row"]
    rp = np.zeros(len(cols) + 1, np.int64)
    rp[1:] = np.cumsum([len(c) for c in cols])
    A = W.CSR(len(cols), 8, rp, np.array(sum(cols, []), np.int32),
              np.arange(1, rp[-1] + 1, dtype=np.float64))  # value = CSR index + 1
    return ex, A


def test_worked_example_printed_counts(oracle):
    ex, A = worked_example()
    assert list(A.row_ptr[:-1]) == ex["row_first_positions"]
    assert A.nnz == ex["nnz"]
    L = oracle.rgcsr_layout(A, G=ex["paper"]["group_size"])
    assert list(L["gp"]) == ex["paper"]["group_pointers"]
    assert oracle.artificial_zeros(L) == ex["paper"]["artificial_zeros_rgcsr"]


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_worked_example_slot_by_slot(oracle, which):
    ex, A = worked_example()
    spec = ex["layouts"][which]
    L = oracle.rgcsr_layout(A, G=spec["G"], T=spec["T"], sigma=spec["sigma"], tau=spec["tau"])
    assert list(L["gp"]) == spec["gp"]
    assert list(L["short_row"]) == spec["short_row"]
    assert list(L["long_row"]) == spec["long_row"]
    assert len(L["slot_val"]) == len(spec["slots"])
    for s, e in enumerate(spec["slots"]):
        if e[0] == "pad":
            r = e[1]
            last = A.col[A.row_ptr[r + 1] - 1] if A.row_ptr[r + 1] > A.row_ptr[r] else 0
            assert L["slot_val"][s] == 0.0 and np.signbit(L["slot_val"][s]) == False  # noqa: E712
            assert L["slot_col"][s] == last, (s, e)
        else:
            r, j = e
            k = A.row_ptr[r] + j
            assert L["slot_val"][s] == A.val[k], (s, e)
            assert L["slot_col"][s] == A.col[k], (s, e)
    # long rows keep CSR order
    for i, r in enumerate(L["long_row"]):
        seg = slice(L["long_ptr"][i], L["long_ptr"][i + 1])
        np.testing.assert_array_equal(L["long_col"][seg], A.col[A.row_ptr[r]:A.row_ptr[r + 1]])


def test_worked_example_ellpack_zero_count(oracle):
    ex, A = worked_example()
    K = ex["paper"]["ellpack_width"]
    H = oracle.hyb_layout(A, K)
    ell_col = H["ell_col"].reshape(K, H["n_pad"])[:, :A.n_rows]
    assert int((ell_col < 0).sum()) == ex["paper"]["artificial_zeros_ellpack"]
    assert H["coo_nnz"] == 0


PARAMS = [(1, 1, 1, -1), (4, 1, 1, -1), (64, 1, 1, -1), (5, 2, 1, -1), (8, 4, 16, -1),
          (64, 1, 1 << 30, 6), (3, 8, 7, 2), (64, 2, 64, 0)]


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS)
@pytest.mark.parametrize("seed", [0, 1])
def test_round_trip_bit_exact(oracle, G, T, sigma, tau, seed):
    A = W.random_csr(131, 70, seed=seed, max_len=20, long_rows=3, empty_frac=0.2)
    # arbitrary value bit patterns, including -0.0, subnormals, inf and NaN payloads
    bits = np.random.default_rng(seed).integers(0, 2 ** 32, A.nnz, dtype=np.uint64).astype(np.uint32)
    bits[::7] = 0x80000000
    bits[1::11] = 0x00000001
    vals = bits.view(np.float32)
    L = oracle.rgcsr_layout(A, G, T, sigma, tau, values=vals)
    rp, col, val = oracle.rgcsr_decode(L)
    np.testing.assert_array_equal(rp, A.row_ptr)
    np.testing.assert_array_equal(col, A.col)
    np.testing.assert_array_equal(val.view(np.uint32), bits)


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS)
def test_layout_walk_equals_csr_serial_sum(oracle, G, T, sigma, tau):
    """The kernel walk visits every row's nonzeros in CSR order, so in FP64 it
    reproduces the serial CSR SpMV bit for bit."""
    A = W.random_csr(200, 90, seed=G + T, max_len=30, long_rows=4)
    x = np.random.default_rng(T).standard_normal(90)
    L = oracle.rgcsr_layout(A, G, T, sigma, tau)
    np.testing.assert_array_equal(oracle.rgcsr_spmv(L, x), oracle.csr_spmv(A, x))


def test_every_slot_is_a_nonzero_or_padding(oracle):
    A = W.random_csr(97, 60, seed=21, max_len=15)
    L = oracle.rgcsr_layout(A, 8, 2, 1, -1, values=np.arange(1, A.nnz + 1, dtype=np.float64))
    real = L["slot_val"][L["slot_val"] != 0]
    np.testing.assert_array_equal(np.sort(real), np.arange(1, A.nnz + 1))
    assert (L["slot_col"] >= 0).all() and (L["slot_col"] < A.n_cols).all()


def _padding_for_order(lens, order, G):
    pad = 0
    for g in range(0, len(order), G):
        grp = [lens[r] for r in order[g:g + G]]
        pad += len(grp) * max(grp) - sum(grp)
    return pad


@pytest.mark.parametrize("n,G", [(6, 2), (6, 3), (8, 4), (8, 2)])
def test_descending_order_minimises_padding_brute_force(oracle, n, G):
    """Section 4.4.2: descending ordering is optimal for suppressing
    artificial zeros.  Checked against every row permutation.  The claim
    holds when every group is full (n % G == 0); with a smaller last group
    brute force finds better orders (see the next test)."""
    for seed in range(4):
        lens = np.random.default_rng(seed).integers(0, 9, n)
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(lens)
        A = W.CSR(n, 9, rp, np.concatenate([np.arange(l) for l in lens]).astype(np.int32),
                  np.ones(rp[-1]))
        best = min(_padding_for_order(lens, p, G) for p in itertools.permutations(range(n)))
        L = oracle.rgcsr_layout(A, G, 1, n, -1)
        assert oracle.artificial_zeros(L) == best


def test_descending_order_not_optimal_with_partial_last_group(oracle):
    """Counterexample found by brute force: lengths [8,1,1,1,1,1,1] with G=3.
    Descending order puts 8 with two 1s (14 zeros); placing it alone in the
    short last group needs none."""
    lens = np.array([8, 1, 1, 1, 1, 1, 1])
    rp = np.zeros(8, np.int64)
    rp[1:] = np.cumsum(lens)
    A = W.CSR(7, 9, rp, np.concatenate([np.arange(l) for l in lens]).astype(np.int32),
              np.ones(rp[-1]))
    assert oracle.artificial_zeros(oracle.rgcsr_layout(A, 3, 1, 7, -1)) == 14
    assert _padding_for_order(lens, [1, 2, 3, 4, 5, 6, 0], 3) == 0


def test_padding_grows_with_group_size(oracle):
    """Doubling G merges neighbouring groups, so padding never decreases
    (Table 4's trend)."""
    A = W.random_csr(1000, 500, seed=3, max_len=40, long_rows=5, long_len=300)
    pads = [oracle.artificial_zeros(oracle.rgcsr_layout(A, G)) for G in (1, 2, 4, 8, 16, 32, 64, 128, 256)]
    assert pads[0] == 0
    assert all(a <= b for a, b in zip(pads, pads[1:]))


def test_stencil_slot_counts_closed_forms(oracle):
    """At G = 64 a group is one grid line (x fastest).  Slots per group are 64
    times the longest row of that line; derived from the grid geometry."""
    # 2D 5-point on 64^2: boundary lines have width 4, the other 62 width 5
    s = oracle.rgcsr_sizes(W.laplacian_2d_5pt(64), 64)
    assert s["slots"] == 2 * 64 * 4 + 62 * 64 * 5 == 20_352
    assert s["slots"] - 20_224 == 128
    # 3D 7-point on N^3: a line at (y, z) has width 7 - [y on face] - [z on face]
    N = 128
    A = W.laplacian_3d_7pt(N)
    widths = {7: (N - 2) ** 2, 6: 4 * (N - 2), 5: 4}
    expect = 64 * 2 * sum(w * c for w, c in widths.items())  # two groups per line
    assert oracle.rgcsr_sizes(A, 64)["slots"] == expect == 14_614_528


@pytest.mark.slow
def test_27pt_slot_count_closed_form(oracle):
    """27-point on 160^3: a grid line at (y, z) has longest row 3 * m_y * m_z
    (m = 2 on a face, 3 inside); a group of 64 rows may straddle two lines
    and takes the wider one."""
    N, G = 160, 64
    def line_width(l):
        y, z = l % N, l // N
        m = lambda i: 2 if i in (0, N - 1) else 3  # noqa: E731
        return 3 * m(y) * m(z)
    total = 0
    for g in range((N ** 3 + G - 1) // G):
        l0, l1 = (g * G) // N, (g * G + G - 1) // N
        total += G * max(line_width(l0), line_width(l1))
    assert total == 109_764_096
    assert oracle.rgcsr_sizes(W.stencil_3d_27pt(N), G)["slots"] == total

"""Row ordering (Reverse Cuthill-McKee, the bandwidth-reducing ordering built
for the row-ordering study the paper leaves to future work): the oracle's
plain-Python order pinned by hand-worked graphs and by the properties the
definition fixes, then the native library order against the oracle bit for
bit."""
import numpy as np
import pytest

from paper_1012_2270_amd import workloads as W


def csr_of_edges(n, edges, extra_diag=True):
    """Square pattern with the given (i, j) entries (and the diagonal)."""
    cells = set()
    for i, j in edges:
        cells.add((i, j))
    if extra_diag:
        cells |= {(i, i) for i in range(n)}
    rows = [[] for _ in range(n)]
    for i, j in sorted(cells):
        rows[i].append(j)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([j for r in rows for j in r], dtype=np.int32)
    return W.CSR(n, n, rp, col, np.ones(len(col)))


def bandwidth(A) -> int:
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    return int(np.max(np.abs(rows - A.col))) if A.nnz else 0


def test_star_graph_hand_worked(oracle):
    # centre 0 (degree 4), leaves 1..4 (degree 1).  Start: leaf 1 (smallest
    # degree, then index); 1 numbers 0; 0 numbers 2, 3, 4.  CM = [1, 0, 2, 3, 4].
    A = csr_of_edges(5, [(0, k) for k in range(1, 5)])
    np.testing.assert_array_equal(oracle.rcm_order(A), [4, 3, 2, 0, 1])


def test_two_components_and_isolated_vertex(oracle):
    # component {0, 1, 2} as a path 0-1-2, component {3, 4}, isolated 5.
    # Starts in (degree, index) order: 5 (degree 0) first, then 0 (degree 1):
    # 0, 1, 2; then 3: 3, 4.  CM = [5, 0, 1, 2, 3, 4].
    A = csr_of_edges(6, [(0, 1), (1, 2), (3, 4)])
    np.testing.assert_array_equal(oracle.rcm_order(A), [4, 3, 2, 1, 0, 5])


def test_unsymmetric_pattern_is_symmetrised(oracle):
    # only a_01 and a_21 stored: the graph is still the path 0-1-2
    A = csr_of_edges(3, [(0, 1), (2, 1)], extra_diag=False)
    B = csr_of_edges(3, [(0, 1), (1, 0), (1, 2), (2, 1)], extra_diag=False)
    np.testing.assert_array_equal(oracle.rcm_order(A), oracle.rcm_order(B))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_scrambled_path_gets_bandwidth_one(oracle, seed):
    n = 50
    A = csr_of_edges(n, [(i, i + 1) for i in range(n - 1)] + [(i + 1, i) for i in range(n - 1)])
    S, _ = W.scrambled(A, seed)
    assert bandwidth(S) > 1
    perm = oracle.rcm_order(S)
    assert sorted(perm.tolist()) == list(range(n))
    assert bandwidth(W.permute_symmetric(S, perm)) == 1


@pytest.mark.parametrize("N", [5, 9, 16])
def test_scrambled_grid_gets_banded(oracle, N):
    # breadth-first levels of a grid started at a corner are anti-diagonals of
    # at most N vertices, so neighbours are at most 2N - 1 apart
    A = W.laplacian_2d_5pt(N)
    S, _ = W.scrambled(A, N)
    perm = oracle.rcm_order(S)
    assert bandwidth(W.permute_symmetric(S, perm)) <= 2 * N - 1


@pytest.mark.parametrize("seed", range(6))
def test_breadth_first_properties(oracle, seed):
    """In the un-reversed sequence every vertex but a component start has an
    earlier neighbour; the first such neighbour (its parent) positions are
    non-decreasing; siblings come in (degree, index) order; starts have the
    smallest (degree, index) among the vertices left."""
    A = W.random_csr(60, 60, seed=seed, max_len=4, empty_frac=0.15)
    n = A.n_rows
    nb = [set() for _ in range(n)]
    for i in range(n):
        for k in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = int(A.col[k])
            if j != i:
                nb[i].add(j)
                nb[j].add(i)
    deg = [len(s) for s in nb]
    cm = oracle.rcm_order(A)[::-1].tolist()
    pos = {v: p for p, v in enumerate(cm)}
    assert sorted(cm) == list(range(n))
    last_parent = -1
    for p, v in enumerate(cm):
        earlier = [pos[u] for u in nb[v] if pos[u] < p]
        if not earlier:   # a component start
            left = [u for u in range(n) if pos[u] >= p]
            assert (deg[v], v) == min((deg[u], u) for u in left)
            last_parent = -1
            continue
        par = min(earlier)
        assert par >= last_parent
        if par == last_parent:
            prev = cm[p - 1]
            assert (deg[prev], prev) < (deg[v], v)
        last_parent = par


@pytest.mark.parametrize("case", ["random", "zipf", "stencil", "unsym"])
def test_library_order_equals_oracle(oracle, case):
    import paper_1012_2270_amd as rg
    if case == "random":
        A = W.random_csr(700, 700, seed=5, max_len=9, empty_frac=0.1)
    elif case == "zipf":
        A = W.zipf_matrix(3000, seed=4, max_len=200)
    elif case == "stencil":
        A, _ = W.scrambled(W.laplacian_3d_7pt(9), 7)
    else:
        A = csr_of_edges(400, [(i, (7 * i + 3) % 400) for i in range(400)], extra_diag=False)
    np.testing.assert_array_equal(rg.rgcsr_rcm_order(A), oracle.rcm_order(A))


def test_library_order_rejects_bad_input():
    import paper_1012_2270_amd as rg
    with pytest.raises(ValueError):
        rg.rgcsr_rcm_order(W.random_csr(10, 12, seed=1, max_len=3))
    A = W.random_csr(10, 10, seed=1, max_len=3)
    bad = W.CSR(10, 10, A.row_ptr, A.col.copy(), A.val)
    bad.col[bad.row_ptr[-1] - 1] = 10   # column out of range
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_rcm_order(bad)
    assert e.value.status == 2

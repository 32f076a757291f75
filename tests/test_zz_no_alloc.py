"""The allocation-free mixed-precision CG (rgcsr_cg_solve_noalloc, static
device workspace) against the allocating one (rgcsr_cg_solve) through the C
ABI: the same kernels in the same order, so the same bits, on two calls in a
row with the second smaller (the workspace keeps the first call's contents)."""
import numpy as np
import pytest

from gpu_util import dev, host, say

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


def test_noalloc_cg_matches_allocating_cg_on_two_calls(torch_cuda, oracle):
    torch = torch_cuda
    for N, dt in ((40, "bf16"), (22, "f16")):   # 64,000 rows, then 10,648
        A = W.stencil_3d_27pt_spd(N, seed=W.SEEDS["cg_spd"] + N)
        b = oracle.csr_spmv(A, W.uniform_vector(A.n_cols, N))
        Alo = rg.rgcsr_from_csr(A, value_dtype=dt)
        Ahi = rg.rgcsr_from_csr(A, value_dtype="f64")
        bd = dev(b)
        x_ref = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda:0")
        x_na = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda:0")
        say("no-alloc CG", N, dt, "rows", A.n_rows)
        st_ref = rg.rgcsr_cg_solve(Alo, Ahi, bd, x_ref, tol=1e-10, inner_tol=1e-4)
        st_na = rg.rgcsr_cg_solve_noalloc(Alo, Ahi, bd, x_na, tol=1e-10, inner_tol=1e-4)
        say("  ", st_ref, st_na)
        np.testing.assert_array_equal(host(x_na).view(np.uint64), host(x_ref).view(np.uint64))
        for k in ("outer_iterations", "inner_iterations", "relres", "converged"):
            assert st_na[k] == st_ref[k], k
        assert st_na["converged"]
        r = b - oracle.csr_spmv(A, host(x_na))
        assert np.sqrt(np.dot(r, r) / np.dot(b, b)) <= 1e-10


def test_noalloc_cg_refuses_more_rows_than_its_workspace(torch_cuda):
    torch = torch_cuda
    n = (1 << 20) + 1
    D = W.diagonal(np.full(n, 2.0))
    M = rg.rgcsr_from_csr(D, value_dtype="f32")
    bd = torch.ones(n, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    say("no-alloc CG refusal", n)
    with pytest.raises(rg.RgcsrError) as e:
        rg.rgcsr_cg_solve_noalloc(M, M, bd, x)
    assert e.value.status == 6 and "static workspace" in str(e.value)
    assert float(x.abs().max().item()) == 0.0   # nothing ran

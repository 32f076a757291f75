"""The binding refuses mismatched tensors before any call crosses the C ABI
(sizes and dtypes are checked first, so this runs without a GPU)."""
import types

import numpy as np
import pytest
import torch

import paper_1012_2270_amd as rg


def fake_matrix(n_rows=5, n_cols=4, nnz=9):
    # stands in for a device handle: only the sizes the checks read
    return types.SimpleNamespace(n_rows=n_rows, n_cols=n_cols, nnz=nnz, device=None, handle=None,
                                 value_version=0)


def t(n, dtype=torch.float32):
    return torch.zeros(n, dtype=dtype)


@pytest.mark.parametrize("kw,needle", [
    (dict(dy=t(4)), "dy has 4"),
    (dict(dy=t(5), dx=t(5)), "dx has 5"),
    (dict(dy=t(5), x=t(3)), "x has 3"),
    (dict(dy=t(5), x=t(4), dvals=t(8)), "dvals has 8"),
    (dict(dy=t(5), x=t(4), dvals=t(9, torch.float64)), "dvals has dtype"),
    (dict(dy=t(5), x=t(4, torch.float64)), "x has dtype"),
    (dict(dy=t(5), dx=t(4, torch.float64)), "dx has dtype"),
    (dict(dy=t(5, torch.float16)), "dy has dtype"),
    (dict(dy=t(5), dvals=t(9)), "dvals needs x"),
])
def test_transpose_grad_refuses_mismatch(kw, needle):
    A = fake_matrix()
    x = kw.pop("x", None)
    dy = kw.pop("dy")
    with pytest.raises(ValueError, match=needle):
        rg.rgcsr_spmv_transpose_grad(A, x, dy, **kw)


def test_transpose_grad_matching_sizes_reach_the_device_check():
    A = fake_matrix()
    with pytest.raises(ValueError, match="CUDA"):
        rg.rgcsr_spmv_transpose_grad(A, t(4), t(5), t(4), t(9))


@pytest.mark.parametrize("vals,needle", [
    (t(8), "vals has 8"),
    (t(9, torch.float16), "vals has dtype"),
    (np.zeros(10, np.float32), "vals has 10"),
    (np.zeros(9, np.int32), "vals has dtype"),
])
def test_set_values_refuses_mismatch(vals, needle):
    A = fake_matrix()
    with pytest.raises(ValueError, match=needle):
        rg.rgcsr_set_values(A, vals)
    assert A.value_version == 0


def test_set_values_matching_tensor_reaches_the_device_check():
    with pytest.raises(ValueError, match="CUDA"):
        rg.rgcsr_set_values(fake_matrix(), t(9))

"""The device-side converter (rgcsr_from_csr with CSR arrays in device
memory) against the host converter: every layout array bit for bit, the same
kernel schedule, and the same SpMV bits; malformed device input is refused."""
import numpy as np
import pytest

from gpu_util import check_spmv, dev, host, say

import paper_1012_2270_amd as rg
from paper_1012_2270_amd import workloads as W

pytestmark = pytest.mark.gpu

ARRAYS = ("gp", "short_len", "short_row", "slot_col", "long_row", "long_ptr", "long_col")
INFO = ("n_groups", "n_short", "n_long", "slots", "long_nnz", "long_work", "partials", "rows_per_lane", "pad_loads")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rg._lib.load()
    return torch


def on_device(torch, A, vals=None, **kw):
    v = A.val if vals is None else vals
    tv = torch.from_numpy(np.ascontiguousarray(v)).cuda() if isinstance(v, np.ndarray) else v
    return rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(A.row_ptr, np.int64)),
                                    dev(np.ascontiguousarray(A.col, np.int32)), tv, rg.make_opts(**kw))


def same_handles(Md, Mh):
    for k in INFO:
        assert Md.info[k] == Mh.info[k], k
    ed, eh = Md.export(), Mh.export()
    for k in ARRAYS:
        np.testing.assert_array_equal(ed[k], eh[k], err_msg=k)
    for k in ("slot_val", "long_val"):
        np.testing.assert_array_equal(ed[k].view(np.uint8), eh[k].view(np.uint8), err_msg=k)


PARAMS = [(64, 1, 1, -1), (128, 1, 1, -1), (256, 1, 1, -1), (32, 1, 1, -1), (16, 2, 1, -1), (64, 2, 1, -1),
          (64, 4, 1, -1), (8, 8, 1, -1), (64, 1, 1 << 40, 16), (64, 1, 1 << 40, 0), (64, 1, 512, 24),
          (128, 2, 1 << 40, 64), (64, 8, 1 << 40, 100), (4, 1, 1, 3), (64, 1, 7, 5), (512, 1, 3000, -1)]


@pytest.mark.parametrize("G,T,sigma,tau", PARAMS)
def test_device_converter_matches_host(torch_cuda, G, T, sigma, tau):
    A = W.random_csr(3001, 2500, seed=G + 7 * T, max_len=70, empty_frac=0.2, long_rows=5, long_len=2300,
                     dtype=np.float32)
    say("device converter", G, T, sigma, tau)
    Md = on_device(torch_cuda, A, G=G, T=T, sigma=sigma, tau=tau)
    Mh = rg.rgcsr_from_csr(A, G=G, T=T, sigma=sigma, tau=tau)
    same_handles(Md, Mh)


@pytest.mark.parametrize("src,dst", [("f32", "f32"), ("f32", "bf16"), ("f32", "f16"), ("f64", "f64"), ("f64", "f32"),
                                     ("f64", "bf16"), ("f32", "f64"), ("bf16", "f32"), ("f16", "f16")])
def test_device_converter_value_dtypes(torch_cuda, src, dst):
    """Value conversion on the device rounds exactly as the host does,
    including subnormals, signed zeros, infinities and NaN payloads."""
    torch = torch_cuda
    A = W.random_csr(1500, 1500, seed=3, max_len=40, empty_frac=0.1, dtype=np.float64)
    special = np.array([0.0, -0.0, 1e-40, -3e-39, 6e-8, 65504.0, 70000.0, np.inf, -np.inf, np.nan, 1 + 2 ** -9,
                        3.0000001], np.float64)
    v = A.val.copy()
    v[:len(special)] = special
    if src == "f64":
        tv = torch.from_numpy(v).cuda()
        hv = v
    elif src == "f32":
        hv = v.astype(np.float32)
        tv = torch.from_numpy(hv).cuda()
    else:
        tt = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16 if src == "bf16" else torch.float16)
        tv = tt.cuda()
        hv = tt.view(torch.int16).numpy().view(np.uint16) if src == "bf16" else tt.numpy()
    say("device converter dtypes", src, dst)
    Md = on_device(torch, A, vals=tv, G=64, sigma=512, tau=20, value_dtype=dst)
    Mh = rg.rgcsr_from_csr(W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, hv), G=64, sigma=512, tau=20,
                           value_dtype=dst, bf16_bits=(src == "bf16"))
    same_handles(Md, Mh)


def test_device_converter_zipf_spmv_bits(torch_cuda, oracle):
    A = W.zipf_matrix(200_000, seed=11)
    x = W.uniform_vector(A.n_cols, 25, np.float32)
    say("device converter zipf")
    Md = on_device(torch_cuda, A, G=64, sigma=512, tau=16)
    Mh = rg.rgcsr_from_csr(A, G=64, sigma=512, tau=16)
    same_handles(Md, Mh)
    yd, yh = host(Md.spmv(dev(x))), host(Mh.spmv(dev(x)))
    np.testing.assert_array_equal(yd.view(np.uint32), yh.view(np.uint32))
    check_spmv(oracle, A, x, yd)


def test_device_converter_edge_cases(torch_cuda, oracle):
    torch = torch_cuda
    cases = [W.CSR(0, 5, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)),
             W.CSR(7, 3, np.zeros(8, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)),
             W.random_csr(1, 9, seed=1, max_len=9, empty_frac=0.0, dtype=np.float32),
             W.random_csr(65, 200, seed=2, max_len=30, empty_frac=0.5, dtype=np.float32)]
    for A in cases:
        for kw in (dict(G=64), dict(G=64, sigma=1 << 40, tau=2)):
            say("device converter edge", A.n_rows, A.nnz, kw)
            Md = on_device(torch, A, **kw)
            Mh = rg.rgcsr_from_csr(A, **kw)
            same_handles(Md, Mh)
            if A.n_rows:
                x = W.uniform_vector(A.n_cols, 26, np.float32)
                check_spmv(oracle, A, x, host(Md.spmv(dev(x))))


def test_device_converter_rejects_malformed(torch_cuda):
    torch = torch_cuda
    A = W.random_csr(50, 40, seed=4, max_len=8, empty_frac=0.0, dtype=np.float32)
    bad_col = A.col.copy()
    bad_col[A.row_ptr[3]] = 40                      # out of range
    unsorted = A.col.copy()
    r = next(i for i in range(A.n_rows) if A.row_ptr[i + 1] - A.row_ptr[i] >= 2)
    unsorted[A.row_ptr[r]], unsorted[A.row_ptr[r] + 1] = unsorted[A.row_ptr[r] + 1], unsorted[A.row_ptr[r]]
    bad_rp = A.row_ptr.copy()
    bad_rp[5] = bad_rp[6] + 1                       # decreasing
    for rp, col in ((A.row_ptr, bad_col), (A.row_ptr, unsorted), (bad_rp, A.col)):
        with pytest.raises(rg.RgcsrError) as e:
            rg.rgcsr_from_csr_device(A.n_rows, A.n_cols, dev(np.ascontiguousarray(rp, np.int64)),
                                     dev(np.ascontiguousarray(col, np.int32)), dev(A.val), rg.make_opts(G=64))
        assert e.value.status == 2


def test_device_converter_keeps_csr_map(torch_cuda, oracle):
    """keep_csr_map on the device path: set_values then reproduces a host build."""
    torch = torch_cuda
    A = W.random_csr(4000, 3000, seed=5, max_len=30, long_rows=3, long_len=1500, dtype=np.float32)
    Md = on_device(torch, A, G=64, sigma=512, tau=24, keep_csr_map=True)
    theta = W.normal_vector(A.nnz, 27, np.float32)
    rg.rgcsr_set_values(Md, torch.from_numpy(theta).cuda())
    B = W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, theta)
    same_handles(Md, rg.rgcsr_from_csr(B, G=64, sigma=512, tau=24))

"""Shared helpers of the GPU parity tests (not collected as tests)."""
import sys

import numpy as np

TOL_F32 = 1e-5    # max |y - y_ref| / max(|A| |x|) for FP32 accumulation
TOL_F64 = 1e-13   # same for FP64 accumulation


def say(*a):
    """Name the case before each GPU step (the output survives a lost box)."""
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def storage_values(orc, A, dt):
    """What the device stores for A's values in dtype dt, as float64 (exact)."""
    r = orc.round_values(np.asarray(A.val, np.float32) if dt in ("f16", "bf16") else A.val, dt)
    return orc.to_f64(r, bf16_bits=(dt == "bf16"))


def check_spmv(orc, A, x, y, vals64=None, tol=TOL_F32):
    """Scaled error of y against the oracle on (possibly rounded) values."""
    from paper_1012_2270_amd import workloads as W
    B = A if vals64 is None else W.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col, vals64)
    ref = orc.csr_spmv(B, x)
    s = orc.csr_absmv(B, x)
    e = orc.scaled_error(y, ref, s)
    assert e <= tol, f"scaled error {e:.3e} > {tol:.1e}"
    return e

"""The allocation-free operator apply (mofem_op_apply_noalloc) against
mofem_op_apply, called through the C ABI: the same outputs and the same fused
<X, Y> bit for bit (same kernels, same fixed-order reduction), on two calls
in a row, the second with a smaller input (fewer items and a smaller
operator), plus the size limit of its static scratch."""
import ctypes

import numpy as np
import pytest

from gpu_cases import gpu_xnormal, to_dev, to_host

pytestmark = pytest.mark.gpu


def _call(fn, op, X, Y, dots, B):
    in_stride = op.in_shape[0] * op.in_shape[1]
    out_stride = op.shape[0] * op.shape[1]
    return fn(op.handle, ctypes.c_void_p(X.data_ptr()), in_stride, ctypes.c_void_p(Y.data_ptr()), out_stride, B,
              None, ctypes.c_void_p(dots.data_ptr()) if dots is not None else None, None)


def test_noalloc_apply_matches_apply_twice():
    import torch
    from paper_2109_01173_amd import mofem as mf
    cases = [(gpu_xnormal(2, 300, "dirichlet", 1.0), 5), (gpu_xnormal(3, 41, "neumann", 1.0), 2)]
    rng = np.random.default_rng(91)
    for G, B in cases:                       # second call: fewer items, smaller operator
        X = to_dev(rng.standard_normal((B, G.q, G.q)))
        Y0, Y1 = (torch.full_like(X, np.nan) for _ in range(2))
        d0 = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
        d1 = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
        assert _call(mf.mofem_op_apply, G.op, X, Y0, d0, B) == 0
        assert _call(mf.mofem_op_apply_noalloc, G.op, X, Y1, d1, B) == 0
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Y1), to_host(Y0))
        assert np.array_equal(to_host(d1), to_host(d0))
        assert np.all(np.isfinite(to_host(d1)))
        # without the dot the scratch is not touched
        Y2 = torch.full_like(X, np.nan)
        assert _call(mf.mofem_op_apply_noalloc, G.op, X, Y2, None, B) == 0
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Y2), to_host(Y0))


def test_noalloc_apply_rejects_batches_beyond_the_scratch():
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(1, 8, "dirichlet", 1.0)          # q = 7: one tile per item
    B = (1 << 20) // 8 + 1                            # one more item than partial sums fit (51 MB per array)
    X = torch.zeros((B, G.q, G.q), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    d = torch.zeros(B, dtype=torch.float64, device="cuda")
    assert _call(mf.mofem_op_apply_noalloc, G.op, X, Y, d, B) == mf.E_ARG   # rejected before any launch
    assert b"scratch" in mf.mofem_last_error()
    # the same batch without the dot needs no scratch
    assert _call(mf.mofem_op_apply_noalloc, G.op, X, Y, None, B) == 0
    torch.cuda.synchronize()

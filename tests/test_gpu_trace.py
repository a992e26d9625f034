"""Kernel tracing (mofem_trace_*): per-class launch counts, item counts and
times from HIP events, and the class selection."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, to_dev

pytestmark = pytest.mark.gpu


def test_trace_counts_and_selection():
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 40, "dirichlet", 1.0, precision=mf.PREC_BF16_FWD)
    X = to_dev(np.random.default_rng(0).standard_normal((3, G.q, G.q)))
    torch.cuda.synchronize()
    mf.trace_enable(True)
    G.op.apply(X)
    G.prec.apply(X)
    torch.cuda.synchronize()
    mf.trace_enable(False)
    band, x3, bf = (mf.trace_read(c) for c in (mf.TRACE_BAND, mf.TRACE_GEMM_BF16X3, mf.TRACE_GEMM_BF16))
    assert band[1] == 1 and band[2] == 3 and band[0] > 0
    assert x3[1] == 2 and x3[2] == 6 and x3[0] > 0     # the two split back transforms
    assert bf[1] == 2 and bf[2] == 6                    # the two plain forward transforms
    # only the selected classes record events
    mf.trace_select((mf.TRACE_GEMM_BF16X3,))
    mf.trace_enable(True)
    G.op.apply(X)
    G.prec.apply(X)
    torch.cuda.synchronize()
    mf.trace_enable(False)
    mf.trace_select(None)
    assert mf.trace_read(mf.TRACE_BAND)[1] == 0
    assert mf.trace_read(mf.TRACE_GEMM_BF16)[1] == 0
    assert mf.trace_read(mf.TRACE_GEMM_BF16X3)[1] == 2


def test_trace_classes_of_the_basis_split_mode():
    """The forward-BF16 mode that rounds S: two plain forward products, one
    two-product back transform (V_s split) and one split back transform."""
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 40, "dirichlet", 1.0, precision=mf.PREC_BF16_FWD_VS)
    X = to_dev(np.random.default_rng(1).standard_normal((3, G.q, G.q)))
    torch.cuda.synchronize()
    mf.trace_enable(True)
    G.prec.apply(X)
    torch.cuda.synchronize()
    mf.trace_enable(False)
    x3, x2, bf = (mf.trace_read(c) for c in (mf.TRACE_GEMM_BF16X3, mf.TRACE_GEMM_BF16X2, mf.TRACE_GEMM_BF16))
    assert x3[1] == 1 and x3[2] == 3
    assert x2[1] == 1 and x2[2] == 3
    assert bf[1] == 2 and bf[2] == 6

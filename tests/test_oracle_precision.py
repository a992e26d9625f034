"""Pins of the CPU emulation of the low-precision transforms (oracle/precision.py)."""
import numpy as np
import pytest

from oracle import precision
from oracle.problems import XNormalProblem
from oracle.solvers import SpectralPrec, mo_pcg
from workloads import L_profile, dL_profile, elliptic_F


def test_bf16_rounding_is_nearest_even():
    # exhaustive over the 65536 BF16 grid points of one binade pair: midpoints go to even
    hi = np.arange(0x3F80, 0x4080, dtype=np.uint32) << 16        # 1.0 .. 4.0
    grid = hi.view(np.float32)
    mid = ((hi + 0x8000).astype(np.uint32)).view(np.float32)      # exact midpoints
    r = precision.bf16(mid)
    even = np.where(((hi >> 16) & 1) == 0, grid, ((hi + 0x10000).astype(np.uint32)).view(np.float32))
    assert np.array_equal(r, even)
    assert np.array_equal(precision.bf16(grid), grid)
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    err = np.abs(precision.bf16(x) - x) / np.abs(x)
    assert err.max() <= 2.0 ** -8  # unit roundoff of an 8-bit significand


def test_split_product_error_levels():
    rng = np.random.default_rng(1)
    A, B = rng.standard_normal((2, 200, 200))
    ref = A @ B
    scale = np.abs(A) @ np.abs(B)
    e_hh = np.abs(precision.product(A, B, "hh") - ref).max() / scale.max()
    e_x3 = np.abs(precision.product(A, B, "x3") - ref).max() / scale.max()
    e_32 = np.abs(precision.product(A, B, "f32") - ref).max() / scale.max()
    assert 1e-4 < e_hh < 2e-2          # 2^-8 level
    assert e_x3 < 1e-5 and e_32 < 1e-5  # FP32 level
    hi, lo = precision.split(A.astype(np.float32))
    assert np.abs(hi.astype(np.float64) + lo - A.astype(np.float32)).max() <= 2.0 ** -16 * np.abs(A).max()


@pytest.mark.parametrize("m", [64, 128])
def test_iteration_counts_of_transform_precisions(m):
    """Split-BF16 everywhere and BF16 forward + split back transforms keep the
    FP64 iteration count (within one); plain BF16 everywhere does not."""
    P = XNormalProblem(2, m, "dirichlet", L_profile, dL_profile, gamma=1.0)
    S = SpectralPrec(*P.prec_pairs("sylv"))
    R = P.rhs(elliptic_F(P.n, 1.0, 1e-3, 1234))
    its = {}
    for name, modes in [("f64", ("f64",) * 4), ("x3", ("x3",) * 4), ("fwd", ("hh", "hh", "x3", "x3")),
                        ("hh", ("hh",) * 4)]:
        _, info = mo_pcg(P.apply, precision.prec_apply(S, modes), R, tol=1e-8, maxit=300)
        its[name] = info["iters"]
    assert its["x3"] <= its["f64"] + 1
    assert its["fwd"] <= its["f64"] + 1
    assert its["hh"] >= its["f64"]

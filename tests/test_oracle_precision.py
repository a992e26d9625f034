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


def test_two_product_modes_use_the_rounded_operand():
    """x2a / x2b equal the product with the BF16-rounded other operand to FP32
    accuracy (the split operand is carried to 2^-16, the rounded one exactly)."""
    rng = np.random.default_rng(4)
    A, B = rng.standard_normal((2, 150, 150))
    scale = (np.abs(A) @ np.abs(B)).max()
    Bh = precision.bf16(B).astype(np.float64)
    Ah = precision.bf16(A).astype(np.float64)
    assert np.abs(precision.product(A, B, "x2a") - A.astype(np.float32).astype(np.float64) @ Bh).max() < 1e-5 * scale
    assert np.abs(precision.product(A, B, "x2b") - Ah @ B.astype(np.float32).astype(np.float64)).max() < 1e-5 * scale
    # and they differ from the exact product at the BF16 level
    assert np.abs(precision.product(A, B, "x2a") - A @ B).max() > 1e-4 * scale


# The GPU comparison of tests/test_gpu_prec.py allows the GPU's result of a
# transform precision to differ from this emulation (same FP64 eigenbasis) by
# at most AGREE_FRAC times the emulated error against the exact FP64 inverse
# (modes that round operands to BF16: the rounding pattern is reproduced), or
# to have an error at most LEVEL_FACTOR times the emulated one with
# one-k-at-a-time FP32 sums (FP32-level modes, whose error is the summation
# order itself).  This test derives both from three summation orders on the
# CPU.
AGREE_FRAC = 0.05
LEVEL_FACTOR = 2.0


@pytest.mark.parametrize("mode", ["F32", "BF16", "BF16X3", "BF16X2", "BF16_FWD"])
def test_accumulation_order_sensitivity(mode):
    P = XNormalProblem(2, 150, "dirichlet", L_profile, dL_profile, gamma=1.0)
    S = SpectralPrec(*P.prec_pairs("sylv"))
    R = np.random.default_rng(2).standard_normal((P.q, P.q))
    Zx = S.apply(R)
    nx = np.linalg.norm(Zx)
    Z = {acc: precision.prec_apply(S, precision.MODES[mode], acc)(R) for acc in ("f32", "seq", "exact")}
    err = {acc: np.linalg.norm(Z[acc] - Zx) / nx for acc in Z}
    if mode in ("F32", "BF16X3"):
        # error at the level of the FP32 sums (F32) or of the 16-bit split
        # significand (BF16X3, 2^-17 per operand), where another summation
        # order changes a sizeable part of it: the blocked and the
        # one-k-at-a-time orders stay within a factor 1.5 of each other and
        # above a single rounding of exact sums, so LEVEL_FACTOR times the
        # larger of them covers FP32 summation orders
        assert err["seq"] < 2e-5
        assert err["exact"] <= max(err["f32"], err["seq"])
        assert max(err["f32"], err["seq"]) <= 1.5 * min(err["f32"], err["seq"])
    else:
        # BF16 rounding of operands dominates: any two summation orders agree
        # to a small fraction of the error they share
        assert err["exact"] > 1e-4
        for a, b in (("f32", "exact"), ("seq", "exact"), ("f32", "seq")):
            between = np.linalg.norm(Z[a] - Z[b]) / nx
            assert between <= AGREE_FRAC / 4 * err["exact"], (a, b, between, err)

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
    FP64 iteration count (within one), the INT8 digit products exactly; plain
    BF16 everywhere does not."""
    P = XNormalProblem(2, m, "dirichlet", L_profile, dL_profile, gamma=1.0)
    S = SpectralPrec(*P.prec_pairs("sylv"))
    R = P.rhs(elliptic_F(P.n, 1.0, 1e-3, 1234))
    its = {}
    for name, modes in [("f64", ("f64",) * 4), ("x3", ("x3",) * 4), ("fwd", ("hh", "hh", "x3", "x3")),
                        ("hh", ("hh",) * 4), ("oz", ("oz7",) * 4)]:
        _, info = mo_pcg(P.apply, precision.prec_apply(S, modes), R, tol=1e-8, maxit=300)
        its[name] = info["iters"]
    assert its["oz"] == its["f64"]
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


@pytest.mark.parametrize("mode", ["F32", "BF16", "BF16X3", "BF16X2", "BF16_FWD", "BF16_FWD_VS"])
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


# ---- error-free INT8 digit products (mode "oz7") ------------------------------
def test_ozaki_digits_reconstruct_the_rows():
    """Digits are integers within the int8 range, the remainder after s
    digits is at most 2^(-7s)/2 of the row's power of two, the exponent is
    the smallest with max |x| <= (127/128) 2^e, and 8 digits hold entries
    within a factor 4 of the row maximum exactly (their last bit lies at or
    above 2^-56 of the exponent)."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((20, 50)) * np.exp2(rng.integers(-30, 30, size=(20, 1)))
    X[3] = 0.0
    X[5, 7] = 127.0 / 128.0 * 2.0 ** 4  # at the exponent boundary
    X[5, 8] = -X[5, 7]
    for s in (2, 4, 7):
        e, D = precision.oz_digits(X, s)
        assert all(np.array_equal(d, np.rint(d)) for d in D)
        assert np.abs(D[0]).max() <= 127 and all(np.abs(d).max() <= 64 for d in D[1:])
        rec = sum(d * 2.0 ** (-7 * (p + 1)) for p, d in enumerate(D))
        rem = np.ldexp(X, -e[:, None]) - rec
        assert np.abs(rem).max() <= 2.0 ** (-7 * s) / 2
    mx = np.abs(X).max(axis=1)
    nz = mx > 0
    assert np.all(mx[nz] <= 127.0 / 128.0 * np.exp2(e[nz]))
    assert np.all(mx[nz] > 127.0 / 128.0 * np.exp2(e[nz] - 1))
    assert e[3] == 0 and e[5] == 4
    Y = rng.uniform(0.25, 1.0, (10, 40)) * rng.choice([-1.0, 1.0], (10, 40)) * np.exp2(rng.integers(-9, 9, (10, 1)))
    e8, D8 = precision.oz_digits(Y, 8)
    rec8 = sum(d * 2.0 ** (-7 * (p + 1)) for p, d in enumerate(D8))
    assert np.array_equal(np.ldexp(rec8, e8[:, None]), Y)


def test_ozaki_product_is_exact_on_short_inputs():
    """Entries of a few significant bits relative to their row (A) and column
    (B) maxima fit in two digits, so every digit product is kept and the
    result equals the exact product (integer arithmetic); row and column
    scalings by powers of two and a non-square shape catch a wrong exponent,
    a dropped diagonal or a transposed operand."""
    rng = np.random.default_rng(4)
    Ai = rng.integers(-1000, 1001, (13, 37))
    Bi = rng.integers(-1000, 1001, (37, 9))
    ra = rng.integers(-20, 20, 13)
    cb = rng.integers(-20, 20, 9)
    A = np.ldexp(Ai.astype(np.float64), ra[:, None])
    B = np.ldexp(Bi.astype(np.float64), cb[None, :])
    exact = np.ldexp((Ai @ Bi).astype(np.float64), ra[:, None] + cb[None, :])
    assert np.array_equal(precision.ozaki(A, B, 7), exact)
    assert np.array_equal(precision.product(A, B, "oz7"), exact)


def test_ozaki_error_bound_and_digit_count():
    """Against the exact product (rational arithmetic): the error per entry
    is below (s + 1) 2^(-7s) K 2^(ea + eb) plus the FP64 rounding of the
    final sums, and every further digit buys about 2^7 in accuracy."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 25))
    B = rng.standard_normal((25, 5))
    exact = np.array([[float(sum(Fraction(A[i, k]) * Fraction(B[k, j]) for k in range(25))) for j in range(5)]
                      for i in range(6)])
    ea, _ = precision.oz_digits(A, 1)
    eb, _ = precision.oz_digits(B.T, 1)
    scale = np.exp2(ea[:, None] + eb[None, :])
    errs = []
    for s in (2, 3, 4, 7):
        C = precision.ozaki(A, B, s)
        err = np.abs(C - exact)
        assert np.all(err <= (s + 1) * 2.0 ** (-7 * s) * 25 * scale + 8 * np.finfo(float).eps * np.abs(exact))
        errs.append(err.max())
    assert errs[0] > 30 * errs[1] > 30 * 30 * errs[2] and errs[3] < 1e-13 * np.abs(exact).max()


def test_ozaki_fp64_level_at_the_transform_length():
    """At the inner length of the q = 2047 transforms the seven-digit product
    stays within 5e-14 of the largest entry of the product (extended-precision
    reference; plain FP64 products are near 1e-15 here)."""
    rng = np.random.default_rng(6)
    A = rng.standard_normal((24, 2048))
    B = rng.standard_normal((2048, 16))
    ref = A.astype(np.longdouble) @ B.astype(np.longdouble)
    err = np.abs(precision.ozaki(A, B, 7) - ref).max() / np.abs(ref).max()
    assert err < 5e-14

"""CPU emulation of the low-precision spectral transforms.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The preconditioner of Sec. 4 (eqs. (55)-(59)) applied as four dense
products, Z = V_s ((V_s^T R V_t) ./ D) V_t^T, each product evaluated in one
of the working precisions of the library:
  f64  plain FP64;
  f32  operands rounded to FP32, FP32 products and sums;
  hh   operands rounded to BF16 (round to nearest even), FP32 accumulation;
  x3   operands split x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (in
       FP32), and A B ~ Ah Bh + Ah Bl + Al Bh accumulated in FP32;
  x2a  A split, B rounded to BF16:  Ah Bh + Al Bh  (the product with the
       BF16-rounded B, to FP32 accuracy);
  x2b  B split, A rounded to BF16:  Ah Bh + Ah Bl.
  oz7  FP64-accurate product from exact 7-bit integer digits (the
       error-free splitting of Ozaki, Ogita, Oishi and Rump, Numer.
       Algorithms 59 (2012), with 8-bit integer slices as in Ootomo, Ozaki
       and Yokota, IJHPCA 38 (2024)): every row of A and every column of B
       gets a power-of-two exponent above its largest magnitude and is cut
       into 7 signed base-128 digits (round to nearest); the digit products
       with p + q <= 8
       are exact integers, summed per diagonal p + q and then in FP64 from
       the smallest scale up (see ``ozaki``).
Accumulation: acc="f32" sums in FP32 (NumPy's single-precision BLAS, one
blocked accumulation order); acc="seq" adds the rank-one terms one k at a
time into FP32 sums (the longest chain of FP32 roundings, as a matrix-core
accumulator over k does); acc="exact" sums the same rounded operands in FP64
and rounds the result to FP32 once (the limit of any FP32 accumulation
order).  Their spread bounds what another FP32 summation order (the GPU's)
can change, so the GPU's result is compared with this emulation at that
level, not bit for bit.  Pins: tests/test_oracle_precision.py
(rounding against exhaustive bit-level checks, split exactness, error levels,
accumulation-order sensitivity and iteration counts of the flexible MO-PCG
with each mode).
"""
import numpy as np


def bf16(x):
    """Round FP32 values to BF16 (nearest, ties to even), returned as FP32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16(x)
    return hi, bf16(x - hi)


def _mm(A, B, acc):
    if acc == "f32":
        return A @ B
    if acc == "exact":
        return (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    raise ValueError(acc)


def _seq(pairs):
    """sum over k and over the (A, B) operand pairs of A[:, k] B[k, :], added
    one rank-one term at a time into FP32 sums (pairs innermost)."""
    A0, B0 = pairs[0]
    out = np.zeros((A0.shape[0], B0.shape[1]), dtype=np.float32)
    for k in range(A0.shape[1]):
        for A, B in pairs:
            out += np.multiply.outer(A[:, k], B[k, :]).astype(np.float32)
    return out


def oz_digits(X, s, beta=7):
    """Exponents and digits of the rows of X: the smallest e_r with
    max |X[r, :]| <= (1 - 2^-beta) 2^e_r (0 for a zero row), and s
    integer-valued arrays d_1 .. d_s, each the nearest integer (ties to even)
    to 2^beta times the remainder so far:  |d_1| <= 2^beta - 1,
    |d_p| <= 2^(beta - 1) for p > 1, and X = 2^e (sum_p d_p 2^(-beta p) + rem)
    with |rem| <= 2^(-beta s) / 2; every step is exact in FP64."""
    X = np.asarray(X, dtype=np.float64)
    f, e = np.frexp(np.abs(X).max(axis=1) if X.shape[1] else np.zeros(X.shape[0]))
    e = e + (f > 1.0 - 2.0 ** -beta)
    x = np.ldexp(X, -e[:, None])
    digits = []
    for _ in range(s):
        y = x * 2.0 ** beta
        d = np.rint(y)
        x = y - d
        digits.append(d)
    return e.astype(np.int64), digits


def ozaki(A, B, s=7, beta=7):
    """A @ B from exact digit products: A's rows and B's columns cut by
    oz_digits; the products a_p b_q with p + q <= s + 1 are exact integers
    (FP64 products of integer matrices whose sums stay below 2^53), summed
    per diagonal d = p + q; the diagonals are added in FP64 from d = s + 1
    down to 2 with their scales 2^(-beta d), then scaled by 2^(ea + eb)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape[1] * (2 ** beta - 1) ** 2 * s >= 2.0 ** 53:
        raise ValueError("inner dimension too long for exact digit sums")
    ea, Da = oz_digits(A, s, beta)
    eb, Db = oz_digits(B.T, s, beta)
    C = np.zeros((A.shape[0], B.shape[1]))
    for d in range(s + 1, 1, -1):
        acc = np.zeros_like(C)
        for p in range(1, d):
            acc += Da[p - 1] @ Db[d - p - 1].T
        C = C + acc * 2.0 ** (-beta * d)
    return np.ldexp(C, ea[:, None] + eb[None, :])


def product(A, B, mode, acc="f32"):
    """A @ B in the given transform precision, returned as FP64."""
    if mode == "f64":
        return A @ B
    if mode == "oz7":
        return ozaki(A, B, 7)
    if mode == "f32":
        A32, B32 = A.astype(np.float32), B.astype(np.float32)
        if acc == "seq":
            return _seq([(A32, B32)]).astype(np.float64)
        return _mm(A32, B32, acc).astype(np.float64)
    Ah, Al = split(A)
    Bh, Bl = split(B)
    if acc == "seq":
        pairs = {"hh": [(Ah, Bh)], "x3": [(Ah, Bh), (Ah, Bl), (Al, Bh)],
                 "x2a": [(Ah, Bh), (Al, Bh)], "x2b": [(Ah, Bh), (Ah, Bl)]}
        if mode not in pairs:
            raise ValueError(mode)
        return _seq(pairs[mode]).astype(np.float64)
    if mode == "hh":
        out = _mm(Ah, Bh, acc)
    elif mode == "x3":
        if acc == "exact":
            out = (Ah.astype(np.float64) @ Bh + Ah.astype(np.float64) @ Bl
                   + Al.astype(np.float64) @ Bh).astype(np.float32)
        else:
            out = Ah @ Bh + Ah @ Bl + Al @ Bh
    elif mode == "x2a":
        out = _mm(Ah, Bh, acc) + _mm(Al, Bh, acc) if acc == "f32" else \
            (Ah.astype(np.float64) @ Bh + Al.astype(np.float64) @ Bh).astype(np.float32)
    elif mode == "x2b":
        out = _mm(Ah, Bh, acc) + _mm(Ah, Bl, acc) if acc == "f32" else \
            (Ah.astype(np.float64) @ Bh + Ah.astype(np.float64) @ Bl).astype(np.float32)
    else:
        raise ValueError(mode)
    return out.astype(np.float64)


def prec_apply(S, modes, acc="f32"):
    """P^-1 with the four products in modes = (G1, G2, G3, G4):
    G1 = R V_t, G2 = V_s^T (.), G3 = V_s (. ./ D), G4 = (.) V_t^T.
    S: oracle.solvers.SpectralPrec (eigenbases Vs, Vt, divisor D)."""
    Vs, Vt, D = S.Vs, S.Vt, S.D

    def apply(R):
        T1 = product(R, Vt, modes[0], acc)
        T2 = product(Vs.T, T1, modes[1], acc) / D
        T3 = product(Vs, T2, modes[2], acc)
        return product(T3, Vt.T, modes[3], acc)
    return apply


# the library's transform precisions as emulation modes (G1, G2, G3, G4);
# in G1 and G4 the eigenbasis is the right operand, in G2 and G3 the left
MODES = {
    "F64": ("f64",) * 4,
    "F32": ("f32",) * 4,
    "BF16": ("hh",) * 4,
    "BF16X3": ("x3",) * 4,
    "BF16X2": ("x2a", "x2b", "x2b", "x2a"),
    "BF16_FWD": ("hh", "hh", "x3", "x3"),
    "BF16_FWD_VS": ("hh", "hh", "x2a", "x3"),
    "F64_INT8": ("oz7",) * 4,
}

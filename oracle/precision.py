"""CPU emulation of the low-precision spectral transforms.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The preconditioner of Sec. 4 (eqs. (55)-(59)) applied as four dense
products, Z = V_s ((V_s^T R V_t) ./ D) V_t^T, each product evaluated in one
of the working precisions of the library:
  f64  plain FP64;
  f32  operands rounded to FP32, FP32 products and sums;
  hh   operands rounded to BF16 (round to nearest even), FP32 accumulation;
  x3   operands split x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (in
       FP32), and A B ~ Ah Bh + Ah Bl + Al Bh accumulated in FP32.
FP32 accumulation order differs from the GPU's, so this emulates the error
level, not the bits.  Pins: tests/test_oracle_precision.py (rounding against
exhaustive bit-level checks, split exactness, error levels and iteration
counts of the flexible MO-PCG with each mode).
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


def product(A, B, mode):
    """A @ B in the given transform precision, returned as FP64."""
    if mode == "f64":
        return A @ B
    if mode == "f32":
        return (A.astype(np.float32) @ B.astype(np.float32)).astype(np.float64)
    Ah, Al = split(A)
    Bh, Bl = split(B)
    if mode == "hh":
        return (Ah @ Bh).astype(np.float64)
    if mode == "x3":
        return (Ah @ Bh + Ah @ Bl + Al @ Bh).astype(np.float64)
    raise ValueError(mode)


def prec_apply(S, modes):
    """P^-1 with the four products in modes = (G1, G2, G3, G4):
    G1 = R V_t, G2 = V_s^T (.), G3 = V_s (. ./ D), G4 = (.) V_t^T.
    S: oracle.solvers.SpectralPrec (eigenbases Vs, Vt, divisor D)."""
    Vs, Vt, D = S.Vs, S.Vt, S.D

    def apply(R):
        T1 = product(R, Vt, modes[0])
        T2 = product(Vs.T, T1, modes[1]) / D
        T3 = product(Vs, T2, modes[2])
        return product(T3, Vt.T, modes[3])
    return apply

"""GPU parity of the spectral preconditioner (mofem_prec_setup / apply).

FP64 transforms: compared with the oracle's P^{-1}(R) (SciPy eigenbasis) and
checked backward with the oracle's explicit operator P(Z) = R, bound
50 eps cond(D).  FP32, split-BF16 and BF16 transforms: norm-wise error
against the FP64 result within their arithmetic (2^-24 per FP32 rounding,
about 3 * 2^-16 per product for the split, 2^-8 for plain BF16, times the
transform depth and the growth through D^-1).
Sizes (q ~ 150..300) span several 128-wide GEMM tiles with ragged tails."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, oracle_xnormal, rel, to_dev, to_host
from oracle.solvers import SpectralPrec

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


@pytest.mark.parametrize("k,m,bc", [(2, 150, "dirichlet"), (1, 131, "neumann"), (3, 101, "dirichlet")])
def test_prec_fp64(k, m, bc):
    from paper_2109_01173_amd import mofem as mf
    gamma = 1.0
    G = gpu_xnormal(k, m, bc, gamma)
    P = oracle_xnormal(k, m, bc, gamma)
    S = SpectralPrec(*P.prec_pairs("sylv"))
    lam, mu = G.prec.eigenvalues()
    assert np.abs(lam - S.lam).max() <= 1e-12 * S.lam.max()
    assert np.abs(mu - S.mu).max() <= 1e-12 * S.mu.max()
    R = np.random.default_rng(1).standard_normal((3, P.q, P.q))
    Z = to_host(G.prec.apply(to_dev(R)))
    condD = np.abs(S.D).max() / np.abs(S.D).min()
    for b in range(3):
        assert rel(S.forward(Z[b]), R[b]) < 50 * EPS * condD
        assert rel(Z[b], S.apply(R[b])) < 1e-10
    # per-item coefficient: D = 1 + c (lam + mu), the IMEX split
    G.prec.set_coeffs(1.0, 1.0, 1.0, 0.0)
    cs = np.array([1e-3, 1e-1, 10.0])
    Z = to_host(G.prec.apply(to_dev(R), item_scale=to_dev(cs)))
    for b in range(3):
        Sb = SpectralPrec(*P.imex_prec_pairs("sylv-imex", cs[b]))
        cond_b = np.abs(Sb.D).max() / np.abs(Sb.D).min()
        assert rel(Sb.forward(Z[b]), R[b]) < 50 * EPS * cond_b
        assert rel(Z[b], Sb.apply(R[b])) < 50 * EPS * cond_b * 10
    G.prec.set_coeffs(gamma, 1.0, 1.0, 0.0)
    _ = mf


@pytest.mark.parametrize("precision,tol", [("F32", 2e-5), ("BF16X3", 2e-4), ("BF16X2", 5e-2), ("BF16", 3e-2),
                                           ("BF16_FWD", 3e-2)])
def test_prec_low_precision(precision, tol):
    from paper_2109_01173_amd import mofem as mf
    p = getattr(mf, "PREC_" + precision)
    G = gpu_xnormal(2, 150, "dirichlet", 1.0)
    R = np.random.default_rng(2).standard_normal((2, G.q, G.q))
    Z64 = to_host(G.prec.apply(to_dev(R)))
    G.prec.set_precision(p)
    Zlo = to_host(G.prec.apply(to_dev(R)))
    G.prec.set_precision(mf.PREC_F64)
    for b in range(2):
        assert rel(Zlo[b], Z64[b]) < tol
        # still a positive definite action: <R, Z> > 0
        assert np.sum(R[b] * Zlo[b]) > 0
    if precision == "BF16X2":
        # a fixed symmetric operator (the BF16-rounded basis) applied to
        # split-BF16 accuracy: <X, P^-1 Y> = <P^-1 X, Y> to ~1e-5
        G.prec.set_precision(p)
        Zx = to_host(G.prec.apply(to_dev(R[:1])))[0]
        Zy = to_host(G.prec.apply(to_dev(R[1:])))[0]
        G.prec.set_precision(mf.PREC_F64)
        a1, a2 = np.sum(R[0] * Zy), np.sum(Zx * R[1])
        assert abs(a1 - a2) <= 1e-4 * np.sqrt(np.sum(R[0] * Zx) * np.sum(R[1] * Zy))


def test_prec_tiny_and_errors():
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(1, 3, "dirichlet", 1.0)      # q = 2
    P = oracle_xnormal(1, 3, "dirichlet", 1.0)
    S = SpectralPrec(*P.prec_pairs("sylv"))
    R = np.random.default_rng(3).standard_normal((1, 2, 2))
    assert rel(to_host(G.prec.apply(to_dev(R)))[0], S.apply(R[0])) < 1e-13
    with pytest.raises(mf.MofemError):
        G.prec.set_precision(99)


@pytest.mark.parametrize("precision", ["F64", "F32", "BF16X3", "BF16X2", "BF16", "BF16_FWD"])
def test_block_tiles_agree_and_tuner(precision):
    """Both block tiles of the transforms compute the same products in the same
    k order (BF16 on 128-row tiles loads through LDS directly, on 64-row tiles
    through registers): the results agree to the last bits; the tuner picks
    one of them."""
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 150, "dirichlet", 1.0)   # q = 299: ragged against 64 and 128
    G.prec.set_precision(getattr(mf, "PREC_" + precision))
    R = to_dev(np.random.default_rng(5).standard_normal((2, G.q, G.q)))
    out = {}
    for tile in (64, 128):
        G.prec.set_tile(2, tile)
        out[tile] = to_host(G.prec.apply(R))
    assert rel(out[64], out[128]) <= 1e-15
    assert G.prec.tune(2) in (64, 128)
    assert rel(to_host(G.prec.apply(R)), out[128]) <= 1e-15
    G.prec.set_precision(mf.PREC_F64)

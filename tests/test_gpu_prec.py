"""GPU parity of the spectral preconditioner (mofem_prec_setup / apply).

FP64 transforms: compared with the oracle's P^{-1}(R) (SciPy eigenbasis) and
checked backward with the oracle's explicit operator P(Z) = R, bound
50 eps cond(D).  FP32, split-BF16 and BF16 transforms: against the oracle's
CPU emulation of the same transform precision on the same eigenbasis.
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
    S = SpectralPrec(*P.prec_pairs("sylv-matched"))   # the library's elliptic pencils
    lam, mu = G.prec.eigenvalues()
    assert np.abs(lam - S.lam).max() <= 1e-12 * S.lam.max()
    assert np.abs(mu - S.mu).max() <= 1e-12 * S.mu.max()
    R = np.random.default_rng(1).standard_normal((3, P.q, P.q))
    Z = to_host(G.prec.apply(to_dev(R)))
    condD = np.abs(S.D).max() / np.abs(S.D).min()
    for b in range(3):
        assert rel(S.forward(Z[b]), R[b]) < 50 * EPS * condD
        assert rel(Z[b], S.apply(R[b])) < 1e-10
    # per-item coefficient: D = 1 + c (lam + mu), the form of the IMEX split
    G.prec.set_coeffs(1.0, 1.0, 1.0, 0.0)
    cs = np.array([1e-3, 1e-1, 10.0])
    Z = to_host(G.prec.apply(to_dev(R), item_scale=to_dev(cs)))
    pencil_s, pencil_t, _ = P.prec_pairs("sylv-matched")
    for b in range(3):
        Sb = SpectralPrec(pencil_s, pencil_t, (1.0, cs[b], cs[b], 0.0))
        cond_b = np.abs(Sb.D).max() / np.abs(Sb.D).min()
        assert rel(Sb.forward(Z[b]), R[b]) < 50 * EPS * cond_b
        assert rel(Z[b], Sb.apply(R[b])) < 50 * EPS * cond_b * 10
    G.prec.set_coeffs(gamma, 1.0, 1.0, 0.0)
    _ = mf


@pytest.mark.parametrize("precision", ["F32", "BF16X3", "BF16X2", "BF16", "BF16_FWD", "BF16_FWD_VS"])
def test_prec_low_precision_vs_emulation(precision):
    """Each low-precision transform mode against the oracle's CPU emulation of
    that mode (oracle/precision.py: RNE BF16 / FP32 rounding of the operands,
    FP32 sums) with the SAME FP64 eigenbasis (the oracle's, handed to the
    library through mofem_prec_setup_eig), both measured against the
    oracle's exact FP64 inverse.  Modes that round operands to BF16 must
    reproduce the emulated rounding pattern: the GPU result lies within
    AGREE_FRAC of the emulated error from the emulation.  FP32-level modes,
    whose error is the summation order, must stay within LEVEL_FACTOR of the
    emulated error.  Both factors are derived on the CPU from three summation
    orders (tests/test_oracle_precision.py)."""
    from oracle import precision as em
    from paper_2109_01173_amd import mofem as mf
    from test_oracle_precision import AGREE_FRAC, LEVEL_FACTOR
    P = oracle_xnormal(2, 150, "dirichlet", 1.0)          # q = 299: ragged against 64 and 128
    S = SpectralPrec(*P.prec_pairs("sylv"))
    pr = mf.Preconditioner.from_eigen(S.lam, S.Vs, S.mu, S.Vt, (1.0, 1.0, 1.0, 0.0),
                                      precision=getattr(mf, "PREC_" + precision))
    R = np.random.default_rng(2).standard_normal((2, P.q, P.q))
    Zg = to_host(pr.apply(to_dev(R)))
    for b in range(2):
        Zx = S.apply(R[b])
        em_f32 = em.prec_apply(S, em.MODES[precision], "f32")(R[b])
        err_em = rel(em_f32, Zx)
        if precision in ("F32", "BF16X3"):
            em_seq = em.prec_apply(S, em.MODES[precision], "seq")(R[b])
            level = max(err_em, rel(em_seq, Zx))
            assert rel(Zg[b], Zx) <= LEVEL_FACTOR * level, (b, rel(Zg[b], Zx), level)
        else:
            assert rel(Zg[b], em_f32) <= AGREE_FRAC * err_em, (b, rel(Zg[b], em_f32), err_em)
        # still a positive definite action: <R, Z> > 0
        assert np.sum(R[b] * Zg[b]) > 0
    if precision == "BF16X2":
        # a fixed symmetric operator (the BF16-rounded basis) applied to
        # split-BF16 accuracy: <X, P^-1 Y> = <P^-1 X, Y> to ~1e-5
        a1, a2 = np.sum(R[0] * Zg[1]), np.sum(Zg[0] * R[1])
        assert abs(a1 - a2) <= 1e-4 * np.sqrt(np.sum(R[0] * Zg[0]) * np.sum(R[1] * Zg[1]))


def test_prec_tiny_and_errors():
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(1, 3, "dirichlet", 1.0)      # q = 2
    P = oracle_xnormal(1, 3, "dirichlet", 1.0)
    S = SpectralPrec(*P.prec_pairs("sylv-matched"))
    R = np.random.default_rng(3).standard_normal((1, 2, 2))
    assert rel(to_host(G.prec.apply(to_dev(R)))[0], S.apply(R[0])) < 1e-13
    with pytest.raises(mf.MofemError):
        G.prec.set_precision(99)


@pytest.mark.parametrize("precision", ["F64", "F32", "BF16X3", "BF16X2", "BF16", "BF16_FWD", "BF16_FWD_VS",
                                       "F64_INT8"])
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


@pytest.mark.parametrize("precision", ["BF16_FWD", "BF16X3"])
def test_block_tiles_agree_on_whole_chunks(precision):
    """q = 1023, batch 8: the 128-row BF16 tiles then fill 64-tile chunks (8 x 8
    tile blocks per XCD, two items at a time), the 64-row tiles keep the banded
    order; every item must still get exactly its own products."""
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 512, "dirichlet", 1.0)   # q = 1023: 8 x 8 tiles of 128 per item
    G.prec.set_precision(getattr(mf, "PREC_" + precision))
    R = to_dev(np.random.default_rng(6).standard_normal((8, G.q, G.q)))
    out = {}
    for tile in (64, 128):
        G.prec.set_tile(8, tile)
        out[tile] = to_host(G.prec.apply(R))
    assert rel(out[64], out[128]) <= 1e-15
    # each item alone (batch 1 never fills a chunk) gives the same result
    G.prec.set_tile(1, 128)
    for i in (0, 5):
        assert rel(to_host(G.prec.apply(R[i:i + 1]))[0], out[128][i]) <= 1e-15
    G.prec.set_precision(mf.PREC_F64)


def test_added_bands_form_the_pencils():
    """Bands added to Ks and Kt (summed by the library before the eigen-
    solves) give the preconditioner of the summed bands: Ks = B1 given as
    (B1 - M3/2) + M3/2, Kt = A + w B2 given as A with B2 added at weight w,
    against the oracle's pencils (B1, M1) x (A + w B2, M)."""
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 60, "dirichlet", 1.0)      # q = 119
    P = oracle_xnormal(2, 60, "dirichlet", 1.0)
    b = G.bands
    w = float(b["M2"].sum() / b["M1"].sum())
    pr = mf.Preconditioner(b["B1"] - 0.5 * b["M3"], b["M1"], b["A"], b["M"], (1.0, 1.0, 1.0, 0.0), 1, 1,
                           Ks_add=[(b["M3"], 0.5)], Kt_add=[(b["B2"], w)])
    S = SpectralPrec(*P.prec_pairs("sylv-matched"))
    lam, mu = pr.eigenvalues()
    assert np.abs(lam - S.lam).max() <= 1e-12 * S.lam.max()
    assert np.abs(mu - S.mu).max() <= 1e-12 * S.mu.max()
    R = np.random.default_rng(11).standard_normal((2, P.q, P.q))
    Z = to_host(pr.apply(to_dev(R)))
    for i in range(2):
        assert rel(Z[i], S.apply(R[i])) < 1e-10

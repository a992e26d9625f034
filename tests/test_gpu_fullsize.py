"""Parity at the headline size, in the launch configuration of the bench:
P2 x-normal, n = 2049 (q = 2047), Dirichlet, gamma = 1, manufactured load
plus noise, batch 16, forward-BF16 transforms (the bench's variant that also
rounds S to BF16 in the first back transform, and the one that splits it),
flexible MO-PCG to a relative residual of 1e-8 (128 x 128 transform tiles,
16-item batched launches).

The oracle's operators are dense NumPy products (about a second per item at
this size), so whole items 0 and 15 of the batch are compared: the load and
the operator element by element within the rounding bound of the smaller
operator tests, the FP64 preconditioner backward through the oracle's
explicit single-term operator, the forward-BF16 preconditioner against the
FP64 one within its arithmetic, and the solves (mixed to 1e-8, FP64 to
1e-10) by their backward errors under the oracle's load and operator and
their forward errors against the oracle's own MO-PCG solutions (recurrence
residual 1e-13)."""
import numpy as np
import pytest

from gpu_cases import oracle_abs_apply, rel, to_dev, to_host
from oracle.problems import XNormalProblem
from oracle.solvers import SpectralPrec, mo_pcg
from workloads import GEOM_AMP, L_profile, dL_profile, elliptic_batch

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps
ITEMS = (0, 15)
B = 16
MIXED = ("BF16_FWD_VS", "BF16_FWD")   # the bench's mixed mode first


@pytest.fixture(scope="module")
def full():
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.problems import XNormal
    G = XNormal(2, 1024, "dirichlet", gamma=1.0, amp=GEOM_AMP, precision=getattr(mf, "PREC_" + MIXED[0]))
    P = XNormalProblem(2, 1024, "dirichlet", L_profile, dL_profile, gamma=1.0)
    F = elliptic_batch(G.n, 1.0, B, sigma=1e-3, seed0=1234)
    S = SpectralPrec(*P.prec_pairs("sylv-matched"))   # the library's elliptic pencils
    return G, P, F, S


def test_fullsize_load_and_operator(full):
    G, P, F, _ = full
    assert G.q == 2047
    rhs = to_host(G.rhs_op.apply(to_dev(F)))
    X = np.random.default_rng(77).standard_normal((B, G.q, G.q))
    Y = to_host(G.op.apply(to_dev(X)))
    for b in ITEMS:
        ref = P.rhs(F[b])
        assert rel(rhs[b], ref) < 1e-13
        ref = P.apply(X[b])
        bound = 64 * (2 * G.kb + 1) * EPS * oracle_abs_apply(P, X[b])
        assert np.all(np.abs(Y[b] - ref) <= bound), np.abs(Y[b] - ref).max()


@pytest.mark.parametrize("mode", MIXED)
def test_fullsize_preconditioner(full, mode):
    """FP64 transforms of the library's own preconditioner backward through
    the oracle's explicit single-term operator (items 0 and 15).  The
    forward-BF16 transforms (both variants) against the oracle's CPU emulation
    of that mode (oracle/precision.py) on every item of the batch, on a
    shared eigenbasis (the oracle's, handed to the library through
    mofem_prec_setup_eig): the GPU must reproduce the emulated rounding
    pattern to AGREE_FRAC of the emulated error.  A shared basis is needed
    because the s pencil (B1, M1) has a pair of high eigenvalues about 1e-8
    apart (relative), whose eigenvectors any two solvers may rotate within
    their plane; P^{-1} does not notice, but the BF16 roundings of the
    rotated vectors differ.  An item whose emulated rounding pattern itself
    depends on the FP32 summation order (with these pencils item 6: the
    blocked and the exact-sum emulations differ by 4.5 % of its error, where
    the other items stay below 0.5 %) is held to twice that spread instead,
    the GPU's order being a third one.  The library's own forward-BF16
    preconditioner must then have the emulated error level (within a factor
    1.25) against the exact inverse.  (The error itself varies from item to
    item by a factor of about two: the few lowest modes, divided by the
    smallest D, dominate Z.)

    The variant that also rounds S (the divided coefficients) to BF16 makes
    the rounding pattern of those dominant modes depend on the FP32
    summation order: the blocked and the exact-sum emulations differ by up
    to 29 % of the error on one item, and the GPU's order, a third one,
    lands as far from the blocked one on a few items.  For that mode every
    item is held to the emulated error level (factor 1.25) and the median
    item to the emulated pattern (AGREE_FRAC); the pattern is checked item
    by item at q = 299 (tests/test_gpu_prec.py)."""
    from oracle import precision as em
    from paper_2109_01173_amd import mofem as mf
    from test_oracle_precision import AGREE_FRAC
    G, P, _, S = full
    R = np.random.default_rng(78).standard_normal((B, G.q, G.q))
    G.prec.set_precision(mf.PREC_F64)
    try:
        Z64 = to_host(G.prec.apply(to_dev(R)))
        G.prec.set_precision(getattr(mf, "PREC_" + mode))
        Zown = to_host(G.prec.apply(to_dev(R)))
    finally:
        G.prec.set_precision(getattr(mf, "PREC_" + MIXED[0]))
    condD = np.abs(S.D).max() / np.abs(S.D).min()
    for b in ITEMS:
        assert rel(S.forward(Z64[b]), R[b]) < 50 * EPS * condD
    shared = mf.Preconditioner.from_eigen(S.lam, S.Vs, S.mu, S.Vt, S.coeffs, precision=getattr(mf, "PREC_" + mode))
    Zmx = to_host(shared.apply(to_dev(R)))
    del shared
    emulate = em.prec_apply(S, em.MODES[mode], "f32")
    emulate_exact = em.prec_apply(S, em.MODES[mode], "exact")
    ratios = []
    for b in range(B):
        Zx = S.apply(R[b])
        Zem = emulate(R[b])
        err_em = rel(Zem, Zx)
        d = rel(Zmx[b], Zem)
        if mode == "BF16_FWD_VS":
            assert rel(Zmx[b], Zx) <= 1.25 * err_em, (b, rel(Zmx[b], Zx), err_em)
            ratios.append(d / err_em)
            if b in ITEMS:
                assert rel(Zown[b], Zx) <= 1.25 * err_em, (b, rel(Zown[b], Zx), err_em)
            continue
        bar = AGREE_FRAC * err_em
        if d > bar:
            bar = max(bar, 2 * rel(emulate_exact(R[b]), Zem))
        assert d <= bar, (b, d, err_em, bar)
        if b in ITEMS:
            assert rel(Zown[b], Zx) <= 1.25 * err_em, (b, rel(Zown[b], Zx), err_em)
    if ratios:
        assert np.median(ratios) <= AGREE_FRAC, ratios


@pytest.fixture(scope="module")
def oracle_ref(full):
    """The oracle's FP64 MO-PCG solutions of items 0 and 15, iterated until the
    recurrence residual is 1e-13 (about 40 iterations each): three orders
    below the FP64 path's stopping tolerance, so they stand for the exact
    solution in the forward-error checks.  Their TRUE residual cannot be
    certified below the rounding floor of one FP64 evaluation of the operator
    at this size (0.6-2e-10 measured: the true residual stagnates there), so
    it is asserted below the first-order rounding scale eps ||(|L| |U|)|| /
    ||R|| instead."""
    _, P, F, S = full
    out = {}
    for b in ITEMS:
        R = P.rhs(F[b])
        Uo, info = mo_pcg(P.apply, S.apply, R, tol=1e-13, maxit=200, check_true=False)
        floor = EPS * np.linalg.norm(oracle_abs_apply(P, Uo)) / np.linalg.norm(R)
        assert info["relres"] <= floor, (b, info["relres"], floor)
        out[b] = Uo
    return out


def _backward_under_oracle(G, P, F, Uh, b):
    """Backward error of the GPU solution of item b under the oracle's load
    and operator, and the part of it that is only the two implementations'
    rounding difference: ||Rg - Ro|| + ||G.op(U) - P.apply(U)||, both measured
    on this U (triangle inequality: back <= relres_gpu + that difference),
    plus the first-order rounding scale of one FP64 evaluation of the
    operator on U, eps ||(|L| |U|)||_F / ||R||, that the difference must stay
    under."""
    Ro = P.rhs(F[b])
    Rg = to_host(G.rhs_op.apply(to_dev(F[b:b + 1])))[0]
    LgU = to_host(G.op.apply(to_dev(Uh[b:b + 1])))[0]
    LoU = P.apply(Uh[b])
    nR = np.linalg.norm(Ro)
    back = np.linalg.norm(Ro - LoU) / nR
    diff = (np.linalg.norm(Rg - Ro) + np.linalg.norm(LgU - LoU)) / nR
    scale = EPS * np.linalg.norm(oracle_abs_apply(P, Uh[b])) / nR
    return back, diff, scale


@pytest.mark.parametrize("mode", MIXED)
def test_fullsize_solve(full, oracle_ref, mode):
    import torch
    from paper_2109_01173_amd import mofem as mf
    G, P, F, S = full
    rhs = G.rhs_op.apply(to_dev(F))
    U = torch.empty_like(rhs)
    G.prec.set_precision(getattr(mf, "PREC_" + mode))
    try:
        its, relres, _ = mf.pcg_solve(G.op, G.prec, rhs, U, tol=1e-8, maxit=300,
                                      flags=mf.PCG_FLEXIBLE | mf.PCG_ZERO_GUESS)
    finally:
        G.prec.set_precision(getattr(mf, "PREC_" + MIXED[0]))
    assert np.all(relres <= 1e-8) and its.max() <= 30
    Uh = to_host(U)
    for b in ITEMS:
        back, diff, scale = _backward_under_oracle(G, P, F, Uh, b)
        assert diff <= scale, (b, diff, scale)
        assert back <= relres[b] * (1 + 1e-12) + diff, (b, back)
        assert rel(Uh[b], oracle_ref[b]) < 1e-8, b


@pytest.mark.parametrize("precision", ["F64", "F64_INT8"])
def test_fullsize_solve_fp64(full, oracle_ref, precision):
    """The FP64-accurate paths of the bench (FP64 transforms on FP64 MFMA, or
    the same transforms from exact INT8 digit products; standard PCG) at the
    same size: every item to 1e-10 on the true residual; items 0 and 15 within
    1e-10 of the oracle's reference solution (forward) and, under the
    oracle's load and operator, within their GPU residual plus the measured
    rounding difference of the two FP64 operator evaluations (backward; that
    difference sits at the evaluation's own rounding floor, 1e-10 at this
    size, and is asserted below its first-order rounding scale)."""
    import torch
    from paper_2109_01173_amd import mofem as mf
    G, P, F, _ = full
    rhs = G.rhs_op.apply(to_dev(F))
    U = torch.empty_like(rhs)
    G.prec.set_precision(getattr(mf, "PREC_" + precision))
    try:
        its, relres, _ = mf.pcg_solve(G.op, G.prec, rhs, U, tol=1e-10, maxit=300, flags=mf.PCG_ZERO_GUESS)
    finally:
        G.prec.set_precision(getattr(mf, "PREC_" + MIXED[0]))
    assert np.all(relres <= 1e-10) and its.max() <= 40
    Uh = to_host(U)
    for b in ITEMS:
        back, diff, scale = _backward_under_oracle(G, P, F, Uh, b)
        assert diff <= scale, (b, diff, scale)
        assert back <= relres[b] * (1 + 1e-12) + diff, (b, back, diff)
        assert rel(Uh[b], oracle_ref[b]) < 1e-10, b

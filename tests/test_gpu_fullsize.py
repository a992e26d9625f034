"""Parity at the headline size, in the launch configuration of the bench:
P2 x-normal, n = 2049 (q = 2047), Dirichlet, gamma = 1, manufactured load
plus noise, batch 16, forward-BF16 transforms, flexible MO-PCG to a relative
residual of 1e-8 (128 x 128 transform tiles, 16-item batched launches).

The oracle's operators are dense NumPy products (about a second per item at
this size), so whole items 0 and 15 of the batch are compared: the load and
the operator element by element within the rounding bound of the smaller
operator tests, the FP64 preconditioner backward through the oracle's
explicit single-term operator, the forward-BF16 preconditioner against the
FP64 one within its arithmetic, and the solve by its backward error under
the oracle's operator and its forward error against the oracle's own
MO-PCG solution; the FP64 path of the bench likewise at 1e-10."""
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


@pytest.fixture(scope="module")
def full():
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.problems import XNormal
    G = XNormal(2, 1024, "dirichlet", gamma=1.0, amp=GEOM_AMP, precision=mf.PREC_BF16_FWD)
    P = XNormalProblem(2, 1024, "dirichlet", L_profile, dL_profile, gamma=1.0)
    F = elliptic_batch(G.n, 1.0, B, sigma=1e-3, seed0=1234)
    S = SpectralPrec(*P.prec_pairs("sylv"))
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


def test_fullsize_preconditioner(full):
    from paper_2109_01173_amd import mofem as mf
    G, P, _, S = full
    R = np.random.default_rng(78).standard_normal((B, G.q, G.q))
    G.prec.set_precision(mf.PREC_F64)
    try:
        Z64 = to_host(G.prec.apply(to_dev(R)))
    finally:
        G.prec.set_precision(mf.PREC_BF16_FWD)
    Zmx = to_host(G.prec.apply(to_dev(R)))
    condD = np.abs(S.D).max() / np.abs(S.D).min()
    for b in ITEMS:
        assert rel(S.forward(Z64[b]), R[b]) < 50 * EPS * condD
        assert rel(Zmx[b], Z64[b]) < 3e-2
    # every item of the batch: the mixed result within the same bound
    for b in range(B):
        assert rel(Zmx[b], Z64[b]) < 3e-2, b


@pytest.fixture(scope="module")
def oracle_u0(full):
    """The oracle's FP64 MO-PCG solution of item 0 to 1e-10 (its attainable
    accuracy at this size is a few 1e-11: eps times the operator's condition
    number)."""
    _, P, F, S = full
    Uo, info = mo_pcg(P.apply, S.apply, P.rhs(F[0]), tol=1e-10, maxit=200)
    assert info["relres"] <= 1e-10
    return Uo


def test_fullsize_solve(full, oracle_u0):
    import torch
    from paper_2109_01173_amd import mofem as mf
    G, P, F, S = full
    rhs = G.rhs_op.apply(to_dev(F))
    U = torch.empty_like(rhs)
    its, relres, _ = mf.pcg_solve(G.op, G.prec, rhs, U, tol=1e-8, maxit=300,
                                  flags=mf.PCG_FLEXIBLE | mf.PCG_ZERO_GUESS)
    assert np.all(relres <= 1e-8) and its.max() <= 30
    Uh = to_host(U)
    for b in ITEMS:
        Ro = P.rhs(F[b])
        back = np.linalg.norm(Ro - P.apply(Uh[b])) / np.linalg.norm(Ro)
        assert back <= 1.05e-8, (b, back)
    assert rel(Uh[0], oracle_u0) < 1e-8


def test_fullsize_solve_fp64(full, oracle_u0):
    """The FP64 path of the bench (FP64 transforms, standard PCG) at the same
    size: every item to 1e-10 on the true residual, item 0 against the
    oracle's solution to the oracle's own attainable accuracy."""
    import torch
    from paper_2109_01173_amd import mofem as mf
    G, P, F, _ = full
    rhs = G.rhs_op.apply(to_dev(F))
    U = torch.empty_like(rhs)
    G.prec.set_precision(mf.PREC_F64)
    try:
        its, relres, _ = mf.pcg_solve(G.op, G.prec, rhs, U, tol=1e-10, maxit=300, flags=mf.PCG_ZERO_GUESS)
    finally:
        G.prec.set_precision(mf.PREC_BF16_FWD)
    assert np.all(relres <= 1e-10) and its.max() <= 40
    Uh = to_host(U)
    # at 1e-10 the residual is near the rounding level of the operator itself:
    # under the oracle's operator the backward error may exceed the GPU's own
    # by the two operators' rounding difference (the bound of the operator test)
    Ro = P.rhs(F[15])
    back = np.linalg.norm(Ro - P.apply(Uh[15])) / np.linalg.norm(Ro)
    slack = np.linalg.norm(64 * (2 * G.kb + 1) * EPS * oracle_abs_apply(P, Uh[15])) / np.linalg.norm(Ro)
    assert back <= 1.05e-10 + slack, (back, slack)
    assert rel(Uh[0], oracle_u0) < 1e-9

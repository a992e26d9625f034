"""Pins of the oracle's preconditioners and MO-PCG (Sec. 4, Sec. 5).

* the spectral inverse satisfies P(P^{-1}(R)) = R with P written as plain
  matrix products (no eigenvectors);
* the product preconditioner of eq. (80) by eigenvectors equals two
  Cholesky solves;
* on a rectangle the preconditioner is the operator: one MO-PCG step, and
  the result equals Bartels-Stewart (scipy.linalg.solve_sylvester) applied
  to the generalised Sylvester form eqs. (52)-(54);
* Sec. 4.1: the closed-form P1 reduced solve (sine eigenvectors, eq. (65))
  equals the oracle's numerical solve;
* MO-PCG agrees with the sparse direct solve of the Kronecker system for
  k = 1..4 and lumped P1, both boundary conditions.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.problems import RectProblem, XNormalProblem
from oracle.solvers import BandedProductPrec, SpectralPrec, direct_solve, mo_pcg
from workloads import L_profile, dL_profile


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_spectral_prec_inverts_explicit_operator(k):
    P = XNormalProblem(k, 5, "dirichlet", L_profile, dL_profile, gamma=1.0)
    rng = np.random.default_rng(0)
    R = rng.standard_normal((P.q, P.q))
    for pairs in (P.prec_pairs("sylv"), P.prec_pairs("sylv-matched"), P.prec_pairs("paper-product"),
                  P.imex_prec_pairs("sylv-imex", 0.01), P.imex_prec_pairs("sylv-imex-matched", 0.01),
                  P.imex_prec_pairs("paper-imex", 0.01)):
        S = SpectralPrec(*pairs)
        Z = S.apply(R)
        # backward error of a two-sided spectral solve: a few eps times cond(D)
        assert rel(S.forward(Z), R) < 50 * np.finfo(float).eps * np.abs(S.D).max() / np.abs(S.D).min()
        # symmetric positive definite preconditioner
        X = rng.standard_normal((P.q, P.q))
        assert np.isclose(np.sum(S.apply(X) * R), np.sum(X * S.apply(R)), rtol=1e-10)
        assert np.sum(R * Z) > 0


def test_product_prec_cholesky_equals_spectral():
    P = XNormalProblem(2, 6, "dirichlet", L_profile, dL_profile)
    T = P.mat
    rng = np.random.default_rng(1)
    R = rng.standard_normal((P.q, P.q))
    S = SpectralPrec(*P.prec_pairs("paper-product"))
    B = BandedProductPrec(T["B1"], T["A"] + T["B2"])
    assert rel(S.apply(R), B.apply(R)) < 1e-11


@pytest.mark.parametrize("k,lumped", [(1, True), (2, False), (3, False)])
def test_rect_one_step_and_bartels_stewart(k, lumped):
    m = 6
    Rp = RectProblem(k, m, "neumann", lx=20.0, ly=20.0, lumped=lumped)
    c = 0.3
    rng = np.random.default_rng(2)
    Rhs = rng.standard_normal((Rp.q, Rp.q))
    S = SpectralPrec(*Rp.imex_prec_pairs("rect", c))
    U, info = mo_pcg(lambda X: Rp.apply_imex(X, c), S.apply, Rhs, tol=1e-13)
    assert info["iters"] == 1 and info["relres"] < 1e-13
    # Mx U My + c (Ax U My + Mx U Ay) = R  ->  Z1 U + U Z2 = Mx^-1 R My^-1
    n = Rp.q
    Z1 = 0.5 * np.eye(n) + c * np.linalg.solve(Rp.Mx, Rp.Ax)
    Z2 = 0.5 * np.eye(n) + c * np.linalg.solve(Rp.My.T, Rp.Ay.T).T
    Ft = np.linalg.solve(Rp.Mx, np.linalg.solve(Rp.My.T, Rhs.T).T)
    U_bs = sla.solve_sylvester(Z1, Z2, Ft)
    assert rel(U, U_bs) < 1e-10


def test_sec41_closed_form_reduced_solve():
    """Sec. 4.1: -Lap u + gamma u = f on the unit square, trimmed P1: the
    generalized Sylvester eq. (52) solved with sine eigenvectors and the
    eigenvalues of eq. (65)."""
    N, gamma = 16, 0.4
    Rp = RectProblem(1, N, "dirichlet", gamma=gamma)
    rng = np.random.default_rng(3)
    Fint = rng.standard_normal((N - 1, N - 1))
    # eq. (54): Z1 U + U Z2 = F with Z1 = M^-1 A + gamma/2 I, here F = interior nodal F
    i = np.arange(1, N)
    lamA = 2.0 * N * (1.0 - np.cos(i * np.pi / N))
    lam = ((12 * N ** 2 - gamma) * lamA + 6 * N * gamma) / (12 * N - 2 * lamA)
    X = np.sin(np.outer(i, i) * np.pi / N)
    Fh = np.linalg.solve(X, Fint) @ X
    Uh = Fh / (lam[:, None] + lam[None, :])
    U_closed = X @ Uh @ np.linalg.inv(X)
    # oracle: solve (A+g/2 M) U M + M U (A+g/2 M) = M F M with the spectral prec
    Rhs = Rp.Mx @ Fint @ Rp.My
    S = SpectralPrec(*Rp.prec_pairs())
    U, info = mo_pcg(Rp.apply, S.apply, Rhs, tol=1e-13)
    assert info["iters"] == 1
    assert rel(U, U_closed) < 1e-11


CASES = [(1, 8, False), (2, 5, False), (3, 4, False), (4, 3, False), (1, 9, True)]


@pytest.mark.parametrize("k,m,lumped", CASES)
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_pcg_equals_direct(k, m, lumped, bc):
    gamma = 1.0
    P = XNormalProblem(k, m, bc, L_profile, dL_profile, gamma=gamma, lumped=lumped)
    rng = np.random.default_rng(4)
    F = rng.standard_normal((P.n, P.n))
    Rhs = P.rhs(F)
    U_d = direct_solve(P.kron(), Rhs)
    for preset in ("sylv", "paper-product"):
        if bc == "neumann" and preset == "paper-product":
            continue    # B1 is singular with Neumann ends
        S = SpectralPrec(*P.prec_pairs(preset))
        U, info = mo_pcg(P.apply, S.apply, Rhs, tol=1e-12, maxit=2000)
        assert info["relres"] < 1e-12
        assert rel(U, U_d) < 1e-9
    # IMEX step operator
    c = 0.05
    U_d = direct_solve(P.kron(c=c, imex=True), Rhs)
    S = SpectralPrec(*P.imex_prec_pairs("sylv-imex", c))
    U, info = mo_pcg(lambda X: P.apply_imex(X, c), S.apply, Rhs, tol=1e-12)
    assert rel(U, U_d) < 1e-9


def test_pcg_tau_stop_rule_and_breakdown():
    P = XNormalProblem(2, 5, "dirichlet", L_profile, dL_profile, gamma=1.0)
    rng = np.random.default_rng(5)
    Rhs = P.rhs(rng.standard_normal((P.n, P.n)))
    S = SpectralPrec(*P.prec_pairs("sylv"))
    U, info = mo_pcg(P.apply, S.apply, Rhs, stop="tau", tau=1e-2)
    assert info["history"][-1] <= 1e-2 * info["history"][0] + 1e-15
    with pytest.raises(FloatingPointError):
        mo_pcg(lambda X: -P.apply(X), None, Rhs, tol=1e-10)


def test_matched_pencils_reduce_to_sylv_and_never_need_more_iterations():
    """The elliptic default pencils (B1, M1) x (A + w B2, M), w = the ratio of
    the total masses of M2 and M1 (a reading: the single-term preconditioner
    that keeps the operator's M1 U A and B1 U M terms exact).  On a flat
    profile L = 1 the weight is exactly 0 and M1 = M3, so they are the
    (B1, M3) x (A, M) pencils, which are then the whole operator: one
    iteration.  On the workload's profile and on a nearly flat one they need
    no more MO-PCG iterations than (B1, M3) x (A, M); likewise the IMEX
    pencils (B1, M3) x (A + w3 B2, M) against (B1, M3) x (A, M)."""
    import math
    flat = XNormalProblem(2, 12, "dirichlet", lambda s: np.ones_like(s), lambda s: np.zeros_like(s), gamma=1.0)
    ps, pt, co = flat.prec_pairs("sylv-matched")
    ps0, pt0, co0 = flat.prec_pairs("sylv")
    assert flat.full["M2"].sum() == 0.0
    assert np.array_equal(ps[1], ps0[1]) and np.array_equal(pt[0], pt0[0]) and co == co0
    R = np.random.default_rng(4).standard_normal((flat.q, flat.q))
    _, info = mo_pcg(flat.apply, SpectralPrec(ps, pt, co).apply, R, tol=1e-12, maxit=10)
    assert info["iters"] == 1
    for amp in (0.3, 0.05):
        P = XNormalProblem(2, 64, "dirichlet", lambda s, a=amp: 1 + a * np.sin(math.pi * s),
                           lambda s, a=amp: a * math.pi * np.cos(math.pi * s), gamma=1.0)
        R = P.rhs(np.random.default_rng(5).standard_normal((P.n, P.n)))
        its = {}
        for preset in ("sylv", "sylv-matched"):
            _, info = mo_pcg(P.apply, SpectralPrec(*P.prec_pairs(preset)).apply, R, tol=1e-10, maxit=100)
            its[preset] = info["iters"]
        assert its["sylv-matched"] <= its["sylv"], (amp, its)
        # the IMEX pencils with w3 B2 (heat-like c = 1e-4, and 1e-2)
        for c in (1e-4, 1e-2):
            its = {}
            for preset in ("sylv-imex", "sylv-imex-matched"):
                S = SpectralPrec(*P.imex_prec_pairs(preset, c))
                _, info = mo_pcg(lambda X: P.apply_imex(X, c), S.apply, R, tol=1e-10, maxit=100)
                its[preset] = info["iters"]
            assert its["sylv-imex-matched"] <= its["sylv-imex"], (amp, c, its)
    ps, pt, co = flat.imex_prec_pairs("sylv-imex-matched", 0.1)
    ps0, pt0, co0 = flat.imex_prec_pairs("sylv-imex", 0.1)
    assert np.array_equal(pt[0], pt0[0]) and co == co0

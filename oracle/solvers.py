"""Spectral single-term preconditioner, MO-PCG and a sparse direct solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sources in the paper:
* reduced (spectral) solve of a generalised Sylvester equation, Sec. 4,
  eqs. (52)-(59): diagonalise both one-dimensional pencils, divide in the
  spectral space by the matrix of eigenvalue sums, transform back;
* single-term preconditioners, Sec. 5 "Choice of the preconditioners",
  eq. (80), and for IMEX eq. (95);
* MO-PCG, Sec. 5, eqs. (77)-(78): PCG on matrices with the Frobenius
  product sum(sum(X o Y)).

Readings:
* the printed eq. (78) is garbled; the oracle uses
  alpha = <Q, R> / <Q, L(Q)>,  beta = <L(Q), Z_new> / <L(Q), Q>,
  Q_new = Z_new - beta Q  (a conjugation step that makes Q_new L-conjugate
  to Q; in exact arithmetic it is standard PCG);
* the paper's stopping rule needs a comparison solver; the oracle stops on
  the relative residual ||R - L(U)||_F <= tol ||R||_F (checked on the true
  residual), and offers the IMEX rule ||R^(s)|| <= tau ||R^(0)|| of Sec. 6;
* the spectral preconditioner keeps the generalised eigenvectors
  (V^T M V = I), so X^(1)^-1 of eq. (59) is V^T times the mass matrix, and
  the preconditioner inverse is Z = V_s ((V_s^T R V_t) / D) V_t^T.

Pins: tests/test_oracle_solvers.py - P(Z) = R with the explicit operator
P(U) = a Ms U Mt + bs Ks U Mt + bt Ms U Kt + d Ks U Kt; the reduced solve
against the closed-form P1 eigenpairs of Sec. 4.1; the rectangle case where
the preconditioner is the operator (one PCG step, equal to Bartels-Stewart
via scipy.linalg.solve_sylvester); PCG against the sparse direct solve of
the Kronecker system on small grids.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def frob(X, Y):
    """sum(sum(X o Y)) of Sec. 5."""
    return float(np.sum(X * Y))


class SpectralPrec:
    """Z = P^{-1}(R) with P(U) = a Ms U Mt + bs Ks U Mt + bt Ms U Kt + d Ks U Kt.

    (Ks, Ms), (Kt, Mt): symmetric pencils with Ms, Mt positive definite.
    coeffs = (a, bs, bt, d);  D_ij = a + bs lam_i + bt mu_j + d lam_i mu_j.
    """

    def __init__(self, pair_s, pair_t, coeffs):
        (Ks, Ms), (Kt, Mt) = pair_s, pair_t
        self.Ks, self.Ms, self.Kt, self.Mt = Ks, Ms, Kt, Mt
        self.coeffs = coeffs
        self.lam, self.Vs = sla.eigh(Ks, Ms)
        self.mu, self.Vt = sla.eigh(Kt, Mt)
        self.D = self.make_D(coeffs)

    def make_D(self, coeffs):
        a, bs, bt, d = coeffs
        L, M = self.lam[:, None], self.mu[None, :]
        return a + bs * L + bt * M + d * L * M

    def apply(self, R, D=None):
        D = self.D if D is None else D
        return self.Vs @ ((self.Vs.T @ R @ self.Vt) / D) @ self.Vt.T

    def forward(self, U):
        """The preconditioning operator P itself (no eigenvectors involved)."""
        a, bs, bt, d = self.coeffs
        Ks, Ms, Kt, Mt = self.Ks, self.Ms, self.Kt, self.Mt
        return a * Ms @ U @ Mt + bs * Ks @ U @ Mt + bt * Ms @ U @ Kt + d * Ks @ U @ Kt


class BandedProductPrec:
    """Inverse of the product preconditioner P(U) = Ks U Kt (eq. (80), (95))
    by two Cholesky solves; independent of any eigen-decomposition."""

    def __init__(self, Ks, Kt):
        self.cs = sla.cho_factor(Ks)
        self.ct = sla.cho_factor(Kt)

    def apply(self, R):
        Y = sla.cho_solve(self.cs, R)
        return sla.cho_solve(self.ct, Y.T).T


def mo_pcg(apply_L, prec, Rhs, U0=None, tol=1e-10, maxit=1000, stop="relres",
           tau=None, check_true=True):
    """MO-PCG of Sec. 5, eqs. (77)-(78), in the reading stated above.

    apply_L : U -> L(U);  prec : R -> P^{-1}(R)  (None = identity).
    stop    : "relres"  -> ||R_true||_F <= tol ||Rhs||_F
              "tau"     -> ||R^(s)||_F <= tau ||R^(0)||_F   (Sec. 6)
    Returns (U, info) with info = dict(iters, relres, history).
    """
    P = (lambda R: R) if prec is None else prec
    U = np.zeros_like(Rhs) if U0 is None else U0.copy()
    nrhs = np.linalg.norm(Rhs)
    if nrhs == 0.0:
        return np.zeros_like(Rhs), dict(iters=0, relres=0.0, history=[0.0])
    R = Rhs - apply_L(U)
    r0 = np.linalg.norm(R)
    target = tol * nrhs if stop == "relres" else tau * r0
    hist = [r0 / nrhs]
    it = 0
    if r0 <= target:
        return U, dict(iters=0, relres=r0 / nrhs, history=hist)
    Z = P(R)
    Q = Z.copy()
    while it < maxit:
        LQ = apply_L(Q)
        qLq = frob(Q, LQ)
        if not np.isfinite(qLq) or qLq <= 0.0:
            raise FloatingPointError("MO-PCG breakdown: <Q, L(Q)> = %r" % qLq)
        alpha = frob(Q, R) / qLq
        U = U + alpha * Q
        R = R - alpha * LQ
        it += 1
        rn = np.linalg.norm(R)
        hist.append(rn / nrhs)
        if rn <= target:
            if not check_true:
                break
            Rt = Rhs - apply_L(U)
            if np.linalg.norm(Rt) <= target:
                break
            R = Rt              # restart on the true residual
            Z = P(R)
            Q = Z.copy()
            continue
        Z = P(R)
        beta = frob(LQ, Z) / qLq
        Q = Z - beta * Q
    relres = np.linalg.norm(Rhs - apply_L(U)) / nrhs
    return U, dict(iters=it, relres=relres, history=hist)


def direct_solve(K, Rhs):
    """Sparse direct solve of K vec_r(U) = vec_r(Rhs) (the vector form
    eq. (68)); small grids only."""
    q_s, q_t = Rhs.shape
    x = spla.spsolve(K.tocsc(), Rhs.reshape(-1))
    return np.asarray(x).reshape(q_s, q_t)

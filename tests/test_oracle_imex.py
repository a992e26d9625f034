"""Pins of the oracle's IMEX Euler steps and DIB kinetics (Sec. 6, Sec. 7).

* heat equation with Neumann ends and f = 0 conserves the discrete mass
  sum(M3 U M) (the stiffness terms annihilate constants);
* (eta, theta) = (0, 1/2) is a fixed point of the DIB step with D = 9C/11;
* the kinetics' Jacobian at the equilibrium equals hand-derived partial
  derivatives and puts the cap parameter set in the Turing regime;
* a single generalised eigenmode grows by the closed-form 2 x 2
  amplification matrix G = diag(1/(1 + tau kappa), 1/(1 + tau d kappa))
  (I + tau rho J) (linearised step, small amplitude);
* one step equals a sparse direct solve of the vector form eq. (87).
"""
import json
import math
import os

import numpy as np
import scipy.linalg as sla

from oracle import imex
from oracle.problems import RectProblem, XNormalProblem
from oracle.solvers import SpectralPrec, direct_solve, mo_pcg
from workloads import L_profile, dL_profile, dib_params

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def make_solver(P, preset="sylv-imex"):
    def solve(c, R, U0):
        S = SpectralPrec(*P.imex_prec_pairs(preset, c))
        U, _ = mo_pcg(lambda X: P.apply_imex(X, c), S.apply, R, U0=U0, tol=1e-13)
        return U
    return solve


def test_heat_neumann_mass_conservation():
    P = XNormalProblem(4, 3, "neumann", L_profile, dL_profile)
    U = np.random.default_rng(0).random((P.q, P.q))
    solve = make_solver(P)
    m0 = P.mass_apply(U).sum()
    for _ in range(20):
        U = imex.imex_step(P, U, 1e-3, 0.1, solve)
    assert abs(P.mass_apply(U).sum() - m0) < 1e-13 * abs(m0)


def test_dib_parameters_and_equilibrium():
    g = GOLDEN["dib_parameters"]
    p = dib_params()
    for key in ("alpha", "gamma", "A1", "k2", "k3", "d_theta"):
        assert p[key] == g[key]
    for key in ("A2", "B", "C"):
        assert p[key] == g["cap"][key]
    e, th = g["equilibrium"]
    assert imex.dib_f(e, th, p) == 0.0
    assert abs(imex.dib_g(e, th, p)) < 1e-15
    # the printed D leaves a nonzero reaction at (0, 1/2) for C = 7
    q = dict(p, D=g["D_printed"])
    assert abs(imex.dib_g(e, th, q)) > 1.0
    # fixed point of the full discrete step (lumped P1 rectangle)
    R = RectProblem(1, 8, "neumann", lx=20.0, ly=20.0, lumped=True)
    eta = np.zeros((R.q, R.q))
    theta = np.full((R.q, R.q), 0.5)
    e1, t1 = imex.rds_step(R, eta, theta, 1e-2, p, make_solver(R, "rect"))
    assert np.abs(e1).max() < 1e-14 and np.abs(t1 - 0.5).max() < 1e-14


def jacobian_by_hand(eta, th, p):
    a, gm = p["alpha"], p["gamma"]
    fe = p["A1"] * (1 - th) - 3 * p["A2"] * eta ** 2
    ft = -p["A1"] * eta - p["B"]
    ge = (p["C"] * p["k2"] * (1 - th) * (1 - gm * (1 - th))
          - p["D"] * th * (1 + gm * th) * p["k3"])
    gt = (p["C"] * (1 + p["k2"] * eta) * (-(1 - gm * (1 - th)) + gm * (1 - th))
          - p["D"] * (1 + 2 * gm * th) * (1 + p["k3"] * eta))
    return np.array([[fe, ft], [ge, gt]])


def test_kinetics_jacobian_and_turing_regime():
    p = dib_params()
    rng = np.random.default_rng(1)
    for eta, th in [(0.0, 0.5)] + [tuple(rng.uniform(-0.5, 1.0, 2)) for _ in range(4)]:
        J = jacobian_by_hand(eta, th, p)
        h = 1e-6
        Jfd = np.array([
            [(imex.dib_f(eta + h, th, p) - imex.dib_f(eta - h, th, p)) / (2 * h),
             (imex.dib_f(eta, th + h, p) - imex.dib_f(eta, th - h, p)) / (2 * h)],
            [(imex.dib_g(eta + h, th, p) - imex.dib_g(eta - h, th, p)) / (2 * h),
             (imex.dib_g(eta, th + h, p) - imex.dib_g(eta, th - h, p)) / (2 * h)]])
        assert np.allclose(J, Jfd, rtol=1e-7, atol=1e-7)
    J = jacobian_by_hand(0.0, 0.5, p)
    d = p["d_theta"]
    tr, det = np.trace(J), np.linalg.det(J)
    assert tr < 0 and det > 0                                  # stable without diffusion
    assert d * J[0, 0] + J[1, 1] > 2 * math.sqrt(d * det)     # diffusion-driven instability


def test_linear_mode_amplification():
    p = dib_params()
    R = RectProblem(2, 5, "neumann", lx=20.0, ly=20.0)
    lam, Vx = sla.eigh(R.Ax, R.Mx)
    mu, Vy = sla.eigh(R.Ay, R.My)
    i, j = 3, 2
    mode = np.outer(Vx[:, i], Vy[:, j])
    eps = 1e-7
    a0 = np.array([1.0, -0.4]) * eps
    eta = a0[0] * mode
    theta = 0.5 + a0[1] * mode
    tau = 1e-2
    e1, t1 = imex.rds_step(R, eta, theta, tau, p, make_solver(R, "rect"))
    # project back on the mode with the mass inner product
    proj = lambda U: np.sum((R.Mx @ Vx[:, i]) * (U @ (R.My @ Vy[:, j])))
    a1 = np.array([proj(e1), proj(t1 - 0.5)])
    kappa = lam[i] + mu[j]
    J = jacobian_by_hand(0.0, 0.5, p)
    G = np.diag([1 / (1 + tau * kappa), 1 / (1 + tau * p["d_theta"] * kappa)]) @ (
        np.eye(2) + tau * p["rho"] * J)
    assert np.allclose(a1, G @ a0, rtol=1e-5, atol=1e-13)


def test_imex_step_equals_direct():
    P = XNormalProblem(2, 4, "dirichlet", L_profile, dL_profile)
    U = np.random.default_rng(2).random((P.q, P.q))
    tau, d = 1e-2, 0.1
    fU = np.sin(U)
    U1 = imex.imex_step(P, U, tau, d, make_solver(P), fU)
    Ud = direct_solve(P.kron(c=d * tau, imex=True), P.rhs_imex(U, tau, fU))
    assert np.linalg.norm(U1 - Ud) / np.linalg.norm(Ud) < 1e-11

"""Reverse-mode (adjoint) gradients of the MO-FEM solve and of IMEX Euler
rollouts.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper defines the discrete maps but does not differentiate them; the
gradients below are the exact derivatives of those maps, derived by hand:

* Elliptic solve (Sec. 5, eqs. (73)-(74)): U = L_gamma^{-1}(M3r F Mr^T), with
  M3r, Mr the row-trimmed mass matrices of the full-node load.  For a scalar
  loss J(U) with G = dJ/dU, the operator is symmetric (its Kronecker matrix,
  eqs. (35)/(45), is), so the adjoint state is a second solve with the same
  operator, Lambda = L_gamma^{-1}(G), and
      dJ/dF     = M3r^T Lambda Mr,
      dJ/dgamma = -<Lambda, M3 U M>   (d L_gamma / d gamma = M3 (.) M).
* IMEX Euler step (Sec. 6, eqs. (91)-(93); Sec. 7, eq. (98)):
      U+ = L_c^{-1}(M3 (U + tau rho f(U, V)) M),  c = d tau,
  and likewise V+ with g and its own d.  Given lam+ = dJ/dU+ (and for V+),
      mu  = L_c^{-1}(lam+),  nu = M3 mu M,
      dJ/dU = nu_U + tau rho (f_U o nu_U + g_U o nu_V),
      dJ/dV = nu_V + tau rho (f_V o nu_U + g_V o nu_V),
      dJ/dd += -tau <mu, K(U+)>,
  where K is the stiffness part of L_c = mass + c K and o the entrywise
  product (the kinetics act node by node).

Pins: tests/test_oracle_adjoint.py checks every gradient against central
finite differences of the forward maps (directional derivatives along random
directions, and the scalar parameters), on problems small enough for sparse
direct solves.
"""
import numpy as np

from .imex import dib_f, dib_g
from .solvers import frob


def kinetics_partials(eta, theta, p):
    """Entrywise partial derivatives of the DIB kinetics eqs. (99)-(100):
    returns (f_eta, f_theta, g_eta, g_theta)."""
    A1, A2, B, C, D = p["A1"], p["A2"], p["B"], p["C"], p["D"]
    ga, k2, k3 = p["gamma"], p["k2"], p["k3"]
    f_e = A1 * (1.0 - theta) - 3.0 * A2 * eta ** 2
    f_t = -A1 * eta - B
    g_e = C * k2 * (1.0 - theta) * (1.0 - ga * (1.0 - theta)) - D * k3 * theta * (1.0 + ga * theta)
    g_t = (C * (1.0 + k2 * eta) * (-1.0 + 2.0 * ga * (1.0 - theta))
           - D * (1.0 + k3 * eta) * (1.0 + 2.0 * ga * theta))
    return f_e, f_t, g_e, g_t


def elliptic_gradients(P, U, G, solve):
    """dJ/dF (n x n, full nodes) and dJ/dgamma of an elliptic solve.

    P: XNormalProblem; U: the solution; G = dJ/dU; solve(R) returns
    L_gamma^{-1}(R)."""
    Lam = solve(G)
    dF = P.M3_rows.T @ Lam @ P.M_rows
    dgamma = -frob(Lam, P.mass_apply(U))
    return dF, dgamma, Lam


def rds_rollout(P, eta, theta, tau, p, nsteps, solve, d_eta=1.0):
    """Forward DIB rollout, all states kept: [(eta0, theta0), ..., (etaN, thetaN)].
    solve(c, R, U0) returns L_c^{-1}(R); d_eta is 1 in the model."""
    states = [(eta, theta)]
    for _ in range(nsteps):
        fe = p["rho"] * dib_f(eta, theta, p)
        ge = p["rho"] * dib_g(eta, theta, p)
        eta_n = solve(tau * d_eta, P.rhs_imex(eta, tau, fe), eta)
        theta_n = solve(tau * p["d_theta"], P.rhs_imex(theta, tau, ge), theta)
        eta, theta = eta_n, theta_n
        states.append((eta, theta))
    return states


def rds_gradients(P, states, tau, p, lam_eta, lam_theta, solve, d_eta=1.0):
    """Reverse sweep over a DIB rollout.

    states: the forward states (from rds_rollout); lam_*: dJ/d(final state).
    Returns dJ/deta0, dJ/dtheta0, dJ/dd_eta, dJ/dd_theta (d_eta = 1 in the
    model; its gradient is still defined)."""
    d_theta = p["d_theta"]
    grad_de = grad_dt = 0.0
    for n in range(len(states) - 2, -1, -1):
        eta, theta = states[n]
        eta1, theta1 = states[n + 1]
        mu_e = solve(tau * d_eta, lam_eta, None)
        mu_t = solve(tau * d_theta, lam_theta, None)
        grad_de += -tau * frob(mu_e, P.apply(eta1, gamma=0.0))
        grad_dt += -tau * frob(mu_t, P.apply(theta1, gamma=0.0))
        nu_e = P.mass_apply(mu_e)
        nu_t = P.mass_apply(mu_t)
        f_e, f_t, g_e, g_t = kinetics_partials(eta, theta, p)
        r = tau * p["rho"]
        lam_eta = nu_e + r * (f_e * nu_e + g_e * nu_t)
        lam_theta = nu_t + r * (f_t * nu_e + g_t * nu_t)
    return lam_eta, lam_theta, grad_de, grad_dt


def heat_rollout(P, U, tau, d, nsteps, solve):
    """Forward heat rollout (f = 0), all states kept."""
    states = [U]
    for _ in range(nsteps):
        U = solve(d * tau, P.rhs_imex(U, tau), U)
        states.append(U)
    return states


def heat_gradients(P, states, tau, d, lam, solve):
    """Reverse sweep of a heat rollout: dJ/dU0 and dJ/dd."""
    grad_d = 0.0
    for n in range(len(states) - 2, -1, -1):
        mu = solve(d * tau, lam, None)
        grad_d += -tau * frob(mu, P.apply(states[n + 1], gamma=0.0))
        lam = P.mass_apply(mu)
    return lam, grad_d

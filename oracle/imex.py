"""IMEX Euler time stepping of MO-FEM and the DIB reaction kinetics.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sources in the paper:
* IMEX Euler for the semi-discrete system, Sec. 6, eqs. (87)-(88), and its
  matrix-oriented form eqs. (89)-(94): each step solves
  L_c(U^{n+1}) = M3 (U^n + tau f(U^n)) M with c = d tau;
* the DIB reaction-diffusion model, Sec. 7, eq. (98), with kinetics
  eqs. (99)-(100) and the space-time rescaling rho;
* the parameters of eq. (103) and Sec. 7.1 (cap set).

Readings:
* N_T = T / tau steps, n = 0 .. N_T - 1 (eq. (89) prints k = 0 .. N_T);
* the printed D = 3.2727 does not make (0, 1/2) an equilibrium for C = 7;
  the oracle takes D from the parameter dictionary it is given and the
  configurations use D = 9 C / 11, the value for which g(0, 1/2) = 0
  (the paper calls (0, 1/2) the homogeneous equilibrium).

Pins: tests/test_oracle_imex.py - mass conservation of the Neumann heat
equation, the homogeneous equilibrium as a fixed point, linear-mode growth
factors against the closed-form 2 x 2 amplification matrix, the Jacobian
entries of the kinetics against hand-derived partial derivatives, and one
step against a sparse direct solve.
"""
import numpy as np


def dib_f(eta, theta, p):
    """eq. (99): f = A1 (1 - theta) eta - A2 eta^3 - B (theta - alpha)."""
    return p["A1"] * (1.0 - theta) * eta - p["A2"] * eta ** 3 - p["B"] * (theta - p["alpha"])


def dib_g(eta, theta, p):
    """eq. (100): g = C (1 + k2 eta)(1 - theta)[1 - gamma (1 - theta)]
                     - D theta (1 + gamma theta)(1 + k3 eta)."""
    return (p["C"] * (1.0 + p["k2"] * eta) * (1.0 - theta) * (1.0 - p["gamma"] * (1.0 - theta))
            - p["D"] * theta * (1.0 + p["gamma"] * theta) * (1.0 + p["k3"] * eta))


def imex_step(problem, U, tau, d, solve, fU=None):
    """One IMEX Euler step of u_t - d Lap u = f (eqs. (91), (93)).

    solve(c, R, U0) must return the solution of L_c(X) = R (initial guess U0).
    """
    R = problem.rhs_imex(U, tau, fU)
    return solve(d * tau, R, U)


def rds_step(problem, eta, theta, tau, p, solve):
    """One IMEX Euler step of the DIB system eq. (98):
    eta_t - Lap eta = rho f,  theta_t - d_theta Lap theta = rho g."""
    fe = p["rho"] * dib_f(eta, theta, p)
    ge = p["rho"] * dib_g(eta, theta, p)
    eta_new = imex_step(problem, eta, tau, 1.0, solve, fe)
    theta_new = imex_step(problem, theta, tau, p["d_theta"], solve, ge)
    return eta_new, theta_new

"""Pins of the oracle's adjoint gradients (oracle/adjoint.py) against central
finite differences of the forward maps.

The forward maps are solved with sparse direct solves of the Kronecker
systems, so the finite differences only carry the O(h^2) truncation of the
central difference (zero for the loss's dependence on F, which is quadratic)
and rounding.  A wrong sign, a transposed factor or a dropped term in an
adjoint formula shows as an O(1) relative mismatch."""
import numpy as np
import pytest

from oracle import adjoint
from oracle.imex import dib_f, dib_g
from oracle.problems import RectProblem, XNormalProblem
from oracle.solvers import direct_solve, frob
from workloads import L_profile, dL_profile, dib_params


def elliptic_forward(k, m, bc, gamma, F):
    P = XNormalProblem(k, m, bc, L_profile, dL_profile, gamma=gamma)
    K = P.kron()
    U = direct_solve(K, P.rhs(F))
    return P, K, U


@pytest.mark.parametrize("k,m,bc", [(2, 5, "dirichlet"), (1, 8, "neumann"), (3, 3, "dirichlet")])
def test_elliptic_gradients_vs_central_differences(k, m, bc):
    rng = np.random.default_rng(11)
    gamma = 1.3
    P = XNormalProblem(k, m, bc, L_profile, dL_profile, gamma=gamma)
    n = P.n
    F = rng.standard_normal((n, n))
    Ut = rng.standard_normal((P.q, P.q))

    def loss(F_, g_):
        _, _, U_ = elliptic_forward(k, m, bc, g_, F_)
        return 0.5 * np.sum((U_ - Ut) ** 2)

    _, K, U = elliptic_forward(k, m, bc, gamma, F)
    G = U - Ut
    dF, dgamma, _ = adjoint.elliptic_gradients(P, U, G, lambda R: direct_solve(K, R))
    assert dF.shape == (n, n)
    # J is quadratic in F: the central difference is exact up to rounding
    for _ in range(3):
        E = rng.standard_normal((n, n))
        h = 1e-3
        fd = (loss(F + h * E, gamma) - loss(F - h * E, gamma)) / (2 * h)
        assert abs(fd - frob(dF, E)) <= 1e-8 * max(1.0, abs(fd))
    h = 1e-5
    fd = (loss(F, gamma + h) - loss(F, gamma - h)) / (2 * h)
    assert abs(fd - dgamma) <= 1e-6 * max(1.0, abs(fd))


def dib_problem():
    return RectProblem(1, 6, "neumann", lx=20.0, ly=20.0, lumped=True)


def dib_solver(P):
    cache = {}

    def solve(c, R, U0):
        key = round(c, 15)
        if key not in cache:
            cache[key] = P.kron(c=c, imex=True)
        return direct_solve(cache[key], R)
    return solve


def test_dib_rollout_gradients_vs_central_differences():
    rng = np.random.default_rng(5)
    P = dib_problem()
    p = dib_params()
    tau, nsteps = 1e-2, 4
    eta0 = 1e-2 * rng.standard_normal((P.q, P.q))
    theta0 = 0.5 + 1e-2 * rng.standard_normal((P.q, P.q))
    Te, Tt = rng.standard_normal((2, P.q, P.q))
    solve = dib_solver(P)

    def loss(e0, t0, pp):
        st = adjoint.rds_rollout(P, e0, t0, tau, pp, nsteps, solve)
        e, t = st[-1]
        return 0.5 * np.sum((e - Te) ** 2) + 0.5 * np.sum((t - Tt) ** 2), st

    J, st = loss(eta0, theta0, p)
    e, t = st[-1]
    ge0, gt0, gde, gdt = adjoint.rds_gradients(P, st, tau, p, e - Te, t - Tt, solve)
    # directions in the initial state
    for _ in range(2):
        Ee, Et = rng.standard_normal((2, P.q, P.q))
        h = 1e-6
        fd = (loss(eta0 + h * Ee, theta0 + h * Et, p)[0] - loss(eta0 - h * Ee, theta0 - h * Et, p)[0]) / (2 * h)
        an = frob(ge0, Ee) + frob(gt0, Et)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))
    # d_theta (a model parameter)
    h = 1e-5 * p["d_theta"]
    pp, pm = dict(p), dict(p)
    pp["d_theta"] += h
    pm["d_theta"] -= h
    fd = (loss(eta0, theta0, pp)[0] - loss(eta0, theta0, pm)[0]) / (2 * h)
    assert abs(fd - gdt) <= 1e-6 * max(1.0, abs(fd))
    # d_eta: the model fixes it at 1; its gradient is still defined
    def loss_de(de):
        st_ = adjoint.rds_rollout(P, eta0, theta0, tau, p, nsteps, solve, d_eta=de)
        e_, t_ = st_[-1]
        return 0.5 * np.sum((e_ - Te) ** 2) + 0.5 * np.sum((t_ - Tt) ** 2)
    h = 1e-5
    fd = (loss_de(1.0 + h) - loss_de(1.0 - h)) / (2 * h)
    assert abs(fd - gde) <= 1e-6 * max(1.0, abs(fd))


def test_heat_rollout_gradients_vs_central_differences():
    rng = np.random.default_rng(8)
    P = XNormalProblem(2, 4, "neumann", L_profile, dL_profile)
    tau, d, nsteps = 1e-2, 0.1, 5
    U0 = rng.random((P.q, P.q))
    Ut = rng.random((P.q, P.q))

    def solve(c, R, U0_):
        return direct_solve(P.kron(c=c, imex=True), R)

    def loss(U0_, d_):
        st = adjoint.heat_rollout(P, U0_, tau, d_, nsteps, solve)
        return 0.5 * np.sum((st[-1] - Ut) ** 2), st

    J, st = loss(U0, d)
    g0, gd = adjoint.heat_gradients(P, st, tau, d, st[-1] - Ut, solve)
    E = rng.standard_normal((P.q, P.q))
    h = 1e-4
    fd = (loss(U0 + h * E, d)[0] - loss(U0 - h * E, d)[0]) / (2 * h)
    assert abs(fd - frob(g0, E)) <= 1e-8 * max(1.0, abs(fd))
    h = 1e-6
    fd = (loss(U0, d + h)[0] - loss(U0, d - h)[0]) / (2 * h)
    assert abs(fd - gd) <= 1e-6 * max(1.0, abs(fd))


def test_kinetics_partials_vs_central_differences():
    rng = np.random.default_rng(3)
    p = dib_params()
    eta = 0.3 * rng.standard_normal(50)
    th = 0.5 + 0.3 * rng.standard_normal(50)
    f_e, f_t, g_e, g_t = adjoint.kinetics_partials(eta, th, p)
    h = 1e-6
    assert np.allclose(f_e, (dib_f(eta + h, th, p) - dib_f(eta - h, th, p)) / (2 * h), rtol=1e-7, atol=1e-7)
    assert np.allclose(f_t, (dib_f(eta, th + h, p) - dib_f(eta, th - h, p)) / (2 * h), rtol=1e-7, atol=1e-7)
    assert np.allclose(g_e, (dib_g(eta + h, th, p) - dib_g(eta - h, th, p)) / (2 * h), rtol=1e-7, atol=1e-7)
    assert np.allclose(g_t, (dib_g(eta, th + h, p) - dib_g(eta, th - h, p)) / (2 * h), rtol=1e-7, atol=1e-7)

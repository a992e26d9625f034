"""GPU parity of the adjoint (reverse-mode) path: torch.autograd through the
MO-PCG solve and through checkpointed IMEX rollouts, against the oracle's
hand-derived adjoints (oracle/adjoint.py, sparse direct solves) and against
central finite differences of the GPU forward map (relative 1e-5)."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, oracle_xnormal, rel, to_dev, to_host
from oracle import adjoint
from oracle.problems import RectProblem
from oracle.solvers import direct_solve, frob
from workloads import dib_initial, dib_params

pytestmark = pytest.mark.gpu


def _kin(p):
    return [p["rho"], p["A1"], p["A2"], p["B"], p["C"], p["D"], p["alpha"], p["gamma"], p["k2"], p["k3"]]


@pytest.mark.parametrize("precision,flags,tol_o", [("F64", 0, 1e-9), ("BF16X3", 1, 1e-7)])
def test_elliptic_adjoint(precision, flags, tol_o):
    import torch
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.autograd import EllipticSolve
    k, m, gamma, B = 2, 20, 1.0, 2
    G = gpu_xnormal(k, m, "dirichlet", gamma, precision=getattr(mf, "PREC_" + precision))
    P = oracle_xnormal(k, m, "dirichlet", gamma)
    rng = np.random.default_rng(21)
    F = rng.standard_normal((B, G.n, G.n))
    Ut = rng.standard_normal((B, G.q, G.q))
    Ft = to_dev(F).requires_grad_(True)
    gt = torch.tensor(gamma, dtype=torch.float64, device="cuda", requires_grad=True)
    tol = 1e-13 if precision == "F64" else 1e-11
    U = EllipticSolve.apply(Ft, gt, G, tol, 500, flags)
    J = 0.5 * ((U - to_dev(Ut)) ** 2).sum()
    J.backward()
    dF = to_host(Ft.grad)
    dg = float(gt.grad)
    # oracle adjoint, direct solves
    K = P.kron()
    dg_o = 0.0
    for b in range(B):
        Uo = direct_solve(K, P.rhs(F[b]))
        dFo, dgo, _ = adjoint.elliptic_gradients(P, Uo, Uo - Ut[b], lambda R: direct_solve(K, R))
        assert rel(dF[b], dFo) < tol_o
        dg_o += dgo
    assert abs(dg - dg_o) < tol_o * abs(dg_o)

    # central differences of the GPU forward map
    def loss(F_, G_):
        with torch.no_grad():
            U_ = EllipticSolve.apply(to_dev(F_), torch.tensor(G_.gamma, dtype=torch.float64), G_, tol, 500, flags)
            return 0.5 * float(((U_ - to_dev(Ut)) ** 2).sum())
    E = rng.standard_normal(F.shape)
    h = 1e-3
    fd = (loss(F + h * E, G) - loss(F - h * E, G)) / (2 * h)
    assert abs(fd - float(np.sum(dF * E))) < 1e-5 * abs(fd)
    h = 1e-4
    Gp = gpu_xnormal(k, m, "dirichlet", gamma + h, precision=getattr(mf, "PREC_" + precision))
    Gm = gpu_xnormal(k, m, "dirichlet", gamma - h, precision=getattr(mf, "PREC_" + precision))
    fd = (loss(F, Gp) - loss(F, Gm)) / (2 * h)
    assert abs(fd - dg) < 1e-5 * abs(fd)


def test_dib_rollout_adjoint_checkpointed():
    import torch
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.autograd import ImexRollout
    from paper_2109_01173_amd.problems import Rect
    p = dib_params()
    tau, nsteps = 1e-2, 9
    G = Rect(1, 12, "neumann", length=20.0, lumped=True, imex=True)
    P = RectProblem(1, 12, "neumann", lx=20.0, ly=20.0, lumped=True)
    eta0, theta0 = dib_initial(P.q, seed=7, amp=1e-2)
    rng = np.random.default_rng(4)
    Te, Tt = rng.standard_normal((2, P.q, P.q))
    target = to_dev(np.stack([Te, Tt]))
    s0 = to_dev(np.stack([eta0, theta0])).requires_grad_(True)
    d = torch.tensor([1.0, p["d_theta"]], dtype=torch.float64, device="cuda", requires_grad=True)
    out = ImexRollout.apply(s0, d, G, tau, nsteps, mf.KIN_DIB, _kin(p), 1e-13, 50, 0, 4)
    J = 0.5 * ((out - target) ** 2).sum()
    J.backward()
    gs0 = to_host(s0.grad)
    gd = to_host(d.grad)

    cache = {}

    def solve(c, R, U0):
        key = round(c, 15)
        if key not in cache:
            cache[key] = P.kron(c=c, imex=True)
        return direct_solve(cache[key], R)
    st = adjoint.rds_rollout(P, eta0, theta0, tau, p, nsteps, solve)
    e, t = st[-1]
    assert rel(to_host(out)[0], e) < 1e-11 and rel(to_host(out)[1], t) < 1e-11
    ge0, gt0, gde, gdt = adjoint.rds_gradients(P, st, tau, p, e - Te, t - Tt, solve)
    assert rel(gs0[0], ge0) < 1e-9 and rel(gs0[1], gt0) < 1e-9
    assert abs(gd[0] - gde) < 1e-9 * abs(gde) and abs(gd[1] - gdt) < 1e-9 * abs(gdt)

    # central difference in d_theta through the GPU forward
    def loss(dt):
        with torch.no_grad():
            o = ImexRollout.apply(to_dev(np.stack([eta0, theta0])),
                                  torch.tensor([1.0, dt], dtype=torch.float64), G, tau, nsteps, mf.KIN_DIB,
                                  _kin(p), 1e-13, 50, 0, 4)
            return 0.5 * float(((o - target) ** 2).sum())
    h = 1e-4 * p["d_theta"]
    fd = (loss(p["d_theta"] + h) - loss(p["d_theta"] - h)) / (2 * h)
    assert abs(fd - gd[1]) < 1e-5 * abs(fd)


def test_heat_rollout_adjoint():
    import torch
    from paper_2109_01173_amd.autograd import ImexRollout
    k, m, tau, dval, nsteps = 2, 8, 1e-2, 0.1, 6
    G = gpu_xnormal(k, m, "neumann", 0.0, imex=True)
    P = oracle_xnormal(k, m, "neumann", 0.0)
    rng = np.random.default_rng(6)
    U0 = rng.random((P.q, P.q))
    Ut = rng.random((P.q, P.q))
    s0 = to_dev(U0[None]).requires_grad_(True)
    d = torch.tensor([dval], dtype=torch.float64, device="cuda", requires_grad=True)
    out = ImexRollout.apply(s0, d, G, tau, nsteps, 0, None, 1e-13, 100, 0, 50)
    J = 0.5 * ((out - to_dev(Ut[None])) ** 2).sum()
    J.backward()

    def solve(c, R, U0_):
        return direct_solve(P.kron(c=c, imex=True), R)
    st = adjoint.heat_rollout(P, U0, tau, dval, nsteps, solve)
    g0, gd = adjoint.heat_gradients(P, st, tau, dval, st[-1] - Ut, solve)
    assert rel(to_host(s0.grad)[0], g0) < 1e-9
    assert abs(float(d.grad[0]) - gd) < 1e-9 * abs(gd)


def test_dot_accumulate_and_full_output_operator():
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(3, 7, "dirichlet", 1.0)
    P = oracle_xnormal(3, 7, "dirichlet", 1.0)
    rng = np.random.default_rng(9)
    L = rng.standard_normal((3, G.q, G.q))
    out = to_host(G.rhs_adjoint_op.apply(to_dev(L)))
    assert out.shape == (3, G.n, G.n)
    for b in range(3):
        ref = P.M3_rows.T @ L[b] @ P.M_rows
        assert rel(out[b], ref) < 1e-14
    X, Y = rng.standard_normal((2, 4, 17, 5))
    acc = to_dev(np.array([1.0, 2.0, 3.0, 4.0]))
    mf.dot_accumulate(to_dev(X), to_dev(Y), acc, alpha=-2.0, beta=0.5)
    ref = 0.5 * np.array([1.0, 2.0, 3.0, 4.0]) - 2.0 * np.einsum("bij,bij->b", X, Y)
    assert np.allclose(to_host(acc), ref, rtol=1e-14, atol=1e-13)
    _ = torch

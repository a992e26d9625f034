"""GPU tests of the host-synchronisation-free paths: MO-PCG queued with a
fixed iteration budget (mofem_pcg_solve_async) on several streams, and the
IMEX step captured as a HIP graph and replayed (mofem_imex_graph_*).

The masked iterations after convergence change nothing, so both must
reproduce the synchronous path's states and iteration counts (the kernels
and their order are the same).  Graph replays are checked one by one, with
unrelated eager work and synchronisations between them.  Every result is
also compared with the oracle: IMEX states with its steps (MO-PCG to 1e-13),
solves with its sparse direct solve of the Kronecker system."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, oracle_xnormal, rel, to_dev, to_host
from oracle import imex
from oracle.problems import RectProblem
from oracle.solvers import SpectralPrec, direct_solve, mo_pcg
from workloads import dib_initial, dib_params, heat_initial

pytestmark = pytest.mark.gpu


def oracle_solver(P, preset):
    def solve(c, R, U0):
        S = SpectralPrec(*P.imex_prec_pairs(preset, c))
        U, _ = mo_pcg(lambda X: P.apply_imex(X, c), S.apply, R, U0=U0, tol=1e-13, maxit=300)
        return U
    return solve


def _kin(p):
    return [p["rho"], p["A1"], p["A2"], p["B"], p["C"], p["D"], p["alpha"], p["gamma"], p["k2"], p["k3"]]


def test_imex_graph_replays_match_eager_dib():
    import torch
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.problems import Rect
    p = dib_params()
    G = Rect(1, 24, "neumann", length=20.0, lumped=True, imex=True)
    eta, theta = dib_initial(G.q, seed=7, amp=1e-2)
    s_eager = to_dev(np.stack([eta, theta]))
    s_graph = s_eager.clone()
    mk = lambda: mf.Imex(G.op, G.prec, G.mass, 1e-2, [1.0, p["d_theta"]], kinetics=mf.KIN_DIB, kin=_kin(p),
                         tol=1e-12, maxit=20)
    eager, graphed = mk(), mk()
    g = mf.ImexGraph(graphed, s_graph, 1, iters_per_step=4)
    noise = to_dev(np.random.default_rng(0).standard_normal((2, G.q, G.q)))
    P = RectProblem(1, 24, "neumann", lx=20.0, ly=20.0, lumped=True)
    solve = oracle_solver(P, "rect")
    eta_o, theta_o = eta.copy(), theta.copy()
    for step in range(5):
        its = eager.step(s_eager, 1)
        g.launch(1)
        _ = G.op.apply(noise)          # unrelated eager work between replays
        torch.cuda.synchronize()
        assert rel(to_host(s_graph), to_host(s_eager)) <= 1e-14, step
        max_its, status, relres = g.result()
        assert np.all(status == 0) and np.all(max_its == its) and np.all(relres < 1e-12)
        eta_o, theta_o = imex.rds_step(P, eta_o, theta_o, 1e-2, p, solve)
        out = to_host(s_graph)
        assert rel(out[0], eta_o) < 1e-10 and rel(out[1], theta_o) < 1e-12, step


def test_imex_graph_heat_and_budget_too_small():
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 16, "neumann", 0.0, imex=True)
    U0 = heat_initial(G.q, seed=42)
    s_eager, s_graph = to_dev(U0[None]), to_dev(U0[None])
    eager = mf.Imex(G.op, G.prec, G.mass, 1e-3, [0.1], tol=1e-12, maxit=60)
    g = mf.ImexGraph(mf.Imex(G.op, G.prec, G.mass, 1e-3, [0.1], tol=1e-12, maxit=60), s_graph, 1, iters_per_step=40)
    its = []
    for _ in range(3):
        its.append(int(eager.step(s_eager, 1)[0]))
    g.launch(3)
    torch.cuda.synchronize()
    assert rel(to_host(s_graph), to_host(s_eager)) <= 1e-14
    P = oracle_xnormal(2, 16, "neumann", 0.0)
    U = U0.copy()
    for _ in range(3):
        U = imex.imex_step(P, U, 1e-3, 0.1, oracle_solver(P, "sylv-imex"))
    assert rel(to_host(s_graph)[0], U) < 1e-10
    max_its, status, _ = g.result()
    assert status[0] == 0 and max_its[0] == max(its)
    # a budget below the iteration count is reported as MAXIT for that step
    g2 = mf.ImexGraph(mf.Imex(G.op, G.prec, G.mass, 1e-3, [0.1], tol=1e-12, maxit=60), to_dev(U0[None]), 1,
                      iters_per_step=2)
    g2.launch(1)
    with pytest.raises(mf.MofemError):
        g2.result()
    _, status, _ = g2.result(raise_on_error=False)  # the accumulation restarted: nothing since
    assert status[0] == 0


def test_imex_graph_heat_forward_bf16_rounding_s():
    """Heat steps replayed from a graph with the forward-BF16 transforms that
    round S (flexible PCG, as in the bench's second heat leg): the replay
    reproduces the eager steps, the masked iterations after convergence change
    nothing, and both follow the oracle's steps to the solve tolerance."""
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 16, "neumann", 0.0, imex=True, precision=mf.PREC_BF16_FWD_VS)
    U0 = heat_initial(G.q, seed=42)
    s_eager, s_graph = to_dev(U0[None]), to_dev(U0[None])
    mk = lambda: mf.Imex(G.op, G.prec, G.mass, 1e-3, [0.1], tol=1e-11, maxit=60, flags=mf.PCG_FLEXIBLE)
    eager = mk()
    g = mf.ImexGraph(mk(), s_graph, 1, iters_per_step=40)
    its = [int(eager.step(s_eager, 1)[0]) for _ in range(3)]
    g.launch(3)
    torch.cuda.synchronize()
    assert rel(to_host(s_graph), to_host(s_eager)) <= 1e-14
    max_its, status, _ = g.result()
    assert status[0] == 0 and max_its[0] == max(its)
    P = oracle_xnormal(2, 16, "neumann", 0.0)
    U = U0.copy()
    for _ in range(3):
        U = imex.imex_step(P, U, 1e-3, 0.1, oracle_solver(P, "sylv-imex"))
    assert rel(to_host(s_graph)[0], U) < 1e-9


def test_pcg_async_uneven_shapes_on_two_streams():
    import torch
    from paper_2109_01173_amd import mofem as mf
    specs = [(2, 20, "dirichlet"), (3, 11, "neumann")]
    cases = [gpu_xnormal(k, m, bc, 1.0) for k, m, bc in specs]
    oracles = [oracle_xnormal(k, m, bc, 1.0) for k, m, bc in specs]
    rng = np.random.default_rng(12)
    runs = []
    for G in cases:
        B = 3
        R = to_dev(rng.standard_normal((B, G.q, G.q)))
        U_sync = torch.empty_like(R)
        its_sync, rr_sync, _ = mf.pcg_solve(G.op, G.prec, R, U_sync, tol=1e-11, maxit=80, flags=mf.PCG_ZERO_GUESS)
        runs.append((G, R, U_sync, its_sync, rr_sync))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for (G, R, _, its_sync, _), st in zip(runs, streams):
        B = R.shape[0]
        U = torch.empty_like(R)
        ws = mf.pcg_workspace(G.op, G.prec, B)
        iters = torch.empty(B, dtype=torch.int32, device="cuda")
        status = torch.empty(B, dtype=torch.int32, device="cuda")
        relres = torch.empty(B, dtype=torch.float64, device="cuda")
        st.wait_stream(torch.cuda.current_stream())
        mf.pcg_solve_async(G.op, G.prec, R, U, ws, iters, status, relres, tol=1e-11, maxit=int(its_sync.max()) + 3,
                           flags=mf.PCG_ZERO_GUESS, stream=st)
        outs.append((U, iters, status, relres, ws))
    torch.cuda.synchronize()
    for (G, R, U_sync, its_sync, rr_sync), (U, iters, status, relres, _), P in zip(runs, outs, oracles):
        assert np.all(to_host(status) == 0)
        assert np.array_equal(to_host(iters), its_sync)
        assert rel(to_host(U), to_host(U_sync)) <= 1e-14
        assert np.allclose(to_host(relres), rr_sync, rtol=1e-12, atol=0)
        Rh, Uh, K = to_host(R), to_host(U), P.kron()
        for b in range(Rh.shape[0]):
            # backward under the oracle's operator, forward against its direct solve
            assert rel(P.apply(Uh[b]), Rh[b]) < 2e-11, b
            assert rel(Uh[b], direct_solve(K, Rh[b])) < 1e-8, b


def test_pcg_solve_many_uneven_groups():
    """Uneven instances (orders 1-4 and lumped P1, several node counts, both
    boundary conditions) solved together on three streams equal the
    one-at-a-time solves and the oracle's direct solves."""
    import torch
    from paper_2109_01173_amd import mofem as mf
    specs = [(1, 64, "dirichlet", False, 3), (2, 64, "dirichlet", False, 2), (3, 21, "neumann", False, 1),
             (4, 16, "dirichlet", False, 2), (2, 16, "neumann", False, 4), (1, 128, "dirichlet", True, 1)]
    rng = np.random.default_rng(33)
    groups, ref = [], []
    for k, m, bc, lumped, B in specs:
        G = gpu_xnormal(k, m, bc, 1.0, lumped=lumped)
        R = to_dev(rng.standard_normal((B, G.q, G.q)))
        G._oracle = oracle_xnormal(k, m, bc, 1.0, lumped=lumped)
        U1 = torch.empty_like(R)
        its, rr, _ = mf.pcg_solve(G.op, G.prec, R, U1, tol=1e-11, maxit=100, flags=mf.PCG_ZERO_GUESS)
        ref.append((U1, its, rr))
        groups.append(dict(op=G.op, prec=G.prec, rhs=R, U=torch.empty_like(R), tol=1e-11, maxit=100,
                           flags=mf.PCG_ZERO_GUESS, _keep=G))
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs, status = mf.pcg_solve_many(groups, [streams[i % 3] for i in range(len(groups))])
    torch.cuda.synchronize()
    assert status == [0] * len(groups)
    for g, (its, rr), (U1, its1, rr1) in zip(groups, outs, ref):
        assert np.array_equal(its, its1)
        assert np.allclose(rr, rr1, rtol=1e-12, atol=0)
        assert rel(to_host(g["U"]), to_host(U1)) <= 1e-14
        # each group against the oracle's sparse direct solve
        P = g["_keep"]._oracle
        K, Rh, Uh = P.kron(), to_host(g["rhs"]), to_host(g["U"])
        for b in range(Rh.shape[0]):
            assert rel(P.apply(Uh[b]), Rh[b]) < 2e-11, b
            assert rel(Uh[b], direct_solve(K, Rh[b])) < 1e-8, b

"""GPU parity of the grouped solve of uneven instances
(mofem_pcg_solve_grouped): instances of P1..P4 elements that share a shape
(q = 59) form one class solved with one launch per stage (the operator: one
launch per element order), a second shape forms its own class on a second
stream.  Every group's solution is checked against the oracle's sparse
direct solve of its own operator (eq. (73)), and its iteration counts against
the same group solved alone."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, oracle_xnormal, rel, to_dev, to_host
from oracle.solvers import direct_solve

pytestmark = pytest.mark.gpu

SHAPES = [(1, 60, 2), (2, 30, 1), (3, 20, 3), (4, 15, 2), (2, 40, 2)]   # (k, m, batch): q = 59 x4, then q = 79


@pytest.mark.parametrize("precision,flags,tol,bar", [("F64", 0, 1e-11, 1e-9), ("BF16_FWD", 1, 1e-9, 1e-7),
                                                ("BF16_FWD_VS", 1, 1e-9, 1e-7)])
def test_grouped_solve_vs_oracle(precision, flags, tol, bar):
    import torch
    from paper_2109_01173_amd import mofem as mf
    rng = np.random.default_rng(31)
    groups, oracle, alone = [], [], []
    fl = (mf.PCG_FLEXIBLE if flags else 0) | mf.PCG_ZERO_GUESS
    for k, m, B in SHAPES:
        G = gpu_xnormal(k, m, "dirichlet", 1.0, precision=getattr(mf, "PREC_" + precision))
        R = rng.standard_normal((B, G.q, G.q))
        groups.append(dict(op=G.op, prec=G.prec, rhs=to_dev(R), U=torch.full((B, G.q, G.q), np.nan,
                                                                             dtype=torch.float64, device="cuda"),
                           tol=tol, maxit=300, flags=fl, _keep=G))
        oracle.append((oracle_xnormal(k, m, "dirichlet", 1.0), R))
        U1 = torch.zeros_like(groups[-1]["U"])
        its1, _, _ = mf.pcg_solve(G.op, G.prec, groups[-1]["rhs"], U1, tol=tol, maxit=300, flags=fl)
        alone.append(its1)
    streams = [torch.cuda.Stream() for _ in groups]
    outs, status = mf.pcg_solve_many(groups, streams, grouped=True)
    torch.cuda.synchronize()
    assert status == [mf.OK] * len(groups)
    for (its, relres), g, (P, R), its1 in zip(outs, groups, oracle, alone):
        assert np.all(relres <= tol)
        assert np.all(np.abs(its - its1) <= 1), (its, its1)
        K = P.kron()
        U = to_host(g["U"])
        for b in range(R.shape[0]):
            assert rel(U[b], direct_solve(K, R[b])) < bar


def test_grouped_rejects_banded_and_keeps_empty_groups():
    import torch
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(2, 20, "dirichlet", 1.0)
    R = to_dev(np.random.default_rng(2).standard_normal((2, G.q, G.q)))
    empty = dict(op=G.op, prec=G.prec, rhs=R[:0], U=torch.zeros_like(R[:0]), tol=1e-10, maxit=50)
    full = dict(op=G.op, prec=G.prec, rhs=R, U=torch.zeros_like(R), tol=1e-10, maxit=50, flags=mf.PCG_ZERO_GUESS)
    outs, status = mf.pcg_solve_many([empty, full], [torch.cuda.Stream(), torch.cuda.Stream()], grouped=True)
    assert status == [mf.OK, mf.OK] and np.all(outs[1][1] <= 1e-10)
    bp = G.product_prec()
    with pytest.raises(mf.MofemError) as e:
        mf.pcg_solve_many([dict(op=G.op, prec=bp, rhs=R, U=torch.zeros_like(R))], [torch.cuda.Stream()],
                          grouped=True)
    assert e.value.code == mf.E_UNSUPPORTED

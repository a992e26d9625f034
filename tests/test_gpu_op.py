"""GPU parity of the banded multiterm operator (mofem_op_apply) against the
oracle, element by element, with a rounding bound derived from the
arithmetic: |Y_gpu - Y_ref| <= 64 * (2k+1) * eps * (|L| |X| |R|), the
absolute-value operator of the same terms.

Sizes span several column strips and row blocks of the kernel with ragged
tails (q ~ 150..300), every order k = 1..4, lumped P1, both boundary
conditions, the five-term elliptic, six-term IMEX (per-item coefficient)
and the one-term full-node load operator; plus tiny and empty inputs."""
import numpy as np
import pytest

from gpu_cases import gpu_xnormal, oracle_abs_apply, oracle_xnormal, rel, to_dev, to_host
from oracle.problems import RectProblem

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps

CASES = [  # k, m, bc, lumped
    (1, 301, "dirichlet", False),
    (2, 150, "dirichlet", False),
    (2, 73, "neumann", False),
    (3, 61, "neumann", False),
    (4, 40, "dirichlet", False),
    (1, 203, "neumann", True),
]


@pytest.mark.parametrize("k,m,bc,lumped", CASES)
def test_elliptic_operator(k, m, bc, lumped):
    gamma = 0.8
    G = gpu_xnormal(k, m, bc, gamma, lumped)
    P = oracle_xnormal(k, m, bc, gamma, lumped)
    rng = np.random.default_rng(10 + k)
    X = rng.standard_normal((3, P.q, P.q))
    Y, dots = G.op.apply(to_dev(X), dot=True)
    Y, dots = to_host(Y), to_host(dots)
    for b in range(3):
        ref = P.apply(X[b])
        bound = 64 * (2 * G.kb + 1) * EPS * oracle_abs_apply(P, X[b])
        assert np.all(np.abs(Y[b] - ref) <= bound), np.abs(Y[b] - ref).max()
        assert abs(dots[b] - np.sum(X[b] * ref)) <= 1e-12 * np.sum(np.abs(X[b] * ref))


@pytest.mark.parametrize("k,m,bc,lumped", CASES[:4] + CASES[5:])
def test_imex_operator_per_item_coefficient(k, m, bc, lumped):
    G = gpu_xnormal(k, m, bc, 0.0, lumped, imex=True)
    P = oracle_xnormal(k, m, bc, 0.0, lumped)
    rng = np.random.default_rng(20 + k)
    X = rng.standard_normal((2, P.q, P.q))
    cs = np.array([1e-4, 3e-2])
    Y = to_host(G.op.apply(to_dev(X), item_scale=to_dev(cs)))
    for b in range(2):
        ref = P.apply_imex(X[b], cs[b])
        bound = 64 * (2 * G.kb + 1) * EPS * oracle_abs_apply(P, X[b], c=cs[b])
        assert np.all(np.abs(Y[b] - ref) <= bound)


@pytest.mark.parametrize("k,m,bc", [(2, 150, "dirichlet"), (1, 97, "neumann"), (4, 33, "dirichlet")])
def test_full_node_load(k, m, bc):
    G = gpu_xnormal(k, m, bc, 1.0)
    P = oracle_xnormal(k, m, bc, 1.0)
    rng = np.random.default_rng(30)
    F = rng.standard_normal((2, P.n, P.n))
    R = to_host(G.rhs_op.apply(to_dev(F)))
    for b in range(2):
        ref = P.rhs(F[b])
        scale = np.abs(P.M3_rows) @ np.abs(F[b]) @ np.abs(P.M_rows).T
        assert np.all(np.abs(R[b] - ref) <= 64 * EPS * (2 * k + 1) * scale)


@pytest.mark.parametrize("lumped,k,m", [(True, 1, 130), (False, 2, 70)])
def test_rectangle_operators(lumped, k, m):
    from paper_2109_01173_amd.problems import Rect
    for imex in (False, True):
        G = Rect(k, m, "neumann", length=20.0, gamma=0.5, lumped=lumped, imex=imex)
        P = RectProblem(k, m, "neumann", lx=20.0, ly=20.0, lumped=lumped, gamma=0.5)
        X = np.random.default_rng(40).standard_normal((2, P.q, P.q))
        c = np.array([0.01, 0.2])
        Y = to_host(G.op.apply(to_dev(X), item_scale=to_dev(c) if imex else None))
        for b in range(2):
            ref = P.apply_imex(X[b], c[b]) if imex else P.apply(X[b])
            assert rel(Y[b], ref) < 1e-14


def test_tiny_and_empty_inputs():
    import torch
    G = gpu_xnormal(2, 2, "dirichlet", 1.0)       # q = 3: smaller than one tile
    P = oracle_xnormal(2, 2, "dirichlet", 1.0)
    X = np.random.default_rng(50).standard_normal((1, 3, 3))
    Y = to_host(G.op.apply(to_dev(X)))
    assert rel(Y[0], P.apply(X[0])) < 1e-14
    empty = torch.empty((0, 3, 3), dtype=torch.float64, device="cuda")
    out = G.op.apply(empty)
    assert out.shape == (0, 3, 3)


def test_rejects_bad_stride_and_dot_on_load_operator():
    from paper_2109_01173_amd import mofem as mf
    G = gpu_xnormal(1, 9, "dirichlet", 1.0)
    X = to_dev(np.zeros((1, G.n, G.n)))
    with pytest.raises(mf.MofemError):
        G.rhs_op.apply(X, dot=True)
    Xs = to_dev(np.zeros((1, G.q, G.q)))
    with pytest.raises(ValueError):
        G.rhs_op.apply(Xs)


def _dense(band, n):
    """Dense n x n matrix of a DIA band (band[d * n + i] = A[i][i + d - kb])."""
    kb = (band.shape[0] - 1) // 2
    A = np.zeros((n, n))
    for d in range(2 * kb + 1):
        for i in range(n):
            j = i + d - kb
            if 0 <= j < n:
                A[i, j] = band[d, i]
    return A


@pytest.mark.parametrize("n_terms,merges", [(4, 0), (7, 0), (8, 0), (7, 1), (8, 2)])
def test_term_counts_and_merging(n_terms, merges):
    """Operators of 4, 7 and 8 terms (random symmetric-free bands, kb = 2,
    transposes and per-item scaling mixed in) against their plain dense
    definition sum_t c_t op(L_t) X op(R_t); `merges` terms repeat an earlier
    term's right (or left) factor with the same scaling, so the library merges
    them and runs fewer distinct terms."""
    from paper_2109_01173_amd import mofem as mf
    kb, n = 2, 161
    rng = np.random.default_rng(60 + n_terms + 10 * merges)
    terms = []
    for t in range(n_terms):
        L, R = rng.standard_normal((2, 2 * kb + 1, n))
        if t >= n_terms - merges:   # share a factor with term t - 3
            src = terms[t - 3]
            coef = float(rng.uniform(-2, 2))
            if t % 2:
                R = src["right"]
            else:
                L, coef = src["left"], src["coef"]   # a shared left factor merges with an equal coefficient
            terms.append(dict(left=L, right=R, coef=coef, scaled=src["scaled"],
                              left_T=src["left_T"] if t % 2 == 0 else False,
                              right_T=src["right_T"] if t % 2 else False))
        else:
            terms.append(dict(left=L, right=R, coef=float(rng.uniform(-2, 2)), scaled=bool(t % 3 == 1),
                              left_T=bool(t % 2), right_T=bool(t % 4 == 3)))
    op = mf.Operator(terms, n_s=n, n_t=n, kb=kb, trim_s=1, trim_t=1)
    q = n - 2
    X = rng.standard_normal((2, q, q))
    cs = np.array([0.3, -1.7])
    Y, dots = op.apply(to_dev(X), item_scale=to_dev(cs), dot=True)
    Y, dots = to_host(Y), to_host(dots)
    I = slice(1, n - 1)
    for b in range(2):
        ref = np.zeros((q, q))
        scale = np.zeros((q, q))
        for t in terms:
            Ld, Rd = _dense(t["left"], n), _dense(t["right"], n)
            Ld = Ld.T if t["left_T"] else Ld
            Rd = Rd.T if t["right_T"] else Rd
            c = t["coef"] * (cs[b] if t["scaled"] else 1.0)
            ref += c * Ld[I, I] @ X[b] @ Rd[I, I]
            scale += abs(c) * np.abs(Ld[I, I]) @ np.abs(X[b]) @ np.abs(Rd[I, I])
        assert np.all(np.abs(Y[b] - ref) <= 64 * (2 * kb + 1) * EPS * n_terms * scale), b
        assert abs(dots[b] - np.sum(X[b] * ref)) <= 1e-12 * np.sum(np.abs(X[b]) * scale)


def test_more_than_eight_terms_rejected():
    from paper_2109_01173_amd import mofem as mf
    band = np.ones((3, 10))
    with pytest.raises(ValueError):
        mf.Operator([dict(left=band, right=band)] * 9, n_s=10, n_t=10, kb=1)

"""Pins of the oracle's multiterm operators (Sec. 3.2-3.3, Sec. 5, Sec. 6).

* Kronecker identity: the matrix form of eq. (70) / eq. (73) (and the
  lumped eq. (75)) equals the 2D stiffness + gamma mass matrix assembled
  element by element on the mapped domain (``oracle.fem2d``), which never
  uses the decomposition of eq. (35).
* Symmetry, definiteness, the constant kernel for Neumann, and the area of
  the domain as the total mass.
"""
import math

import numpy as np
import pytest

from oracle import fem2d
from oracle.problems import RectProblem, XNormalProblem, vec_r
from workloads import L_profile, dL_profile

CASES = [(1, 3, False), (2, 2, False), (3, 2, False), (4, 2, False), (1, 4, True)]


@pytest.mark.parametrize("k,m,lumped", CASES)
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_kronecker_equals_bruteforce_2d(k, m, lumped, bc):
    gamma = 0.7
    P = XNormalProblem(k, m, bc, L_profile, dL_profile, gamma=gamma, lumped=lumped)
    K = P.kron().toarray()
    A2, M2 = fem2d.assemble_2d(k, m, L_profile, dL_profile, gamma=gamma, lumped=lumped)
    K2 = fem2d.trim(A2, P.n, bc)
    assert np.abs(K - K2).max() <= 1e-13 * np.abs(K2).max()
    # the apply() form equals the Kronecker form
    rng = np.random.default_rng(0)
    U = rng.standard_normal((P.q, P.q))
    assert np.allclose(vec_r(P.apply(U)), K @ vec_r(U), atol=1e-13 * np.abs(K).max() * P.q)
    # total mass = area of the physical domain = int_0^1 L(s) ds
    assert math.isclose(M2.sum(), 1.0 + 0.6 / math.pi, rel_tol=1e-12 if not lumped else 1e-2)


def cap_L(s):
    """L = 2 S for the cap-shaped symmetric domain |X| <= S(Y) = 1 - Y^2 / 2."""
    return 2.0 - s ** 2


def cap_dL(s):
    return -2.0 * s


@pytest.mark.parametrize("k,m,m_t,lumped,bc", [(1, 4, 6, False, "dirichlet"), (2, 3, 2, False, "neumann"),
                                               (3, 2, 3, False, "dirichlet"), (4, 2, 1, False, "neumann"),
                                               (1, 5, 3, True, "neumann")])
def test_cap_domain_and_uneven_mesh_equal_bruteforce_2d(k, m, m_t, lumped, bc):
    """Symmetric x-normal domain (remark after eq. (19): t in [-1/2, 1/2],
    L = 2 S) with the cap profile, different element counts along s and t."""
    gamma = 0.7
    P = XNormalProblem(k, m, bc, cap_L, cap_dL, gamma=gamma, lumped=lumped, m_t=m_t, t_interval=(-0.5, 0.5))
    assert (P.q, P.q_t) != (P.q_t, P.q) or m == m_t
    K = P.kron().toarray()
    A2, M2 = fem2d.assemble_2d(k, m, cap_L, cap_dL, gamma=gamma, lumped=lumped, m_t=m_t, t_interval=(-0.5, 0.5))
    K2 = fem2d.trim(A2, P.n, bc, P.n_t)
    assert K.shape == K2.shape == (P.q * P.q_t, P.q * P.q_t)
    assert np.abs(K - K2).max() <= 1e-13 * np.abs(K2).max()
    rng = np.random.default_rng(1)
    U = rng.standard_normal((P.q, P.q_t))
    assert np.allclose(vec_r(P.apply(U)), K @ vec_r(U), atol=1e-13 * np.abs(K).max() * P.q)
    # area of the cap: int_0^1 2 (1 - y^2 / 2) dy = 5 / 3
    assert math.isclose(M2.sum(), 5.0 / 3.0, rel_tol=1e-12 if not lumped else 5e-2)


@pytest.mark.parametrize("k,m,lumped", CASES)
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_operator_symmetric_positive(k, m, lumped, bc):
    gamma = 0.0 if bc == "dirichlet" else 0.5
    P = XNormalProblem(k, m + 1, bc, L_profile, dL_profile, gamma=gamma, lumped=lumped)
    rng = np.random.default_rng(1)
    X, Y = rng.standard_normal((2, P.q, P.q))
    a, b = np.sum(P.apply(X) * Y), np.sum(X * P.apply(Y))
    assert math.isclose(a, b, rel_tol=1e-12)
    K = P.kron().toarray()
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(K).min() > 0.0
    Ki = P.kron(c=0.3, imex=True).toarray()
    assert np.linalg.eigvalsh(Ki).min() > 0.0


@pytest.mark.parametrize("k,lumped", [(1, False), (2, False), (4, False), (1, True)])
def test_neumann_constant_kernel_and_imex(k, lumped):
    P = XNormalProblem(k, 4, "neumann", L_profile, dL_profile, gamma=0.0, lumped=lumped)
    one = np.ones((P.q, P.q))
    assert np.abs(P.apply(one)).max() < 1e-13
    # IMEX operator of eq. (91) on constants is the mass form
    assert np.allclose(P.apply_imex(one, 0.37), P.mass_apply(one), atol=1e-14)


def test_rect_problem_matches_xnormal_with_flat_profile():
    """On L = 1 the x-normal operator reduces to the square form eq. (28)."""
    k, m = 2, 3
    P = XNormalProblem(k, m, "dirichlet", lambda s: 1.0 + 0 * s, lambda s: 0 * s, gamma=0.3)
    R = RectProblem(k, m, "dirichlet", gamma=0.3)
    rng = np.random.default_rng(2)
    U = rng.standard_normal((P.q, P.q))
    assert np.allclose(P.apply(U), R.apply(U), atol=1e-13)


def test_dirichlet_rhs_uses_full_node_source():
    """eq. (74) with the full-node F equals the 2D load vector of the
    interpolant f_h against the interior test functions."""
    k, m = 2, 2
    P = XNormalProblem(k, m, "dirichlet", L_profile, dL_profile)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((P.n, P.n))
    _, M2 = fem2d.assemble_2d(k, m, L_profile, dL_profile)
    interior = np.array([i * P.n + j for i in range(1, P.n - 1) for j in range(1, P.n - 1)])
    load = (M2 @ vec_r(F))[interior]
    assert np.allclose(vec_r(P.rhs(F)), load, atol=1e-14)

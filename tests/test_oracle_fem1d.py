"""Pins of the oracle's 1D finite element layer (Sec. 3, Sec. 4.1).

Each check is fixed by mathematics or by the paper, not by the oracle's own
formulas: Lagrange interpolation properties, quadrature exactness,
Newton-Cotes weights as row sums of the mass matrix, closed-form integrals
of the weights, and the P1 closed forms of Sec. 4.1 (eqs. (60), (63)-(65)).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.integrate as si

from oracle import fem1d
from workloads import L_profile, dL_profile

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_delta_and_partition(k):
    xi = np.arange(k + 1) / k
    phi, dphi = fem1d.lagrange_ref(k, xi)
    assert np.allclose(phi, np.eye(k + 1), atol=1e-14)
    x = np.linspace(0, 1, 37)
    phi, dphi = fem1d.lagrange_ref(k, x)
    assert np.allclose(phi.sum(0), 1.0, atol=1e-13)
    assert np.allclose(dphi.sum(0), 0.0, atol=1e-11)
    # derivative against central differences
    e = 1e-6
    pp, _ = fem1d.lagrange_ref(k, x + e)
    pm, _ = fem1d.lagrange_ref(k, x - e)
    assert np.allclose(dphi, (pp - pm) / (2 * e), atol=1e-7)


def test_gauss_exactness():
    xq, wq = fem1d.gauss_legendre(12)
    for p in range(24):
        assert math.isclose(np.sum(wq * xq ** p), 1.0 / (p + 1), rel_tol=1e-14)


# Newton-Cotes weights = integrals of the equispaced Lagrange basis on one element
NEWTON_COTES = {1: [1 / 2, 1 / 2], 2: [1 / 6, 4 / 6, 1 / 6], 3: [1 / 8, 3 / 8, 3 / 8, 1 / 8],
                4: [7 / 90, 32 / 90, 12 / 90, 32 / 90, 7 / 90]}


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_mass_row_sums_are_newton_cotes(k):
    m = 5
    M = fem1d.assemble(k, m, 0, 0)
    h = 1.0 / m
    w = np.zeros(k * m + 1)
    for e in range(m):
        w[e * k:e * k + k + 1] += h * np.array(NEWTON_COTES[k])
    assert np.allclose(M.sum(1), w, atol=1e-15)
    assert math.isclose(M.sum(), 1.0, rel_tol=1e-14)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_weighted_matrix_identities(k):
    m = 6
    Mat = fem1d.xnormal_matrices(k, m, m, L_profile, dL_profile)
    n = k * m + 1
    one = np.ones(n)
    t = fem1d.node_coords(k, m)
    # stiffness-type matrices annihilate constants (Neumann kernel)
    for key in ("A", "B1", "B2"):
        assert np.abs(Mat[key] @ one).max() < 1e-12
    # d/dx of sum psi_i = 0  ->  column sums of convection matrices vanish
    assert np.abs(one @ Mat["C1"]).max() < 1e-13
    assert np.abs(one @ Mat["C2"]).max() < 1e-12
    # P_k reproduces linear functions exactly: t = sum t_i psi_i
    assert math.isclose(t @ Mat["A"] @ t, 1.0, rel_tol=1e-13)          # int 1
    assert math.isclose(t @ Mat["B2"] @ t, 1.0 / 3.0, rel_tol=1e-13)   # int t^2
    assert math.isclose(t @ Mat["C1"] @ one, 0.5, rel_tol=1e-13)       # int t
    # weighted masses: sum_ij = int of the weight (closed form or scipy.quad)
    assert math.isclose(Mat["M3"].sum(), 1.0 + 0.6 / math.pi, rel_tol=1e-13)
    ref_inv = si.quad(lambda s: 1.0 / L_profile(s), 0, 1, epsabs=1e-15)[0]
    assert math.isclose(Mat["M1"].sum(), ref_inv, rel_tol=1e-12)
    ref_m2 = si.quad(lambda s: dL_profile(s) ** 2 / L_profile(s), 0, 1, epsabs=1e-15)[0]
    assert math.isclose(Mat["M2"].sum(), ref_m2, rel_tol=1e-12)
    # s^T C2 s = int s L'(s) ds = [s L]_0^1 - int L ;  s^T C2 1 = int L' = L(1) - L(0)
    s = t
    ref_c2 = L_profile(1.0) - (1.0 + 0.6 / math.pi)
    assert math.isclose(s @ Mat["C2"] @ s, ref_c2, rel_tol=1e-12)
    assert abs(s @ Mat["C2"] @ one - (L_profile(1.0) - L_profile(0.0))) < 1e-13
    # s^T B1 s = int L
    assert math.isclose(s @ Mat["B1"] @ s, 1.0 + 0.6 / math.pi, rel_tol=1e-13)
    # symmetry of the symmetric ones
    for key in ("A", "M", "B1", "B2", "M1", "M2", "M3"):
        assert np.allclose(Mat[key], Mat[key].T, atol=1e-15)


def test_lumped_matrices():
    m = 8
    h = 1.0 / m
    M0 = fem1d.assemble(1, m, 0, 0, lumped=True)
    d = np.full(m + 1, h)
    d[0] = d[-1] = h / 2
    assert np.allclose(M0, np.diag(d), atol=1e-16)
    # stiffness with constant weight is exact under lumping
    assert np.allclose(fem1d.assemble(1, m, 1, 1, lumped=True), fem1d.assemble(1, m, 1, 1), atol=1e-13)
    # convection: exact P1 C = 1/2 skew tridiagonal with -1/2, +1/2 at the ends
    C = fem1d.assemble(1, m, 1, 0, lumped=True)
    Cref = np.zeros((m + 1, m + 1))
    for j in range(m):
        Cref[j + 1, j] = 0.5
        Cref[j, j + 1] = -0.5
    Cref[0, 0], Cref[m, m] = -0.5, 0.5
    assert np.allclose(C, Cref, atol=1e-15)
    # weighted convection = C D_w  (Sec. 3.3: C D3 and C D2)
    x = fem1d.node_coords(1, m)
    Cw = fem1d.assemble(1, m, 1, 0, lambda s: s ** 2 + 1, lumped=True)
    assert np.allclose(Cw, Cref @ np.diag(x ** 2 + 1), atol=1e-15)
    # weighted lumped mass = M0 D_w
    Mw = fem1d.assemble(1, m, 0, 0, lambda s: L_profile(s), lumped=True)
    assert np.allclose(Mw, np.diag(d * L_profile(x)), atol=1e-15)
    # trapezoid stiffness: element-wise psi'psi' times the mean nodal weight
    A2 = fem1d.assemble(1, m, 1, 1, lambda t: t ** 2, lumped=True)
    A2ref = np.zeros((m + 1, m + 1))
    for e in range(m):
        wbar = 0.5 * (x[e] ** 2 + x[e + 1] ** 2)
        A2ref[np.ix_([e, e + 1], [e, e + 1])] += wbar / h * np.array([[1, -1], [-1, 1]])
    assert np.allclose(A2, A2ref, atol=1e-13)


@pytest.mark.parametrize("N", [8, 13, 32])
def test_sec41_p1_closed_forms(N):
    """Sec. 4.1: trimmed P1 Dirichlet matrices on [0, 1] (N intervals)."""
    g = GOLDEN["sec4_1_p1_dirichlet_mass_stiffness"]
    assert g["alpha"] == "-1/(6 N^2)" and g["beta"] == "1/N"
    A = fem1d.assemble(1, N, 1, 1)[1:-1, 1:-1]
    M = fem1d.assemble(1, N, 0, 0)[1:-1, 1:-1]
    alpha, beta = -1.0 / (6 * N ** 2), 1.0 / N            # eq. (60)
    assert np.allclose(M, alpha * A + beta * np.eye(N - 1), atol=1e-15)
    i = np.arange(1, N)
    lamA = 2.0 * N * (1.0 - np.cos(i * np.pi / N))      # eq. (63), corrected factor
    V = np.sin(np.outer(i, i) * np.pi / N)               # eq. (64)
    assert np.allclose(A @ V, V * lamA, atol=1e-11 * N)
    # the printed factor 2/N does not give the spectrum (reading recorded)
    assert not np.allclose(np.linalg.eigvalsh(A), np.sort(2.0 / N * (1 - np.cos(i * np.pi / N))))
    gamma = 0.7
    lam = ((12 * N ** 2 - gamma) * lamA + 6 * N * gamma) / (12 * N - 2 * lamA)   # eq. (65)
    Z1 = np.linalg.solve(M, A) + gamma / 2 * np.eye(N - 1)
    assert np.allclose(np.sort(np.linalg.eigvals(Z1).real), np.sort(lam), rtol=1e-11)

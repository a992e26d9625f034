"""L2 errors of MO-FEM solutions on the mapped x-normal domain.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper reports L2 errors (Sec. 5.2, Sec. 6.1) without fixing the
quadrature.  Reading: the true L2(Omega^L) error
  int_0^1 int_0^1 (u_h - u)^2 L(s) ds dt
by tensor Gauss-Legendre quadrature with k + 3 points per element and
direction; u_h(s, t) = sum_ij U_ij psi_i(s) psi_j(t) over all nodes.
"""
import numpy as np

from .fem1d import gauss_legendre, lagrange_ref


def basis_at_points(k, m, nq):
    """Matrix E (m*nq x n) of all global basis values at all quadrature
    points of [0, 1], plus the points and weights."""
    n = k * m + 1
    xq, wq = gauss_legendre(nq)
    phi, _ = lagrange_ref(k, xq)
    h = 1.0 / m
    E = np.zeros((m * nq, n))
    pts = np.zeros(m * nq)
    wts = np.zeros(m * nq)
    for e in range(m):
        rows = slice(e * nq, (e + 1) * nq)
        pts[rows] = h * (e + xq)
        wts[rows] = h * wq
        for a in range(k + 1):
            E[rows, e * k + a] = phi[a]
    return E, pts, wts


def l2_error(U_full, k, m, u_exact, L):
    """sqrt(int int (u_h - u)^2 L(s) ds dt) for a full-node nodal matrix."""
    nq = k + 3
    E, pts, wts = basis_at_points(k, m, nq)
    Uh = E @ U_full @ E.T
    S, T = np.meshgrid(pts, pts, indexing="ij")
    W = np.outer(wts * L(pts), wts)
    return float(np.sqrt(np.sum(W * (Uh - u_exact(S, T)) ** 2)))


def extend(U, n, bc):
    """Zero-extend interior unknowns to all nodes (Dirichlet)."""
    if bc == "neumann":
        return U
    F = np.zeros((n, n))
    F[1:-1, 1:-1] = U
    return F

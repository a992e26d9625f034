"""Brute-force 2D finite element assembly on the mapped x-normal domain.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Purpose: an independent check of the Kronecker decompositions of Sec. 3.2
(eq. (35)) and Sec. 3.3 (eq. (45)).  The 2D stiffness and mass matrices of
eq. (32) are assembled element by element on the reference square with the
tensor basis phi_(i,j)(s, t) = psi_i(s) psi_j(t), pulled back through the
map (s, t) -> (X, Y) = (s, t L(s)).  The chain rule is applied numerically
with the Jacobian of that map at every quadrature point; the matrix H-hat of
eq. (19) is never written down here, so a mistake in the one-dimensional
weights of ``oracle.fem1d`` or in the term order of ``oracle.problems``
shows up as a mismatch.

Lumped version: the whole 2D integrand is replaced by its element-wise
bilinear interpolant (Sec. 3.3, eq. (42)), i.e. integrated with the 2 x 2
vertex rule on each element.

Row-major unknown ordering: index(i, j) = i * n_t + j  (i = s node).
"""
import numpy as np

from .fem1d import gauss_legendre, lagrange_ref


def assemble_2d(k, m, L, dL, gamma=0.0, lumped=False, nq=12, m_t=None, t_interval=(0.0, 1.0)):
    """Dense (n_s n_t x n_s n_t) matrices  A_2D + gamma M_2D  and  M_2D (full
    nodes).  m elements along s, m_t (default m) along t; t runs over
    t_interval ([-1/2, 1/2] with L = 2 S for the symmetric domains of the
    remark after eq. (19))."""
    kk = 1 if lumped else k
    m_t = m if m_t is None else m_t
    n = kk * m + 1
    n_t = kk * m_t + 1
    h = 1.0 / m
    t0, t1 = t_interval
    ht = (t1 - t0) / m_t
    if lumped:
        xq, wq = np.array([0.0, 1.0]), np.array([0.5, 0.5])
    else:
        xq, wq = gauss_legendre(nq)
    phi, dphi = lagrange_ref(kk, xq)
    nl = kk + 1
    A2 = np.zeros((n * n_t, n * n_t))
    M2 = np.zeros((n * n_t, n * n_t))
    for es in range(m):
        for et in range(m_t):
            for qa in range(xq.size):
                s = h * (es + xq[qa])
                Ls, dLs = L(s), dL(s)
                for qb in range(xq.size):
                    t = t0 + ht * (et + xq[qb])
                    w = wq[qa] * wq[qb] * h * ht
                    # Jacobian of (s, t) -> (X, Y) = (s, t L(s))
                    J = np.array([[1.0, 0.0], [t * dLs, Ls]])
                    detJ = np.linalg.det(J)
                    Jinv_T = np.linalg.inv(J).T
                    # local basis values and reference gradients
                    vals = np.zeros(nl * nl)
                    grads = np.zeros((nl * nl, 2))
                    glob = np.zeros(nl * nl, dtype=int)
                    c = 0
                    for a in range(nl):
                        for b in range(nl):
                            vals[c] = phi[a, qa] * phi[b, qb]
                            grads[c, 0] = dphi[a, qa] / h * phi[b, qb]
                            grads[c, 1] = phi[a, qa] * dphi[b, qb] / ht
                            glob[c] = (es * kk + a) * n_t + (et * kk + b)
                            c += 1
                    pg = grads @ Jinv_T.T          # physical gradients
                    A2[np.ix_(glob, glob)] += w * abs(detJ) * (pg @ pg.T)
                    M2[np.ix_(glob, glob)] += w * abs(detJ) * np.outer(vals, vals)
    return A2 + gamma * M2, M2


def trim(Mat, n, bc, n_t=None):
    """Restrict a full-node 2D matrix to the unknowns of the boundary rule."""
    if bc == "neumann":
        return Mat
    n_t = n if n_t is None else n_t
    idx = np.array([i * n_t + j for i in range(1, n - 1) for j in range(1, n_t - 1)])
    return Mat[np.ix_(idx, idx)]

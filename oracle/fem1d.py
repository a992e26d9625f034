"""1D Lagrange finite elements and the weighted 1D matrices of MO-FEM.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What the paper fixes (Sec. 2.1, Sec. 3):
* uniform mesh of the unit interval, nodes x_m = m/N (Sec. 2.1);
* 1D stiffness and mass a_ij = int psi_i' psi_j', m_ij = int psi_i psi_j
  (Sec. 3.1, eq. (23));
* the seven weighted matrices of Sec. 3.2, eqs. (29)-(31):
  b1 = int psi_i' psi_j' L,  b2 = int psi_i' psi_j' x^2,
  c1 = int psi_i' psi_j x,   c2 = int psi_i' psi_j L',
  m1 = int psi_i psi_j / L,  m2 = int psi_i psi_j L'^2 / L,
  m3 = int psi_i psi_j L   (the row index carries the derivative);
* lumped P1 (Sec. 3.3): every integrand is replaced by its element-wise
  P1 interpolant I_h before integrating, eqs. (36)-(39), (42)-(44).

Readings where the paper is silent:
* P_k nodes are equispaced inside each element ("Lagrangian P_k");
* element integrals use 12-point Gauss-Legendre quadrature;
* lumping = integrating the I_h interpolant exactly, which on each element
  is the two-point trapezoid rule at the element's end points.  This gives
  the lumped M_0, A, A_1, A_2, C D_w of Sec. 3.3 from one definition.

Pins (tests/test_oracle_fem1d.py): Lagrange delta property, partition of
unity, quadrature exactness, mass/stiffness identities (row sums, constants
in the kernel, closed-form weighted integrals), the P1 closed forms of
Sec. 4.1 (eq. (60), corrected eq. (63)), and the 2D brute-force assembly of
``oracle.fem2d`` through the Kronecker identities eqs. (35) and (45).
"""
import numpy as np


def gauss_legendre(nq):
    """nq-point Gauss-Legendre rule mapped to [0, 1] (points, weights)."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (xg + 1.0), 0.5 * wg


def lagrange_ref(k, x):
    """Values and first derivatives of the k+1 Lagrange polynomials on [0, 1]
    with equispaced nodes xi_a = a/k, evaluated at the points ``x``.

    Returns (phi, dphi), each of shape (k+1, len(x)).  Plain product formula:
    phi_a(x) = prod_{b != a} (x - xi_b) / (xi_a - xi_b).
    """
    x = np.asarray(x, dtype=np.float64)
    xi = np.arange(k + 1, dtype=np.float64) / k
    phi = np.ones((k + 1, x.size))
    dphi = np.zeros((k + 1, x.size))
    for a in range(k + 1):
        others = [b for b in range(k + 1) if b != a]
        denom = np.prod([xi[a] - xi[b] for b in others])
        for b in others:
            phi[a] *= (x - xi[b])
        phi[a] /= denom
        # derivative: sum over the dropped factor
        for c in others:
            term = np.ones(x.size)
            for b in others:
                if b != c:
                    term *= (x - xi[b])
            dphi[a] += term
        dphi[a] /= denom
    return phi, dphi


def n_nodes(k, m):
    """Number of Lagrange nodes of P_k on m elements."""
    return k * m + 1


def node_coords(k, m, x0=0.0, x1=1.0):
    """Global node coordinates, element e owns nodes e*k .. e*k+k."""
    return x0 + (x1 - x0) * np.arange(k * m + 1, dtype=np.float64) / (k * m)


def assemble(k, m, di, dj, w=None, x0=0.0, x1=1.0, lumped=False, nq=12):
    """Dense n x n matrix  K_ij = int_{x0}^{x1} psi_i^(di) psi_j^(dj) w dx.

    k      : polynomial order (1..4); lumping requires k = 1.
    m      : number of uniform elements; n = k*m + 1.
    di, dj : derivative order (0 or 1) of the row / column basis function.
    w      : weight function of x (vectorised) or None for w = 1.
    lumped : integrate the element-wise interpolant of the integrand (Sec. 3.3).
    """
    if lumped and k != 1:
        raise ValueError("lumping is defined for P1 only")
    n = n_nodes(k, m)
    h = (x1 - x0) / m
    if lumped:
        xq, wq = np.array([0.0, 1.0]), np.array([0.5, 0.5])
    else:
        xq, wq = gauss_legendre(nq)
    phi, dphi = lagrange_ref(k, xq)
    # reference derivative -> physical derivative: d/dx = (1/h) d/dxi
    basis = {0: phi, 1: dphi / h}
    K = np.zeros((n, n))
    for e in range(m):
        xe = x0 + h * (e + xq)
        we = np.ones_like(xe) if w is None else np.asarray(w(xe), dtype=np.float64)
        for a in range(k + 1):
            for b in range(k + 1):
                val = np.sum(wq * h * we * basis[di][a] * basis[dj][b])
                K[e * k + a, e * k + b] += val
    return K


# ---------------------------------------------------------------------------
# The full set of 1D matrices of Sec. 3.2 for one x-normal geometry.
# ---------------------------------------------------------------------------

def xnormal_matrices(k, m_s, m_t, L, dL, lumped=False, nq=12,
                     s_interval=(0.0, 1.0), t_interval=(0.0, 1.0)):
    """All 1D matrices of eqs. (23), (29)-(31) (or their lumped versions).

    s-direction (base, L-dependent): B1, C2, M1, M2, M3.
    t-direction (normalised, [0, 1]): A, M, B2, C1.
    Returns a dict of dense full-node matrices.
    """
    s0, s1 = s_interval
    t0, t1 = t_interval
    kk = 1 if lumped else k
    S = dict(
        B1=assemble(kk, m_s, 1, 1, lambda s: L(s), s0, s1, lumped, nq),
        C2=assemble(kk, m_s, 1, 0, lambda s: dL(s), s0, s1, lumped, nq),
        M1=assemble(kk, m_s, 0, 0, lambda s: 1.0 / L(s), s0, s1, lumped, nq),
        M2=assemble(kk, m_s, 0, 0, lambda s: dL(s) ** 2 / L(s), s0, s1, lumped, nq),
        M3=assemble(kk, m_s, 0, 0, lambda s: L(s), s0, s1, lumped, nq),
    )
    T = dict(
        A=assemble(kk, m_t, 1, 1, None, t0, t1, lumped, nq),
        M=assemble(kk, m_t, 0, 0, None, t0, t1, lumped, nq),
        B2=assemble(kk, m_t, 1, 1, lambda t: t ** 2, t0, t1, lumped, nq),
        C1=assemble(kk, m_t, 1, 0, lambda t: t, t0, t1, lumped, nq),
    )
    S.update(T)
    return S

"""Multiterm Sylvester operators and right-hand sides of MO-FEM.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sources in the paper:
* elliptic operator, P_k: Sec. 5, eq. (70) and the operator eq. (73)
  L(U) = M1 U A + (B1 + g M3) U M + M2 U B2 - C2 U C1 - C2^T U C1^T,
  right-hand side eq. (74)  R = M3 F M;
* lumped P1: eqs. (71), (75), (76) - the same five-term structure with the
  lumped matrices of Sec. 3.3 (see ``oracle.fem1d`` for the lumping);
* IMEX operator, eq. (91):  M3 U M + d tau (five terms with g = 0),
  right-hand side eq. (93): M3 (U + tau f(U)) M;
* Dirichlet trimming: Remark "Homogeneous Dirichlet boundary conditions"
  (Sec. 3.3) and the dimension q of eq. (48);
* the vec identity of Sec. 1 (eq. (8)) for the Kronecker form.

Readings where the paper is silent or ambiguous:
* Dirichlet right-hand side keeps the full-node interpolant of f: the load
  is M3[I,:] F M[:,I] with F sampled at all n x n nodes;
* the lumped IMEX operator eq. (92) is left-multiplied by D1; the oracle
  divides that factor out (same solution, symmetric operator):
  M0 D1 U M0 + d tau * (lumped elliptic operator with g = 0);
* the rectangle problem of the reaction-diffusion configuration uses the
  square Kronecker form eq. (28) on [0, l]^2 directly.

Pins: tests/test_oracle_problems.py (Kronecker identity against the
brute-force 2D assembly of ``oracle.fem2d``, symmetry, definiteness,
constants in the Neumann kernel, sparse direct solve agreement).
"""
import numpy as np
import scipy.sparse as sp

from . import fem1d


def interior(n, bc):
    """Index set of the unknowns: all nodes (Neumann) or interior (Dirichlet)."""
    if bc == "neumann":
        return np.arange(n)
    if bc == "dirichlet":
        return np.arange(1, n - 1)
    raise ValueError(bc)


class XNormalProblem:
    """P_k (k = 1..4) or lumped P1 MO-FEM on the x-normal domain
    {(X, Y): 0 <= X <= 1, 0 <= Y <= L(X)} mapped from the unit square.

    Parameters
    ----------
    k      : FEM order (1..4); with ``lumped`` it must be 1.
    m      : number of elements per direction (n = k m + 1 nodes).
    bc     : "dirichlet" or "neumann".
    L, dL  : the boundary curve L(s) > 0 and its derivative.
    gamma  : reaction coefficient of -Lap u + gamma u = f.
    """

    def __init__(self, k, m, bc, L, dL, gamma=0.0, lumped=False, nq=12, m_t=None, t_interval=(0.0, 1.0)):
        self.k, self.m, self.bc, self.gamma, self.lumped = k, m, bc, gamma, lumped
        self.m_t = m if m_t is None else m_t
        self.n = fem1d.n_nodes(1 if lumped else k, m)
        self.n_t = fem1d.n_nodes(1 if lumped else k, self.m_t)
        self.I = interior(self.n, bc)
        self.J = interior(self.n_t, bc)
        self.q = self.I.size
        self.q_t = self.J.size
        full = fem1d.xnormal_matrices(k, m, self.m_t, L, dL, lumped=lumped, nq=nq, t_interval=t_interval)
        self.full = full
        s_keys, t_keys = ("B1", "C2", "M1", "M2", "M3"), ("A", "M", "B2", "C1")
        self.mat = {key: full[key][np.ix_(self.I, self.I)] for key in s_keys}
        self.mat.update({key: full[key][np.ix_(self.J, self.J)] for key in t_keys})
        # row-trimmed (q x n) mass matrices for the full-node load vector
        self.M3_rows = full["M3"][self.I, :]
        self.M_rows = full["M"][self.J, :]

    # -- operators -----------------------------------------------------------
    def apply(self, U, gamma=None):
        """Elliptic operator of eq. (73) (eq. (75) when lumped)."""
        g = self.gamma if gamma is None else gamma
        T = self.mat
        return (T["M1"] @ U @ T["A"]
                + (T["B1"] + g * T["M3"]) @ U @ T["M"]
                + T["M2"] @ U @ T["B2"]
                - T["C2"] @ U @ T["C1"]
                - T["C2"].T @ U @ T["C1"].T)

    def apply_imex(self, U, c):
        """IMEX operator of eq. (91): M3 U M + c * (five stiffness terms),
        c = d * tau (lumped: the D1-free symmetric form of eq. (92))."""
        T = self.mat
        return T["M3"] @ U @ T["M"] + c * self.apply(U, gamma=0.0)

    def mass_apply(self, U):
        """M3 U M on the unknowns (the discrete L-weighted mass form)."""
        return self.mat["M3"] @ U @ self.mat["M"]

    def rhs(self, F_full):
        """Load of eq. (74): M3 F M with F given at all n x n nodes."""
        return self.M3_rows @ F_full @ self.M_rows.T

    def rhs_imex(self, U, tau, fU=None):
        """IMEX right-hand side of eq. (93): M3 (U + tau f(U)) M on the
        unknowns (f evaluated at the unknowns)."""
        V = U if fU is None else U + tau * fU
        return self.mat["M3"] @ V @ self.mat["M"]

    # -- Kronecker form --------------------------------------------------------
    def kron(self, c=None, gamma=None, imex=False):
        """Sparse matrix K with vec_r(L(U)) = K vec_r(U), vec_r = row-major
        flattening; uses vec_r(P U Q) = (P kron Q^T) vec_r(U)."""
        T = {key: sp.csr_matrix(v) for key, v in self.mat.items()}
        g = self.gamma if gamma is None else gamma
        if imex:
            g = 0.0
        K = (sp.kron(T["M1"], T["A"].T) + sp.kron(T["B1"] + g * T["M3"], T["M"].T)
             + sp.kron(T["M2"], T["B2"].T) - sp.kron(T["C2"], T["C1"].T)
             - sp.kron(T["C2"].T, T["C1"]))
        if imex:
            K = sp.kron(T["M3"], T["M"].T) + c * K
        return sp.csr_matrix(K)

    # -- preconditioner pairs ---------------------------------------------------
    def prec_pairs(self, preset):
        """(K_s, M_s), (K_t, M_t) and D-coefficients for a preconditioner
        preset.  D_ij = alpha + beta_s lam_i + beta_t mu_j + delta lam_i mu_j
        and the preconditioning operator is
        P(U) = alpha Ms U Mt + beta_s Ks U Mt + beta_t Ms U Kt + delta Ks U Kt.
        Presets:
          sylv          (B1, M3) x (A, M), D = gamma + lam + mu
          sylv-matched  (B1, M1) x (A + w B2, M), D = gamma + lam + mu,
                        w = sum(M2) / sum(M1) over the untrimmed matrices
                        (= int L'^2/L / int 1/L): the operator's M1 U A and
                        B1 U M terms exact, its M2 U B2 term taken as
                        w M1 U B2 and gamma M3 U M as gamma M1 U M (the
                        library's elliptic default)
          paper-product eq. (80): B1 U (A + B2), D = lam * mu
        IMEX presets (``imex_prec_pairs``) add the coefficient c:
          sylv-imex          (B1, M3) x (A, M), D = 1 + c (lam + mu)
          sylv-imex-matched  (B1, M3) x (A + w3 B2, M), w3 = sum(M2) / sum(M3)
                             (untrimmed): the mass term M3 U M exact, the
                             stiffness part's M2 U B2 taken as w3 M3 U B2
                             (the library's IMEX default)
          paper-imex         eq. (95)
        """
        T = self.mat
        Is, It = np.eye(self.q), np.eye(self.q_t)
        if preset == "sylv":
            return (T["B1"], T["M3"]), (T["A"], T["M"]), (self.gamma, 1.0, 1.0, 0.0)
        if preset == "sylv-matched":
            w = self.full["M2"].sum() / self.full["M1"].sum()
            return (T["B1"], T["M1"]), (T["A"] + w * T["B2"], T["M"]), (self.gamma, 1.0, 1.0, 0.0)
        if preset == "paper-product":
            return (T["B1"], Is), (T["A"] + T["B2"], It), (0.0, 0.0, 0.0, 1.0)
        raise ValueError(preset)

    def imex_prec_pairs(self, preset, c):
        T = self.mat
        if preset == "sylv-imex":
            return (T["B1"], T["M3"]), (T["A"], T["M"]), (1.0, c, c, 0.0)
        if preset == "sylv-imex-matched":
            w3 = self.full["M2"].sum() / self.full["M3"].sum()
            return (T["B1"], T["M3"]), (T["A"] + w3 * T["B2"], T["M"]), (1.0, c, c, 0.0)
        if preset == "paper-imex":
            # eq. (95): (M3 + c B1)^-1 U (M + c (A + B2))^-1
            return ((T["M3"] + c * T["B1"], np.eye(self.q)), (T["M"] + c * (T["A"] + T["B2"]), np.eye(self.q_t)),
                    (0.0, 0.0, 0.0, 1.0))
        raise ValueError(preset)


class RectProblem:
    """Square-domain Kronecker form eq. (28) on the rectangle
    [0, lx] x [0, ly]:  mass  Mx kron My, stiffness Ax kron My + Mx kron Ay.
    Used for the reaction-diffusion configuration (Sec. 7 with a rectangle).
    IMEX operator (eq. (91) with L = 1): Mx U My + c (Ax U My + Mx U Ay).
    """

    def __init__(self, k, m, bc, lx=1.0, ly=1.0, lumped=False, nq=12, gamma=0.0):
        self.k, self.m, self.bc, self.lumped, self.gamma = k, m, bc, lumped, gamma
        kk = 1 if lumped else k
        self.n = fem1d.n_nodes(kk, m)
        self.I = interior(self.n, bc)
        self.q = self.I.size
        ix = np.ix_(self.I, self.I)
        self.Ax = fem1d.assemble(kk, m, 1, 1, None, 0.0, lx, lumped, nq)[ix]
        self.Mx = fem1d.assemble(kk, m, 0, 0, None, 0.0, lx, lumped, nq)[ix]
        self.Ay = fem1d.assemble(kk, m, 1, 1, None, 0.0, ly, lumped, nq)[ix]
        self.My = fem1d.assemble(kk, m, 0, 0, None, 0.0, ly, lumped, nq)[ix]

    def apply(self, U, gamma=None):
        g = self.gamma if gamma is None else gamma
        return self.Ax @ U @ self.My + self.Mx @ U @ self.Ay + g * self.Mx @ U @ self.My

    def apply_imex(self, U, c):
        return self.Mx @ U @ self.My + c * self.apply(U, gamma=0.0)

    def mass_apply(self, U):
        return self.Mx @ U @ self.My

    def rhs_imex(self, U, tau, fU=None):
        V = U if fU is None else U + tau * fU
        return self.Mx @ V @ self.My

    def kron(self, c=None, gamma=None, imex=False):
        Ax, Mx, Ay, My = (sp.csr_matrix(a) for a in (self.Ax, self.Mx, self.Ay, self.My))
        g = self.gamma if gamma is None else gamma
        S = sp.kron(Ax, My.T) + sp.kron(Mx, Ay.T)
        if imex:
            return sp.csr_matrix(sp.kron(Mx, My.T) + c * S)
        return sp.csr_matrix(S + g * sp.kron(Mx, My.T))

    def prec_pairs(self, preset="rect"):
        return (self.Ax, self.Mx), (self.Ay, self.My), (self.gamma, 1.0, 1.0, 0.0)

    def imex_prec_pairs(self, preset, c):
        if preset not in ("rect", "sylv-imex"):
            raise ValueError(preset)
        return (self.Ax, self.Mx), (self.Ay, self.My), (1.0, c, c, 0.0)


def vec_r(U):
    """Row-major vectorisation."""
    return np.ascontiguousarray(U).reshape(-1)

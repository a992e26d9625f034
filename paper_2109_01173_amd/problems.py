"""Composition of the MO-FEM operators from the library's 1D matrices.

Only bookkeeping happens here: which assembled 1D matrix goes into which term
of the multiterm operator.  Assembly (``mofem_assemble_1d``), the
eigen-decomposition, every sum of bands (the library merges terms that share
a factor, and forms the preconditioners' A + B2 and A + w B2 itself) and every
apply/solve run in libmofem; no band is formed in Python (the numbers taken
from bands are the weights w, ratios of two bands' total masses).

Operators (rows = s, the base coordinate; columns = t):
* x-normal elliptic, eq. (73) (lumped: eq. (75)):
    M1 U A + (B1 + g M3) U M + M2 U B2 - C2 U C1 - C2^T U C1^T
  right-hand side eq. (74): M3 F M with F on all nodes (rows/cols trimmed);
* x-normal IMEX, eq. (91): M3 U M + c (the five terms with g = 0), with
  c = d tau passed per batch item;
* rectangle (eq. (28) on [0, l]^2): elliptic (A + g M) U M + M U A,
  IMEX  M U M + c (A U M + M U A).
Preconditioners: the spectral single-term form with the pencils
(B1, M1) x (A + w B2, M), D = g + lam + mu, w = sum(M2) / sum(M1), for the
x-normal elliptic operator (its M1 U A and B1 U M terms exact, M2 U B2 taken
as w M1 U B2), (B1, M3) x (A + w3 B2, M), w3 = sum(M2) / sum(M3), for the
x-normal IMEX operator (its mass term M3 U M exact) and (A, M) x (A, M) on
the rectangle;
the paper's product preconditioners eqs. (80), (95), (96) by banded Cholesky
solves (XNormal.product_prec).
"""
import math

from . import mofem as mf


def _assemble(order, m, di, dj, kind=mf.W_ONE, p=(0, 0, 0, 0), x0=0.0, x1=1.0):
    w = None if kind == mf.W_ONE else mf.weight(kind, p)
    return mf.assemble_1d(order, m, di, dj, w, x0, x1)


class XNormal:
    """P_k (k = 1..4) or lumped P1 (lumped=True, k = 1) on an x-normal domain
    mapped from [0, 1] x [t0, t1] by (s, t) -> (s, t L(s)).

    profile: ("sine", amp): L(s) = 1 + amp sin(pi s) on t in [0, 1] (the
             domain {0 <= Y <= L(X)}); ("poly", (p0, p1, p2, p3)): a cubic
             L(s); the symmetric domains {|X| <= S(Y)} of the remark after
             eq. (19) use t_interval = (-1/2, 1/2) and L = 2 S, e.g. the
             cap-shaped domain S = 1 - s^2 / 2: ("poly", (2, 0, -1, 0)).
    m_t:     elements along t (default m), so q_s and q_t may differ."""

    def __init__(self, k, m, bc, gamma=0.0, amp=0.3, lumped=False, precision=mf.PREC_F64,
                 imex=False, m_t=None, profile=None, t_interval=(0.0, 1.0)):
        self.k, self.m, self.bc, self.gamma, self.lumped = k, m, bc, gamma, lumped
        m_t = m if m_t is None else m_t
        self.m_t = m_t
        order = 0 if lumped else k
        self.kb = 1 if lumped else k
        self.n = self.kb * m + 1
        self.n_t = self.kb * m_t + 1
        trim = 1 if bc == "dirichlet" else 0
        self.trim = trim
        self.q = self.n - 2 * trim
        self.q_t = self.n_t - 2 * trim
        kind, prof = profile if profile is not None else ("sine", amp)
        if kind == "sine":
            p = (1.0, prof, math.pi, 0.0)
            wL, wD, wI, wD2 = mf.W_PROFILE, mf.W_PROFILE_D, mf.W_PROFILE_INV, mf.W_PROFILE_D2L
        elif kind == "poly":
            p = tuple(float(c) for c in prof)
            wL, wD, wI, wD2 = mf.W_POLY, mf.W_PPROFILE_D, mf.W_PPROFILE_INV, mf.W_PPROFILE_D2L
        else:
            raise ValueError("profile kind must be 'sine' or 'poly'")
        t0, t1 = t_interval
        B1 = _assemble(order, m, 1, 1, wL, p)
        C2 = _assemble(order, m, 1, 0, wD, p)
        M1 = _assemble(order, m, 0, 0, wI, p)
        M2 = _assemble(order, m, 0, 0, wD2, p)
        M3 = _assemble(order, m, 0, 0, wL, p)
        A = _assemble(order, m_t, 1, 1, x0=t0, x1=t1)
        M = _assemble(order, m_t, 0, 0, x0=t0, x1=t1)
        B2 = _assemble(order, m_t, 1, 1, mf.W_POLY, (0, 0, 1, 0), x0=t0, x1=t1)
        C1 = _assemble(order, m_t, 1, 0, mf.W_POLY, (0, 1, 0, 0), x0=t0, x1=t1)
        self.bands = dict(B1=B1, C2=C2, M1=M1, M2=M2, M3=M3, A=A, M=M, B2=B2, C1=C1)
        eo = 0 if lumped else k
        common = dict(n_s=self.n, n_t=self.n_t, kb=self.kb, trim_s=trim, trim_t=trim, elem_order=eo)
        if imex:
            terms = [dict(left=M3, right=M),
                     dict(left=M1, right=A, scaled=True),
                     dict(left=B1, right=M, scaled=True),
                     dict(left=M2, right=B2, scaled=True),
                     dict(left=C2, right=C1, coef=-1.0, scaled=True),
                     dict(left=C2, right=C1, coef=-1.0, left_T=True, right_T=True, scaled=True)]
            coeffs = (1.0, 1.0, 1.0, 0.0)
        else:
            terms = [dict(left=M1, right=A),
                     dict(left=B1, right=M),
                     dict(left=M3, right=M, coef=gamma),      # merged with B1 U M by the library
                     dict(left=M2, right=B2),
                     dict(left=C2, right=C1, coef=-1.0),
                     dict(left=C2, right=C1, coef=-1.0, left_T=True, right_T=True)]
            coeffs = (gamma, 1.0, 1.0, 0.0)
        self.op = mf.Operator(terms, **common)
        self.rhs_op = mf.Operator([dict(left=M3, right=M)], full_input=True, **common)
        # transpose of the full-node load: dJ/dF = M3[:, I] Lambda M[I, :]
        self.rhs_adjoint_op = mf.Operator([dict(left=M3, right=M)], full_output=True, **common)
        self.mass = mf.Operator([dict(left=M3, right=M)], **common)
        # stiffness part K of L_c = Mass + c K (for the gradient in d)
        self.stiff = mf.Operator([dict(t, scaled=False) for t in terms[1:]], **common) if imex else None
        if imex:
            # the stiffness part's M2 U B2 taken as w3 M3 U B2, w3 = sum(M2) / sum(M3)
            w3_b2 = float(M2.sum() / M3.sum())
            self.prec = mf.Preconditioner(B1, M3, A, M, coeffs, trim, trim, precision, Kt_add=[(B2, w3_b2)])
        else:
            # the operator's M2 U B2 taken as w M1 U B2, w the ratio of the
            # total masses of M2 and M1 (the integrals of L'^2 / L and 1 / L)
            w_b2 = float(M2.sum() / M1.sum())
            self.prec = mf.Preconditioner(B1, M1, A, M, coeffs, trim, trim, precision, Kt_add=[(B2, w_b2)])
        self.imex = imex

    def product_prec(self, scales=(1.0,)):
        """The paper's own product preconditioner by banded Cholesky solves:
        elliptic eq. (80), B1 U (A + B2) (lumped: A1 U (A + A2));
        IMEX eq. (95), (M3 + c B1) U (M + c (A + B2)) (lumped eq. (96):
        M0 D1 and M0 in place of M3 and M), one factor pair per c = d tau in
        `scales` (the item scale of each item selects its pair)."""
        b = self.bands
        AB2 = [(b["A"], 1.0), (b["B2"], 1.0)]    # summed by the library
        if self.imex:
            return mf.BandedPreconditioner(b["B1"], b["M3"], AB2, b["M"], a=1.0, bs=1.0, bt=1.0, scales=scales,
                                           trim_s=self.trim, trim_t=self.trim)
        return mf.BandedPreconditioner(b["B1"], None, AB2, None, a=0.0, bs=1.0, bt=1.0, scales=(1.0,),
                                       trim_s=self.trim, trim_t=self.trim)


class Rect:
    """Square Kronecker form eq. (28) on [0, length]^2 (P_k or lumped P1).

    closed_form: for P1 (consistent mass with Dirichlet conditions, or lumped
    mass) the preconditioner's eigenpairs come from the closed forms of
    Sec. 4.1 (mofem_eig_p1_closed) instead of a dense eigen-decomposition."""

    def __init__(self, k, m, bc, length=1.0, gamma=0.0, lumped=False, precision=mf.PREC_F64,
                 imex=False, closed_form=False):
        order = 0 if lumped else k
        self.kb = 1 if lumped else k
        self.n = self.kb * m + 1
        trim = 1 if bc == "dirichlet" else 0
        self.trim = trim
        self.q = self.n - 2 * trim
        A = _assemble(order, m, 1, 1, x1=length)
        M = _assemble(order, m, 0, 0, x1=length)
        self.bands = dict(A=A, M=M)
        eo = 0 if lumped else k
        common = dict(n_s=self.n, n_t=self.n, kb=self.kb, trim_s=trim, trim_t=trim, elem_order=eo)
        if imex:
            terms = [dict(left=M, right=M), dict(left=A, right=M, scaled=True),
                     dict(left=M, right=A, scaled=True)]
            coeffs = (1.0, 1.0, 1.0, 0.0)
        else:
            terms = [dict(left=A, right=M), dict(left=M, right=M, coef=gamma), dict(left=M, right=A)]
            coeffs = (gamma, 1.0, 1.0, 0.0)
        self.op = mf.Operator(terms, **common)
        self.rhs_op = mf.Operator([dict(left=M, right=M)], full_input=True, **common)
        self.rhs_adjoint_op = mf.Operator([dict(left=M, right=M)], full_output=True, **common)
        self.mass = mf.Operator([dict(left=M, right=M)], **common)
        self.stiff = mf.Operator([dict(t, scaled=False) for t in terms[1:]], **common) if imex else None
        if closed_form:
            if self.kb != 1:
                raise ValueError("closed-form eigenpairs exist for P1 only")
            lam, V = mf.eig_p1_closed(m, length, lumped, trim == 1)
            self.prec = mf.Preconditioner.from_eigen(lam, V, lam, V, coeffs, precision)
        else:
            self.prec = mf.Preconditioner(A, M, A, M, coeffs, trim, trim, precision)

"""Matching problem pairs for the GPU parity tests: the library's problem
(paper_2109_01173_amd.problems, assembled by libmofem) and the oracle's
problem (oracle.problems, assembled in NumPy) for the same discretisation."""
import numpy as np

from oracle.problems import RectProblem, XNormalProblem
from workloads import GEOM_AMP, L_profile, dL_profile


def oracle_xnormal(k, m, bc, gamma, lumped=False):
    return XNormalProblem(k, m, bc, L_profile, dL_profile, gamma=gamma, lumped=lumped)


def gpu_xnormal(k, m, bc, gamma, lumped=False, imex=False, precision=None):
    from paper_2109_01173_amd import mofem as mf
    from paper_2109_01173_amd.problems import XNormal
    prec = mf.PREC_F64 if precision is None else precision
    return XNormal(k, m, bc, gamma=gamma, amp=GEOM_AMP, lumped=lumped, precision=prec, imex=imex)


def oracle_abs_apply(P, X, c=None):
    """|L| applied to |X| term by term (a forward rounding-error scale)."""
    T = {key: np.abs(v) for key, v in P.mat.items()}
    A = np.abs(X)
    g = abs(P.gamma) if c is None else 0.0
    s = (T["M1"] @ A @ T["A"] + (T["B1"] + g * T["M3"]) @ A @ T["M"] + T["M2"] @ A @ T["B2"]
         + T["C2"] @ A @ T["C1"] + T["C2"].T @ A @ T["C1"].T)
    if c is not None:
        s = T["M3"] @ A @ T["M"] + abs(c) * s
    return s


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()

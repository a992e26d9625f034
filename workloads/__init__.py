"""Seeded synthetic inputs and workload descriptions.

This module is shared by the oracle (``oracle/``) and by the GPU path's
callers (tests, ``bench.py``).  It holds problem DATA only - domain shape,
manufactured solutions, random fields and configuration sizes - and none of
the method's arithmetic (no assembly, operators, preconditioners or
solvers).  Every random array is drawn here from
``numpy.random.default_rng(seed)`` and handed to both sides.

Workloads (all FP64, all synthetic; the paper uses no external dataset):

* ``elliptic_small``  P1, homogeneous Dirichlet, n = 65 nodes per direction,
  gamma = 1, domain {0 < X < 1, 0 < Y < 1 + 0.3 sin(pi X)}, F from the
  manufactured solution u = sin(pi X) sin(pi Y / L(X)).
* ``elliptic_p2``     the headline: P2 (also P3), Dirichlet, n = 1025 or 2049,
  gamma = 1, F = manufactured source + N(0, 1e-3^2) noise at every node,
  seed 1234 + b for batch item b, batch 16.
* ``heat_p4``         P4, Neumann, n = 2049, d = 0.1, tau = 1e-3, 1000 steps,
  f = 0, U0 ~ U[0, 1) (seed 42).
* ``dib_rect``        DIB kinetics on the rectangle [0, 20]^2, Neumann,
  lumped P1 (m = 1024) and P2 (m = 512), n = 1025, d_theta = 20, rho = 1,
  tau = 1e-2, T = 100; eta0 = U[-1e-3, 1e-3), theta0 = 0.5 + U[-1e-3, 1e-3)
  (seed 7, eta drawn first).
"""
import numpy as np

# ---------------------------------------------------------------------------
# Domain shape: Y in [0, L(X)], L(s) = 1 + a sin(pi s)  (x-normal domain of
# Sec. 2.2 with the roles of the axes named as in the configuration).
# ---------------------------------------------------------------------------
GEOM_AMP = 0.3


def L_profile(s, a=GEOM_AMP):
    return 1.0 + a * np.sin(np.pi * s)


def dL_profile(s, a=GEOM_AMP):
    return a * np.pi * np.cos(np.pi * s)


def exact_u(s, t):
    """Manufactured solution in reference coordinates: u = sin(pi s) sin(pi t),
    i.e. sin(pi X) sin(pi Y / L(X)) on the physical domain."""
    return np.sin(np.pi * s) * np.sin(np.pi * t)


def manufactured_f(s, t, gamma, a=GEOM_AMP):
    """f = -Lap u + gamma u for ``exact_u`` on the physical domain, written in
    the reference coordinates (s, t) with X = s, Y = t L(s)."""
    S, Cs = np.sin(np.pi * s), np.cos(np.pi * s)
    T, Ct = np.sin(np.pi * t), np.cos(np.pi * t)
    L = 1.0 + a * S
    dL = a * np.pi * Cs
    ddL = -a * np.pi ** 2 * S
    g = dL / L
    return (np.pi ** 2 * S * T * (1.0 + t ** 2 * g ** 2 + L ** -2)
            + np.pi * t * (ddL / L - 2.0 * dL ** 2 / L ** 2) * S * Ct
            + 2.0 * np.pi ** 2 * t * g * Cs * Ct + gamma * S * T)


def grid(n):
    """Equispaced node coordinates of P_k on a uniform mesh (all n nodes)."""
    return np.arange(n, dtype=np.float64) / (n - 1)


def elliptic_F(n, gamma, sigma=0.0, seed=None, a=GEOM_AMP):
    """Full-node source field F (n x n, rows = s nodes) for the manufactured
    problem, plus optional seeded Gaussian noise of standard deviation sigma."""
    x = grid(n)
    S, T = np.meshgrid(x, x, indexing="ij")
    F = manufactured_f(S, T, gamma, a)
    if sigma:
        rng = np.random.default_rng(seed)
        F = F + sigma * rng.standard_normal((n, n))
    return np.ascontiguousarray(F)


def elliptic_batch(n, gamma, batch, sigma=1e-3, seed0=1234):
    """Batch of full-node sources, item b seeded with seed0 + b."""
    return np.stack([elliptic_F(n, gamma, sigma, seed0 + b) for b in range(batch)])


def heat_initial(q, seed=42):
    return np.random.default_rng(seed).random((q, q))


def dib_initial(q, seed=7, amp=1e-3, eta_e=0.0, theta_e=0.5):
    rng = np.random.default_rng(seed)
    eta = eta_e + rng.uniform(-amp, amp, (q, q))
    theta = theta_e + rng.uniform(-amp, amp, (q, q))
    return eta, theta


def nodes_for(k, n_target):
    """Elements m and node count n = k m + 1 closest to n_target nodes."""
    m = int(round((n_target - 1) / k))
    return m, k * m + 1


# ---------------------------------------------------------------------------
# DIB parameters (Sec. 7, eq. (103); cap set of Sec. 7.1).  D is set so that
# (eta, theta) = (0, 1/2) is an equilibrium: D = 9 C / 11 (the printed
# 3.2727 = 36/11 corresponds to C = 4).
# ---------------------------------------------------------------------------
def dib_params(C=7.0, A2=30.0, B=25.0, rho=1.0):
    return dict(alpha=0.5, gamma=0.2, A1=10.0, A2=A2, B=B, C=C, D=9.0 * C / 11.0,
                k2=2.5, k3=1.5, d_theta=20.0, rho=rho)


WORKLOADS = {
    "elliptic_small": dict(k=1, n=65, bc="dirichlet", gamma=1.0, tol=1e-10),
    "elliptic_p2": dict(k=2, n=2049, bc="dirichlet", gamma=1.0, sigma=1e-3,
                        batch=16, tol=1e-8, seed0=1234),
    "heat_p4": dict(k=4, n=2049, bc="neumann", d=0.1, tau=1e-3, steps=1000, seed=42),
    "dib_rect": dict(n=1025, bc="neumann", length=20.0, tau=1e-2, T=100.0, seed=7),
}


def describe(name):
    return dict(WORKLOADS[name], name=name)


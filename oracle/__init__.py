"""Plain, slow FP64 CPU oracle for the MO-FEM / MO-PCG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the ``libmofem``
shared library and its Python binding) may import, call or link anything in
this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Reference: M. Frittelli, I. Sgura, "Matrix-oriented FEM formulation for
stationary and time-dependent PDEs on x-normal domains" (arXiv 2109.01173).
Citations name the paper's sections and its equations in the order the
article numbers them, e.g. "Sec. 5, eq. (70)".

Conventions (fixed once, used everywhere):

* ``s`` is the base coordinate of the x-normal domain (the paper's ``y``),
  ``t`` the normalised coordinate in [0, 1] (the paper's ``x``).  A physical
  point is ``(X, Y) = (s, t * L(s))``.
* A nodal matrix ``U`` has shape ``(q_s, q_t)``: row ``i`` is an ``s`` node,
  column ``j`` a ``t`` node.  Left factors act on ``s``, right factors on ``t``
  (this is the orientation of eq. (70)).
* All arithmetic is float64.

Modules:

* :mod:`oracle.fem1d`     - Lagrange P_k basis, quadrature, 1D matrices (Sec. 3)
* :mod:`oracle.fem2d`     - brute-force 2D assembly on the mapped domain (pin)
* :mod:`oracle.problems`  - multiterm operators, right-hand sides (Sec. 4-6)
* :mod:`oracle.solvers`   - spectral preconditioner, MO-PCG, direct solve
* :mod:`oracle.imex`      - IMEX Euler steps and DIB kinetics (Sec. 6-7)
* :mod:`oracle.errors`    - L2 error by quadrature (convergence pins)

Parity pinning status of every function is listed in each module header.
"""

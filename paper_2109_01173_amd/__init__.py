"""MI355X-native MO-FEM / MO-PCG (matrix-oriented FEM multiterm Sylvester
solves, arXiv 2109.01173).

The compute path is the native library ``libmofem.so`` (include/mofem.h):
host C++ for 1D assembly and the one-off eigen-decomposition, hand-written
HIP kernels for gfx950 for the operator, the spectral preconditioner, the
PCG recurrence and the IMEX step.  ``mofem`` is its ctypes binding and
``problems`` composes the operators of the paper from assembled 1D matrices.
"""
__all__ = ["mofem", "problems"]

"""ctypes binding of libmofem (include/mofem.h).

Argument marshalling only: every computation runs in the native library
(host C++ for assembly and eigen-decomposition, HIP kernels on the GPU for
everything else).  Device arrays are torch tensors on the current HIP device
(float64, contiguous); the current torch stream is passed to the library.
If the shared library is missing this module raises at import time - there
is no fallback.
"""
import ctypes
import os

import numpy as np

# torch ships its own HIP runtime (same soname as ROCm's libamdhip64.so.7).
# Import it first so that libmofem binds to that already-loaded runtime; two
# HIP runtimes in one process cannot share the device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MOFEM_LIB", os.path.join(_HERE, "libmofem.so"))

if not os.path.exists(LIB_PATH):
    raise ImportError("libmofem.so not found at %s - build it first "
                      "(python -m paper_2109_01173_amd.build)" % LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (mirror include/mofem.h) -------------------------------------
OK = 0
E_ARG, E_HIP, E_NOMEM, E_BREAKDOWN, E_MAXIT, E_UNSUPPORTED, E_NOTFINITE, E_NUMERIC = (
    -1, -2, -3, -4, -5, -6, -7, -8)
W_ONE, W_POLY, W_PROFILE, W_PROFILE_D, W_PROFILE_INV, W_PROFILE_D2L, W_CALLBACK = range(7)
W_PPROFILE_D, W_PPROFILE_INV, W_PPROFILE_D2L = 7, 8, 9
PREC_F64, PREC_F32, PREC_BF16, PREC_BF16X3, PREC_BF16X2, PREC_BF16_FWD, PREC_F64_INT8, PREC_BF16_FWD_VS = range(8)
PCG_FLEXIBLE, PCG_ZERO_GUESS, PCG_TAU_STOP = 1, 2, 4
KIN_NONE, KIN_DIB = 0, 1
(TRACE_BAND, TRACE_GEMM_F64, TRACE_GEMM_BF16X3, TRACE_GEMM_BF16, TRACE_VEC, TRACE_GEMM_BF16X2, TRACE_GEMM_F32,
 TRACE_BCHOL, TRACE_GEMM_I8) = range(9)
TRACE_CLASSES = 9
MAX_TERMS = 8
MAX_SCALES = 8

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
WeightFn = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_void_p)


class Weight(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("p", ctypes.c_double * 4), ("fn", WeightFn), ("ctx", _vp)]


class OpDesc(ctypes.Structure):
    _fields_ = [("kb", ctypes.c_int), ("elem_order", ctypes.c_int), ("n_s", ctypes.c_int),
                ("n_t", ctypes.c_int), ("trim_s", ctypes.c_int), ("trim_t", ctypes.c_int),
                ("full_input", ctypes.c_int), ("n_terms", ctypes.c_int),
                ("left", _vp * MAX_TERMS), ("right", _vp * MAX_TERMS),
                ("left_transpose", ctypes.c_int * MAX_TERMS),
                ("right_transpose", ctypes.c_int * MAX_TERMS),
                ("coef", ctypes.c_double * MAX_TERMS), ("scaled", ctypes.c_int * MAX_TERMS),
                ("full_output", ctypes.c_int)]


MAX_BAND_SUM = 4


class BandSum(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("band", _vp * MAX_BAND_SUM), ("coef", ctypes.c_double * MAX_BAND_SUM)]


class PrecDesc(ctypes.Structure):
    _fields_ = [("kb", ctypes.c_int), ("n_s", ctypes.c_int), ("n_t", ctypes.c_int),
                ("trim_s", ctypes.c_int), ("trim_t", ctypes.c_int),
                ("Ks", _vp), ("Ms", _vp), ("Kt", _vp), ("Mt", _vp),
                ("alpha", ctypes.c_double), ("beta_s", ctypes.c_double),
                ("beta_t", ctypes.c_double), ("delta", ctypes.c_double),
                ("precision", ctypes.c_int), ("Ks_add", BandSum), ("Kt_add", BandSum)]




class BPrecDesc(ctypes.Structure):
    _fields_ = [("kb", ctypes.c_int), ("n_s", ctypes.c_int), ("n_t", ctypes.c_int),
                ("trim_s", ctypes.c_int), ("trim_t", ctypes.c_int),
                ("Ks", BandSum), ("Ms", BandSum), ("Kt", BandSum), ("Mt", BandSum),
                ("a", ctypes.c_double), ("bs", ctypes.c_double), ("bt", ctypes.c_double),
                ("n_scales", ctypes.c_int), ("scales", ctypes.c_double * MAX_SCALES)]


class PcgGroup(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("prec", ctypes.c_void_p), ("rhs", ctypes.c_void_p),
                ("u", ctypes.c_void_p), ("stride", ctypes.c_longlong), ("batch", ctypes.c_int),
                ("item_scale", ctypes.c_void_p), ("tol", ctypes.c_double), ("maxit", ctypes.c_int),
                ("flags", ctypes.c_uint), ("workspace", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("iters_out", ctypes.c_void_p), ("relres_out", ctypes.c_void_p)]


class ImexDesc(ctypes.Structure):
    _fields_ = [("op", _vp), ("prec", _vp), ("mass", _vp), ("tau", ctypes.c_double),
                ("d", ctypes.c_double * 2), ("n_species", ctypes.c_int),
                ("kinetics", ctypes.c_int), ("kin", ctypes.c_double * 10),
                ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("flags", ctypes.c_uint)]


def _proto(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_ll = ctypes.c_longlong
_sz = ctypes.c_size_t
mofem_version = _proto("mofem_version", ctypes.c_int, [])
mofem_last_error = _proto("mofem_last_error", ctypes.c_char_p, [])
mofem_assemble_1d = _proto("mofem_assemble_1d", ctypes.c_int,
                           [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                            ctypes.c_int, ctypes.c_int, ctypes.POINTER(Weight), ctypes.c_int, _vp])
mofem_geneig_host = _proto("mofem_geneig_host", ctypes.c_int,
                           [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp])
mofem_set_host_threads = _proto("mofem_set_host_threads", ctypes.c_int, [ctypes.c_int])
mofem_eig_p1_closed = _proto("mofem_eig_p1_closed", ctypes.c_int,
                             [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _vp, _vp])
mofem_op_create = _proto("mofem_op_create", ctypes.c_int, [ctypes.POINTER(OpDesc), ctypes.POINTER(_vp)])
mofem_op_destroy = _proto("mofem_op_destroy", ctypes.c_int, [_vp])
mofem_op_shape = _proto("mofem_op_shape", ctypes.c_int, [_vp, _ip, _ip, _ip, _ip])
mofem_op_apply = _proto("mofem_op_apply", ctypes.c_int,
                        [_vp, _vp, _ll, _vp, _ll, ctypes.c_int, _vp, _vp, _vp])
mofem_op_apply_noalloc = _proto("mofem_op_apply_noalloc", ctypes.c_int,
                                [_vp, _vp, _ll, _vp, _ll, ctypes.c_int, _vp, _vp, _vp])
mofem_prec_setup = _proto("mofem_prec_setup", ctypes.c_int, [ctypes.POINTER(PrecDesc), ctypes.POINTER(_vp)])
mofem_prec_destroy = _proto("mofem_prec_destroy", ctypes.c_int, [_vp])
mofem_prec_setup_eig = _proto("mofem_prec_setup_eig", ctypes.c_int,
                              [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_vp)])
mofem_prec_setup_banded = _proto("mofem_prec_setup_banded", ctypes.c_int,
                                 [ctypes.POINTER(BPrecDesc), ctypes.POINTER(_vp)])
mofem_prec_set_coeffs = _proto("mofem_prec_set_coeffs", ctypes.c_int,
                               [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double])
mofem_prec_set_precision = _proto("mofem_prec_set_precision", ctypes.c_int, [_vp, ctypes.c_int])
mofem_prec_eigenvalues = _proto("mofem_prec_eigenvalues", ctypes.c_int, [_vp, _vp, _vp])
mofem_prec_workspace_size = _proto("mofem_prec_workspace_size", _sz, [_vp, ctypes.c_int])
mofem_prec_apply = _proto("mofem_prec_apply", ctypes.c_int,
                          [_vp, _vp, _vp, _ll, ctypes.c_int, _vp, _vp, _sz, _vp])
mofem_prec_tune = _proto("mofem_prec_tune", ctypes.c_int, [_vp, ctypes.c_int, _ip, _vp])
mofem_prec_set_tile = _proto("mofem_prec_set_tile", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int])
mofem_pcg_workspace_size = _proto("mofem_pcg_workspace_size", _sz, [_vp, _vp, ctypes.c_int])
mofem_pcg_solve = _proto("mofem_pcg_solve", ctypes.c_int,
                         [_vp, _vp, _vp, _vp, _ll, ctypes.c_int, _vp, ctypes.c_double, ctypes.c_int,
                          ctypes.c_uint, _vp, _sz, _vp, _vp, _vp])
mofem_imex_workspace_size = _proto("mofem_imex_workspace_size", _sz, [ctypes.POINTER(ImexDesc), ctypes.c_int])
mofem_imex_step = _proto("mofem_imex_step", ctypes.c_int,
                         [ctypes.POINTER(ImexDesc), _vp, _ll, ctypes.c_int, _vp, _sz, _vp, _vp])
mofem_dot_accumulate = _proto("mofem_dot_accumulate", ctypes.c_int,
                              [_vp, _vp, _ll, _ll, ctypes.c_int, ctypes.c_double, ctypes.c_double, _vp, _vp])
mofem_imex_adjoint_workspace_size = _proto("mofem_imex_adjoint_workspace_size", _sz,
                                           [ctypes.POINTER(ImexDesc), ctypes.c_int])
mofem_imex_adjoint_step = _proto("mofem_imex_adjoint_step", ctypes.c_int,
                                 [ctypes.POINTER(ImexDesc), _vp, _vp, _vp, _vp, _vp, _ll, ctypes.c_int, _vp, _sz,
                                  _vp, _vp])
mofem_pcg_solve_async = _proto("mofem_pcg_solve_async", ctypes.c_int,
                               [_vp, _vp, _vp, _vp, _ll, ctypes.c_int, _vp, ctypes.c_double, ctypes.c_int,
                                ctypes.c_uint, _vp, _sz, _vp, _vp, _vp, _vp])
mofem_imex_graph_create = _proto("mofem_imex_graph_create", ctypes.c_int,
                                 [ctypes.POINTER(ImexDesc), _vp, _ll, ctypes.c_int, _vp, _sz, ctypes.c_int,
                                  ctypes.POINTER(_vp), _vp])
mofem_imex_graph_launch = _proto("mofem_imex_graph_launch", ctypes.c_int, [_vp, ctypes.c_int, _vp])
mofem_imex_graph_result = _proto("mofem_imex_graph_result", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp])
mofem_imex_graph_destroy = _proto("mofem_imex_graph_destroy", ctypes.c_int, [_vp])
mofem_pcg_solve_many = _proto("mofem_pcg_solve_many", ctypes.c_int,
                              [ctypes.c_int, ctypes.POINTER(PcgGroup), ctypes.POINTER(_vp), _vp])
mofem_pcg_solve_grouped = _proto("mofem_pcg_solve_grouped", ctypes.c_int,
                                 [ctypes.c_int, ctypes.POINTER(PcgGroup), ctypes.POINTER(_vp), _vp])
mofem_trace_enable = _proto("mofem_trace_enable", ctypes.c_int, [ctypes.c_int])
mofem_trace_select = _proto("mofem_trace_select", ctypes.c_int, [ctypes.c_uint])
mofem_trace_read = _proto("mofem_trace_read", ctypes.c_int,
                          [ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_longlong), _dp])

EXPORTS = ["mofem_version", "mofem_last_error", "mofem_assemble_1d", "mofem_geneig_host", "mofem_eig_p1_closed",
           "mofem_set_host_threads",
           "mofem_prec_setup_eig",
           "mofem_op_create", "mofem_op_destroy", "mofem_op_shape", "mofem_op_apply", "mofem_op_apply_noalloc",
           "mofem_prec_setup", "mofem_prec_destroy", "mofem_prec_set_coeffs",
           "mofem_prec_set_precision", "mofem_prec_eigenvalues", "mofem_prec_workspace_size",
           "mofem_prec_apply", "mofem_prec_tune", "mofem_prec_set_tile", "mofem_prec_setup_banded",
           "mofem_pcg_workspace_size",
           "mofem_pcg_solve",
           "mofem_imex_workspace_size", "mofem_imex_step", "mofem_dot_accumulate",
           "mofem_imex_adjoint_workspace_size", "mofem_imex_adjoint_step", "mofem_pcg_solve_async",
           "mofem_pcg_solve_many", "mofem_pcg_solve_grouped",
           "mofem_imex_graph_create", "mofem_imex_graph_launch", "mofem_imex_graph_result",
           "mofem_imex_graph_destroy", "mofem_trace_enable", "mofem_trace_select", "mofem_trace_read"]


class MofemError(RuntimeError):
    def __init__(self, code, where):
        msg = mofem_last_error().decode(errors="replace")
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


def _check(rc, where):
    if rc != OK:
        raise MofemError(rc, where)


def _hptr(a):
    return a.ctypes.data_as(_vp)


# ---- host entry points ---------------------------------------------------------
def weight(kind=W_ONE, p=(0.0, 0.0, 0.0, 0.0)):
    w = Weight()
    w.kind = kind
    for i, v in enumerate(p):
        w.p[i] = float(v)
    return w


def assemble_1d(order, m_elem, di, dj, w=None, x0=0.0, x1=1.0, nq=0):
    """DIA band (2kb+1, n) of int psi_i^(di) psi_j^(dj) w over [x0, x1]."""
    kb = max(order, 1)
    n = kb * m_elem + 1
    band = np.zeros((2 * kb + 1, n))
    rc = mofem_assemble_1d(order, m_elem, x0, x1, di, dj, ctypes.byref(w) if w is not None else None,
                           nq, _hptr(band))
    _check(rc, "mofem_assemble_1d")
    return band


def set_host_threads(n):
    """Host threads of one host-side call (0 restores the default); returns
    the previous count."""
    return int(mofem_set_host_threads(int(n)))


def geneig_host(K_band, M_band, trim):
    kb = (K_band.shape[0] - 1) // 2
    n = K_band.shape[1]
    q = n - 2 * trim
    lam = np.zeros(q)
    V = np.zeros((q, q))
    K = np.ascontiguousarray(K_band, dtype=np.float64)
    M = np.ascontiguousarray(M_band, dtype=np.float64)
    _check(mofem_geneig_host(n, kb, _hptr(K), _hptr(M), trim, _hptr(lam), _hptr(V)), "mofem_geneig_host")
    return lam, V


def eig_p1_closed(n_elem, length=1.0, lumped=False, dirichlet=True):
    """Closed-form (lam, V) of the uniform P1 pencil (mofem_eig_p1_closed)."""
    q = n_elem - 1 if dirichlet else n_elem + 1
    lam = np.zeros(max(q, 0))
    V = np.zeros((max(q, 0), max(q, 0)))
    _check(mofem_eig_p1_closed(n_elem, length, int(lumped), int(dirichlet), _hptr(lam), _hptr(V)),
           "mofem_eig_p1_closed")
    return lam, V


def band_to_dense(band):
    """Dense matrix of a DIA band (helper for tests and diagnostics)."""
    w, n = band.shape
    kb = (w - 1) // 2
    D = np.zeros((n, n))
    for d in range(w):
        i = np.arange(n)
        j = i + d - kb
        ok = (j >= 0) & (j < n)
        D[i[ok], j[ok]] = band[d, i[ok]]
    return D


# ---- device entry points (torch tensors) -----------------------------------------
def _torch():
    import torch
    return torch


def _dptr(t):
    if t is None:
        return None
    torch = _torch()
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype not in (torch.float64, torch.int32, torch.uint8):
        raise ValueError("expected float64 data")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return _vp(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


class Operator:
    """Y = sum_t c_t op(L_t) X op(R_t) (see mofem_op_desc)."""

    def __init__(self, terms, n_s, n_t, kb, trim_s=0, trim_t=0, full_input=False, elem_order=0,
                 full_output=False):
        if not 1 <= len(terms) <= MAX_TERMS:
            raise ValueError("an operator has 1..%d terms" % MAX_TERMS)
        d = OpDesc()
        d.kb, d.elem_order, d.n_s, d.n_t = kb, elem_order, n_s, n_t
        d.trim_s, d.trim_t, d.full_input, d.n_terms = trim_s, trim_t, int(full_input), len(terms)
        d.full_output = int(full_output)
        self._keep = []
        for i, t in enumerate(terms):
            L = np.ascontiguousarray(t["left"], dtype=np.float64)
            R = np.ascontiguousarray(t["right"], dtype=np.float64)
            self._keep += [L, R]
            d.left[i] = L.ctypes.data
            d.right[i] = R.ctypes.data
            d.left_transpose[i] = int(t.get("left_T", False))
            d.right_transpose[i] = int(t.get("right_T", False))
            d.coef[i] = float(t.get("coef", 1.0))
            d.scaled[i] = int(t.get("scaled", False))
        h = _vp()
        _check(mofem_op_create(ctypes.byref(d), ctypes.byref(h)), "mofem_op_create")
        self.handle = h
        self._keep = None
        qs, qt, i_s, i_t = (ctypes.c_int() for _ in range(4))
        _check(mofem_op_shape(h, ctypes.byref(qs), ctypes.byref(qt), ctypes.byref(i_s), ctypes.byref(i_t)),
               "mofem_op_shape")
        self.shape = (qs.value, qt.value)
        self.in_shape = (i_s.value, i_t.value)

    def __del__(self, _destroy=mofem_op_destroy):
        # the default argument keeps the entry point alive at interpreter exit
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    def apply(self, X, Y=None, item_scale=None, dot=False, stream=None, noalloc=False):
        """Y = L(X) per item (mofem_op_apply; with noalloc=True the
        allocation-free mofem_op_apply_noalloc, which needs Y given)."""
        torch = _torch()
        batch = X.shape[0]
        if tuple(X.shape[1:]) != self.in_shape:
            raise ValueError("input shape %s, operator expects %s" % (tuple(X.shape[1:]), self.in_shape))
        if Y is None:
            if noalloc:
                raise ValueError("noalloc apply needs its output Y (and dot buffer) from the caller")
            Y = torch.empty((batch,) + self.shape, dtype=torch.float64, device=X.device)
        if dot is True:
            dots = torch.empty(batch, dtype=torch.float64, device=X.device)
        else:
            dots = dot if dot is not False else None
        in_stride = self.in_shape[0] * self.in_shape[1]
        out_stride = self.shape[0] * self.shape[1]
        fn, name = (mofem_op_apply_noalloc, "mofem_op_apply_noalloc") if noalloc else (mofem_op_apply, "mofem_op_apply")
        rc = fn(self.handle, _dptr(X), in_stride, _dptr(Y), out_stride, batch, _dptr(item_scale), _dptr(dots),
                _stream(stream))
        _check(rc, name)
        return (Y, dots) if dots is not None else Y


class Preconditioner:
    """Spectral single-term preconditioner (see mofem_prec_desc)."""

    def __init__(self, Ks, Ms, Kt, Mt, coeffs, trim_s=0, trim_t=0, precision=PREC_F64, Ks_add=(), Kt_add=()):
        """Ks_add, Kt_add: lists of (band, coefficient) pairs the library adds
        to Ks and Kt before the eigen-decompositions."""
        d = PrecDesc()
        self._keep = [np.ascontiguousarray(a, dtype=np.float64) for a in (Ks, Ms, Kt, Mt)]
        d.kb = (self._keep[0].shape[0] - 1) // 2
        d.n_s, d.n_t = self._keep[0].shape[1], self._keep[2].shape[1]
        d.trim_s, d.trim_t = trim_s, trim_t
        d.Ks, d.Ms, d.Kt, d.Mt = (a.ctypes.data for a in self._keep)
        d.alpha, d.beta_s, d.beta_t, d.delta = (float(c) for c in coeffs)
        d.precision = precision
        for field, terms, ref in (("Ks_add", Ks_add, self._keep[0]), ("Kt_add", Kt_add, self._keep[2])):
            if len(terms) > MAX_BAND_SUM:
                raise ValueError("at most %d added bands" % MAX_BAND_SUM)
            bs = getattr(d, field)
            bs.n = len(terms)
            for i, (band, coef) in enumerate(terms):
                a = np.ascontiguousarray(band, dtype=np.float64)
                if a.shape != ref.shape:
                    raise ValueError("an added band must have the shape of the band it is added to")
                self._keep.append(a)
                bs.band[i] = a.ctypes.data
                bs.coef[i] = float(coef)
        h = _vp()
        _check(mofem_prec_setup(ctypes.byref(d), ctypes.byref(h)), "mofem_prec_setup")
        self.handle = h
        self._keep = None
        self.shape = (d.n_s - 2 * trim_s, d.n_t - 2 * trim_t)
        self.precision = precision

    def __del__(self, _destroy=mofem_prec_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None

    @classmethod
    def from_eigen(cls, lam, Vs, mu, Vt, coeffs, precision=PREC_F64):
        """The same preconditioner from given generalised eigenpairs
        (mofem_prec_setup_eig), e.g. eig_p1_closed's."""
        self = cls.__new__(cls)
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lam, Vs, mu, Vt)]
        qs, qt = arrs[0].size, arrs[2].size
        if arrs[1].shape != (qs, qs) or arrs[3].shape != (qt, qt):
            raise ValueError("eigenvector matrices must be q x q")
        h = _vp()
        a, bs, bt, d = (float(c) for c in coeffs)
        _check(mofem_prec_setup_eig(qs, qt, _hptr(arrs[0]), _hptr(arrs[1]), _hptr(arrs[2]), _hptr(arrs[3]),
                                    a, bs, bt, d, precision, ctypes.byref(h)), "mofem_prec_setup_eig")
        self.handle = h
        self.shape = (qs, qt)
        self.precision = precision
        return self

    def set_coeffs(self, alpha, beta_s, beta_t, delta):
        _check(mofem_prec_set_coeffs(self.handle, alpha, beta_s, beta_t, delta), "mofem_prec_set_coeffs")

    def tune(self, batch, stream=None):
        """Pick the transforms' block tile for this batch by timing (mofem_prec_tune)."""
        tile = ctypes.c_int()
        _check(mofem_prec_tune(self.handle, batch, ctypes.byref(tile), _stream(stream)), "mofem_prec_tune")
        return tile.value

    def set_tile(self, batch, tile):
        _check(mofem_prec_set_tile(self.handle, batch, tile), "mofem_prec_set_tile")

    def set_precision(self, precision):
        _check(mofem_prec_set_precision(self.handle, precision), "mofem_prec_set_precision")
        self.precision = precision

    def eigenvalues(self):
        lam, mu = np.zeros(self.shape[0]), np.zeros(self.shape[1])
        _check(mofem_prec_eigenvalues(self.handle, _hptr(lam), _hptr(mu)), "mofem_prec_eigenvalues")
        return lam, mu

    def workspace_size(self, batch):
        return int(mofem_prec_workspace_size(self.handle, batch))

    def apply(self, R, Z=None, item_scale=None, workspace=None, stream=None):
        torch = _torch()
        batch = R.shape[0]
        if Z is None:
            Z = torch.empty_like(R)
        ws = workspace
        if ws is None:
            ws = torch.empty(self.workspace_size(batch), dtype=torch.uint8, device=R.device)
        rc = mofem_prec_apply(self.handle, _dptr(R), _dptr(Z), self.shape[0] * self.shape[1], batch,
                              _dptr(item_scale),
                              _dptr(ws), ws.numel(), _stream(stream))
        _check(rc, "mofem_prec_apply")
        return Z


class BandedPreconditioner(Preconditioner):
    """Product preconditioner P_j(U) = S_j U T_j with S_j = a Ms + c_j bs Ks and
    T_j = a Mt + c_j bt Kt, applied by banded Cholesky solves
    (mofem_prec_setup_banded); FP64 only.  Each of Ks, Ms, Kt, Mt is a DIA band
    or a list of (band, coefficient) pairs whose sum the library forms (e.g.
    eq. (80)'s A + B2); Ms, Mt may be None when a == 0."""

    def __init__(self, Ks, Ms, Kt, Mt, a=0.0, bs=1.0, bt=1.0, scales=(1.0,), trim_s=0, trim_t=0):
        if not 1 <= len(scales) <= MAX_SCALES:
            raise ValueError("1..%d scales" % MAX_SCALES)
        d = BPrecDesc()
        self._keep = []

        def fill(dst, spec):
            terms = [] if spec is None else (list(spec) if isinstance(spec, (list, tuple)) else [(spec, 1.0)])
            if len(terms) > MAX_BAND_SUM:
                raise ValueError("at most %d bands in a sum" % MAX_BAND_SUM)
            dst.n = len(terms)
            for i, (band, coef) in enumerate(terms):
                arr = np.ascontiguousarray(band, dtype=np.float64)
                self._keep.append(arr)
                dst.band[i] = arr.ctypes.data
                dst.coef[i] = float(coef)
            return [np.asarray(b) for b, _ in terms]

        ks = fill(d.Ks, Ks)
        fill(d.Ms, Ms)
        kt = fill(d.Kt, Kt)
        fill(d.Mt, Mt)
        d.kb = (ks[0].shape[0] - 1) // 2
        d.n_s, d.n_t = ks[0].shape[1], kt[0].shape[1]
        d.trim_s, d.trim_t = trim_s, trim_t
        d.a, d.bs, d.bt = float(a), float(bs), float(bt)
        d.n_scales = len(scales)
        for j, c in enumerate(scales):
            d.scales[j] = float(c)
        h = _vp()
        _check(mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)), "mofem_prec_setup_banded")
        self._keep = None
        self.handle = h
        self.shape = (d.n_s - 2 * trim_s, d.n_t - 2 * trim_t)
        self.precision = PREC_F64
        self.scales = tuple(float(c) for c in scales)


def pcg_workspace(op, prec, batch, device="cuda"):
    torch = _torch()
    n = int(mofem_pcg_workspace_size(op.handle, prec.handle, batch))
    return torch.empty(n, dtype=torch.uint8, device=device)


def pcg_solve(op, prec, rhs, U, tol=1e-10, maxit=500, flags=0, item_scale=None, workspace=None,
              stream=None, raise_on_error=True):
    """Solve L(U_b) = rhs_b for every item; returns (iters, relres, rc)."""
    batch = rhs.shape[0]
    if workspace is None:
        workspace = pcg_workspace(op, prec, batch, rhs.device)
    iters = np.zeros(batch, dtype=np.int32)
    relres = np.zeros(batch)
    rc = mofem_pcg_solve(op.handle, prec.handle, _dptr(rhs), _dptr(U), op.shape[0] * op.shape[1], batch,
                         _dptr(item_scale), tol, maxit, flags, _dptr(workspace), workspace.numel(),
                         _hptr(iters), _hptr(relres), _stream(stream))
    if raise_on_error:
        _check(rc, "mofem_pcg_solve")
    return iters, relres, rc


def pcg_solve_async(op, prec, rhs, U, workspace, iters, status, relres, tol=1e-10, maxit=100, flags=0,
                    item_scale=None, stream=None):
    """Queue a solve of exactly `maxit` masked iterations with no host
    synchronisation; iters/status (int32) and relres (float64) are device
    tensors [batch] that receive the per-item results."""
    batch = rhs.shape[0]
    rc = mofem_pcg_solve_async(op.handle, prec.handle, _dptr(rhs), _dptr(U), op.shape[0] * op.shape[1], batch,
                               _dptr(item_scale), tol, maxit, flags, _dptr(workspace), workspace.numel(),
                               _dptr(iters), _dptr(status), _dptr(relres), _stream(stream))
    _check(rc, "mofem_pcg_solve_async")


def pcg_solve_many(groups, streams, raise_on_error=True, grouped=False):
    """Solve several batched systems of uneven shapes together
    (mofem_pcg_solve_many; with grouped=True mofem_pcg_solve_grouped, which
    fuses the groups of one shape into one batched solve and ignores the
    workspaces).

    groups: list of dicts with op, prec, rhs, U and optionally tol, maxit,
    flags, item_scale, workspace; streams: one torch.cuda.Stream per group
    (ordered after the current stream here).  Returns per group (iters,
    relres) and the per-group status list."""
    torch = _torch()
    n = len(groups)
    arr = (PcgGroup * n)()
    keep, outs = [], []
    cur = torch.cuda.current_stream()
    for i, g in enumerate(groups):
        op, prec, rhs, U = g["op"], g["prec"], g["rhs"], g["U"]
        batch = rhs.shape[0]
        ws = g.get("workspace")
        if ws is None:
            ws = torch.empty(1, dtype=torch.uint8, device=rhs.device) if grouped else \
                pcg_workspace(op, prec, batch, rhs.device)
        its = np.zeros(batch, dtype=np.int32)
        rr = np.zeros(batch)
        keep.append(ws)
        outs.append((its, rr))
        streams[i].wait_stream(cur)
        a = arr[i]
        a.op, a.prec, a.rhs, a.u = op.handle.value, prec.handle.value, rhs.data_ptr(), U.data_ptr()
        a.stride, a.batch = op.shape[0] * op.shape[1], batch
        a.item_scale = g["item_scale"].data_ptr() if g.get("item_scale") is not None else None
        a.tol, a.maxit, a.flags = g.get("tol", 1e-10), g.get("maxit", 500), g.get("flags", 0)
        a.workspace, a.ws_bytes = ws.data_ptr(), ws.numel()
        a.iters_out, a.relres_out = its.ctypes.data, rr.ctypes.data
    sarr = (_vp * max(n, 1))(*[_vp(st.cuda_stream) for st in streams])
    status = np.zeros(max(n, 1), dtype=np.int32)
    fn = mofem_pcg_solve_grouped if grouped else mofem_pcg_solve_many
    rc = fn(n, arr, sarr, _hptr(status))
    if raise_on_error:
        _check(rc, "mofem_pcg_solve_grouped" if grouped else "mofem_pcg_solve_many")
    for st in streams:
        cur.wait_stream(st)
    return outs, status[:n].tolist()


class ImexGraph:
    """One IMEX step captured as a HIP graph over a fixed state tensor
    (see mofem_imex_graph_create).  Runs on its own stream, ordered after
    and before the caller's current stream."""

    def __init__(self, stepper, state, batch, iters_per_step):
        torch = _torch()
        self.state, self.batch = state, batch
        self.workspace = stepper.workspace(batch, state.device)
        self.stream = torch.cuda.Stream(device=state.device)
        self._refs = stepper
        h = _vp()
        cur = torch.cuda.current_stream(state.device)
        self.stream.wait_stream(cur)
        q_s, q_t = state.shape[1], state.shape[2]
        rc = mofem_imex_graph_create(ctypes.byref(stepper.desc), _dptr(state), q_s * q_t, batch,
                                     _dptr(self.workspace), self.workspace.numel(), iters_per_step,
                                     ctypes.byref(h), ctypes.c_void_p(self.stream.cuda_stream))
        _check(rc, "mofem_imex_graph_create")
        self.handle = h
        cur.wait_stream(self.stream)

    def launch(self, nsteps=1):
        torch = _torch()
        cur = torch.cuda.current_stream(self.state.device)
        self.stream.wait_stream(cur)
        _check(mofem_imex_graph_launch(self.handle, nsteps, ctypes.c_void_p(self.stream.cuda_stream)),
               "mofem_imex_graph_launch")
        cur.wait_stream(self.stream)

    def result(self, raise_on_error=True):
        n = self.state.shape[0]
        iters = np.zeros(n, dtype=np.int32)
        status = np.zeros(n, dtype=np.int32)
        relres = np.zeros(n)
        rc = mofem_imex_graph_result(self.handle, _hptr(iters), _hptr(status), _hptr(relres),
                                     ctypes.c_void_p(self.stream.cuda_stream))
        if raise_on_error:
            _check(rc, "mofem_imex_graph_result")
        return iters, status, relres

    def __del__(self, _destroy=mofem_imex_graph_destroy):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            _destroy(self.handle)
            self.handle = None


def dot_accumulate(X, Y, out, alpha=1.0, beta=0.0, stream=None):
    """out[b] = beta out[b] + alpha <X_b, Y_b>_F for the leading batch dimension."""
    batch = X.shape[0]
    if Y.shape != X.shape or out.numel() < batch:
        raise ValueError("dot_accumulate: shapes")
    n = X[0].numel() if batch else 0
    _check(mofem_dot_accumulate(_dptr(X), _dptr(Y), n, n, batch, alpha, beta, _dptr(out), _stream(stream)),
           "mofem_dot_accumulate")
    return out


def trace_enable(on=True):
    _check(mofem_trace_enable(int(on)), "mofem_trace_enable")


def trace_select(classes=None):
    """Record only these trace classes (None: all)."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << c for c in classes)
    _check(mofem_trace_select(mask), "mofem_trace_select")


def trace_read(cls):
    """(total kernel milliseconds, launches, batch items) for one kernel class."""
    ms, n, items = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(mofem_trace_read(cls, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(items)), "mofem_trace_read")
    return ms.value, n.value, items.value


class Imex:
    """IMEX Euler stepper (see mofem_imex_desc)."""

    def __init__(self, op, prec, mass, tau, d, kinetics=KIN_NONE, kin=None, tol=1e-10, maxit=200, flags=0):
        self.desc = ImexDesc()
        self.desc.op, self.desc.prec, self.desc.mass = op.handle, prec.handle, mass.handle
        self.desc.tau = tau
        self.desc.n_species = len(d)
        for i, v in enumerate(d):
            self.desc.d[i] = v
        self.desc.kinetics = kinetics
        if kin is not None:
            for i, v in enumerate(kin):
                self.desc.kin[i] = v
        self.desc.tol, self.desc.maxit, self.desc.flags = tol, maxit, flags
        self._refs = (op, prec, mass)

    def workspace(self, batch, device="cuda"):
        torch = _torch()
        n = int(mofem_imex_workspace_size(ctypes.byref(self.desc), batch))
        return torch.empty(n, dtype=torch.uint8, device=device)

    def step(self, state, batch, workspace=None, stream=None):
        """state: tensor (n_species * batch, q_s, q_t), species major."""
        if workspace is None:
            workspace = self.workspace(batch, state.device)
        iters = np.zeros(state.shape[0], dtype=np.int32)
        q_s, q_t = state.shape[1], state.shape[2]
        rc = mofem_imex_step(ctypes.byref(self.desc), _dptr(state), q_s * q_t, batch,
                             _dptr(workspace), workspace.numel(), _hptr(iters), _stream(stream))
        _check(rc, "mofem_imex_step")
        return iters

    def adjoint_workspace(self, batch, device="cuda"):
        torch = _torch()
        n = int(mofem_imex_adjoint_workspace_size(ctypes.byref(self.desc), batch))
        return torch.empty(n, dtype=torch.uint8, device=device)

    def adjoint_step(self, stiff, state_n, state_np1, lam, grad_d, batch, workspace=None, stream=None):
        """Reverse step: lam (in dJ/dU^{n+1}, out dJ/dU^n) and grad_d
        (device [n_species * batch], accumulated) - see mofem_imex_adjoint_step."""
        if workspace is None:
            workspace = self.adjoint_workspace(batch, lam.device)
        iters = np.zeros(lam.shape[0], dtype=np.int32)
        q_s, q_t = lam.shape[1], lam.shape[2]
        rc = mofem_imex_adjoint_step(ctypes.byref(self.desc), stiff.handle, _dptr(state_n), _dptr(state_np1),
                                     _dptr(lam), _dptr(grad_d), q_s * q_t, batch, _dptr(workspace),
                                     workspace.numel(), _hptr(iters), _stream(stream))
        _check(rc, "mofem_imex_adjoint_step")
        return iters

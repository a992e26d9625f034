"""CPU tests of libmofem's host side: the shared library loads, exports every
symbol include/mofem.h declares, and its host-only entry points (1D assembly,
generalised eigen-decomposition, argument checking) agree with the oracle.
No GPU call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem1d
from workloads import L_profile, dL_profile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mofem.h")

mf = pytest.importorskip("paper_2109_01173_amd.mofem",
                         reason="libmofem.so not built (python -m paper_2109_01173_amd.build)")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mofem_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(mf.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mf.EXPORTS) == set(names)


PROF = (1.0, 0.3, np.pi, 0.0)


@pytest.mark.parametrize("order", [0, 1, 2, 3, 4])
def test_assembly_matches_oracle(order):
    k = max(order, 1)
    lumped = order == 0
    m = 7
    cases = [
        (1, 1, mf.W_PROFILE, PROF, L_profile),
        (1, 0, mf.W_PROFILE_D, PROF, dL_profile),
        (0, 0, mf.W_PROFILE_INV, PROF, lambda s: 1.0 / L_profile(s)),
        (0, 0, mf.W_PROFILE_D2L, PROF, lambda s: dL_profile(s) ** 2 / L_profile(s)),
        (0, 0, mf.W_ONE, (0, 0, 0, 0), None),
        (1, 1, mf.W_POLY, (0, 0, 1, 0), lambda t: t ** 2),
        (1, 0, mf.W_POLY, (0, 1, 0, 0), lambda t: t),
        # the cap profile L = 2 - s^2 (cubic-polynomial profile kinds)
        (1, 1, mf.W_POLY, (2, 0, -1, 0), lambda s: 2.0 - s ** 2),
        (1, 0, mf.W_PPROFILE_D, (2, 0, -1, 0), lambda s: -2.0 * s),
        (0, 0, mf.W_PPROFILE_INV, (2, 0, -1, 0), lambda s: 1.0 / (2.0 - s ** 2)),
        (0, 0, mf.W_PPROFILE_D2L, (2, 0, -1, 0), lambda s: 4.0 * s ** 2 / (2.0 - s ** 2)),
        (0, 0, mf.W_PPROFILE_D, (0.5, 1.0, -2.0, 3.0), lambda s: 1.0 - 4.0 * s + 9.0 * s ** 2),
    ]
    for di, dj, kind, p, fw in cases:
        w = None if kind == mf.W_ONE else mf.weight(kind, p)
        got = mf.band_to_dense(mf.assemble_1d(order, m, di, dj, w))
        ref = fem1d.assemble(k, m, di, dj, fw, lumped=lumped)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), (di, dj, kind)


def test_assembly_interval_and_callback():
    calls = []

    def f(x, ctx):
        calls.append(x)
        return 2.0 + x

    cb = mf.WeightFn(f)
    w = mf.Weight()
    w.kind = mf.W_CALLBACK
    w.fn = cb
    got = mf.band_to_dense(mf.assemble_1d(2, 3, 0, 0, w, x0=0.0, x1=20.0))
    ref = fem1d.assemble(2, 3, 0, 0, lambda x: 2.0 + x, x0=0.0, x1=20.0)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    assert len(calls) == 3 * 12


# sizes around the solver's blocking (blocks of 8 and 32 eigenvector entries,
# groups of four reflectors) and degenerate orders: q = 1, 2, 5, 256, 301, 209
@pytest.mark.parametrize("k,m,trim", [(1, 40, 1), (2, 30, 1), (3, 20, 0), (4, 15, 1), (1, 2, 1), (1, 3, 1),
                                      (1, 4, 0), (1, 257, 1), (2, 150, 0), (3, 70, 1)])
def test_geneig_matches_scipy(k, m, trim):
    K = mf.assemble_1d(k, m, 1, 1, mf.weight(mf.W_PROFILE, PROF))
    M = mf.assemble_1d(k, m, 0, 0, mf.weight(mf.W_PROFILE, PROF))
    lam, V = mf.geneig_host(K, M, trim)
    Kd, Md = mf.band_to_dense(K), mf.band_to_dense(M)
    if trim:
        Kd, Md = Kd[1:-1, 1:-1], Md[1:-1, 1:-1]
    lr = sla.eigh(Kd, Md, eigvals_only=True)
    assert np.abs(lam - lr).max() <= 1e-12 * np.abs(lr).max()
    assert np.abs(V.T @ Md @ V - np.eye(V.shape[0])).max() < 1e-12
    res = Kd @ V - Md @ V * lam
    assert np.linalg.norm(res) <= 1e-13 * np.linalg.norm(Kd, 2) * np.linalg.norm(V)


def test_geneig_independent_of_host_threads():
    """Every entry is computed by one thread in a fixed order, so the result
    does not depend on the thread count (mofem_set_host_threads)."""
    K = mf.assemble_1d(2, 150, 1, 1, mf.weight(mf.W_PROFILE, PROF))   # q = 299: the threaded path
    M = mf.assemble_1d(2, 150, 0, 0, mf.weight(mf.W_PROFILE, PROF))
    lam1, V1 = mf.geneig_host(K, M, 1)
    prev = mf.set_host_threads(1)
    try:
        assert mf.set_host_threads(3) == 1
        lam3, V3 = mf.geneig_host(K, M, 1)
        mf.set_host_threads(1)
        lam0, V0 = mf.geneig_host(K, M, 1)
    finally:
        mf.set_host_threads(0)
    assert prev >= 1
    assert np.array_equal(lam0, lam1) and np.array_equal(V0, V1)
    assert np.array_equal(lam3, lam1) and np.array_equal(V3, V1)


def test_geneig_rejects_indefinite_mass():
    K = mf.assemble_1d(1, 10, 1, 1)
    M = -mf.assemble_1d(1, 10, 0, 0)
    with pytest.raises(mf.MofemError) as e:
        mf.geneig_host(K, M, 1)
    assert e.value.code == mf.E_NUMERIC


def test_argument_errors_are_reported():
    band = np.zeros(100)
    p = band.ctypes.data_as(ctypes.c_void_p)
    assert mf.mofem_assemble_1d(5, 4, 0.0, 1.0, 0, 0, None, 0, p) == mf.E_ARG
    assert b"order" in mf.mofem_last_error()
    assert mf.mofem_assemble_1d(1, 0, 0.0, 1.0, 0, 0, None, 0, p) == mf.E_ARG
    assert mf.mofem_assemble_1d(1, 4, 1.0, 0.0, 0, 0, None, 0, p) == mf.E_ARG
    assert mf.mofem_assemble_1d(1, 4, 0.0, 1.0, 2, 0, None, 0, p) == mf.E_ARG
    assert mf.mofem_assemble_1d(1, 4, 0.0, 1.0, 0, 0, None, 40, p) == mf.E_ARG
    assert mf.mofem_assemble_1d(1, 4, 0.0, 1.0, 0, 0, None, 0, None) == mf.E_ARG
    # handle entry points reject NULL before touching the device
    assert mf.mofem_op_create(None, None) == mf.E_ARG
    assert mf.mofem_prec_setup(None, None) == mf.E_ARG
    assert mf.mofem_pcg_solve(None, None, None, None, 0, 1, None, 1e-8, 10, 0, None, 0, None, None,
                              None) == mf.E_ARG
    assert mf.mofem_op_apply(None, None, 0, None, 0, 1, None, None, None) == mf.E_ARG
    assert mf.mofem_version() >= 100


def test_banded_product_setup_errors_on_the_host():
    """mofem_prec_setup_banded factorises on the host before any device call:
    an indefinite factor (here -B1) is MOFEM_E_NUMERIC, bad counts E_ARG."""
    B1 = mf.assemble_1d(2, 8, 1, 1)
    A = mf.assemble_1d(2, 8, 1, 1)
    with pytest.raises(mf.MofemError) as e:
        mf.BandedPreconditioner(-B1, None, A, None, a=0.0, trim_s=1, trim_t=1)
    assert e.value.code == mf.E_NUMERIC
    d = mf.BPrecDesc()
    keep = [np.ascontiguousarray(B1), np.ascontiguousarray(A)]
    d.kb, d.n_s, d.n_t, d.trim_s, d.trim_t = 2, B1.shape[1], A.shape[1], 1, 1
    d.Ks.n, d.Ks.band[0], d.Ks.coef[0] = 1, keep[0].ctypes.data, 1.0
    d.Kt.n, d.Kt.band[0], d.Kt.coef[0] = 1, keep[1].ctypes.data, 1.0
    d.a, d.bs, d.bt = 0.0, 1.0, 1.0
    h = ctypes.c_void_p()
    for n_scales in (0, mf.MAX_SCALES + 1):
        d.n_scales = n_scales
        assert mf.mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
    d.n_scales, d.scales[0] = 1, 1.0
    d.a = 1.0  # a != 0 needs the mass bands
    assert mf.mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
    d.a = 0.0
    for bad in (-1, mf.MAX_BAND_SUM + 1):   # band sums of 0..MAX_BAND_SUM terms
        d.Kt.n = bad
        assert mf.mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
    d.Kt.n = 2                              # a NULL band inside the sum
    assert mf.mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
    d.Kt.n = 0                              # Kt needs at least one band
    assert mf.mofem_prec_setup_banded(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
    assert mf.mofem_prec_setup_banded(None, None) == mf.E_ARG


def test_spectral_setup_added_band_errors_on_the_host():
    """mofem_prec_setup's added bands (Ks_add, Kt_add: 0..MAX_BAND_SUM terms,
    no NULL band) are checked before any eigen-solve or device call; the
    binding rejects too many or misshapen added bands itself."""
    K = np.ascontiguousarray(mf.assemble_1d(2, 8, 1, 1))
    M = np.ascontiguousarray(mf.assemble_1d(2, 8, 0, 0))
    d = mf.PrecDesc()
    d.kb, d.n_s, d.n_t, d.trim_s, d.trim_t = 2, K.shape[1], K.shape[1], 1, 1
    d.Ks = d.Kt = K.ctypes.data
    d.Ms = d.Mt = M.ctypes.data
    d.alpha, d.beta_s, d.beta_t, d.delta, d.precision = 1.0, 1.0, 1.0, 0.0, mf.PREC_F64
    h = ctypes.c_void_p()
    for field in ("Ks_add", "Kt_add"):
        bs = getattr(d, field)
        for bad in (-1, mf.MAX_BAND_SUM + 1):
            bs.n = bad
            assert mf.mofem_prec_setup(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
        bs.n = 1                              # a NULL added band
        assert mf.mofem_prec_setup(ctypes.byref(d), ctypes.byref(h)) == mf.E_ARG
        assert b"added band" in mf.mofem_last_error()
        bs.n = 0
    with pytest.raises(ValueError):
        mf.Preconditioner(K, M, K, M, (1.0, 1.0, 1.0, 0.0), 1, 1, Kt_add=[(K, 1.0)] * (mf.MAX_BAND_SUM + 1))
    with pytest.raises(ValueError):
        mf.Preconditioner(K, M, K, M, (1.0, 1.0, 1.0, 0.0), 1, 1, Ks_add=[(K[:, :-1], 1.0)])


@pytest.mark.parametrize("lumped,dirichlet", [(False, True), (True, True), (True, False)])
def test_closed_form_p1_eigenpairs(lumped, dirichlet):
    """mofem_eig_p1_closed (Sec. 4.1) against a dense symmetric-definite
    eigen-solve of the assembled P1 pencil on [0, 2], N = 37."""
    N, length = 37, 2.0
    order = 0 if lumped else 1
    trim = 1 if dirichlet else 0
    K = mf.band_to_dense(mf.assemble_1d(order, N, 1, 1, None, 0.0, length))
    M = mf.band_to_dense(mf.assemble_1d(order, N, 0, 0, None, 0.0, length))
    if trim:
        K, M = K[1:-1, 1:-1], M[1:-1, 1:-1]
    lam, V = mf.eig_p1_closed(N, length, lumped, dirichlet)
    ref = sla.eigh(K, M, eigvals_only=True)
    assert np.allclose(lam, ref, rtol=1e-12, atol=1e-12 * ref.max())
    assert np.abs(V.T @ M @ V - np.eye(len(lam))).max() < 1e-12
    assert np.linalg.norm(K @ V - M @ V * lam) <= 1e-12 * np.linalg.norm(K) * np.linalg.norm(V)
    # the unit-interval stiffness eigenvalues of the corrected eq. (63): 2N(1 - cos(i pi / N))
    lamA = np.linalg.eigvalsh(mf.band_to_dense(mf.assemble_1d(1, N, 1, 1))[1:-1, 1:-1])
    i = np.arange(1, N)
    assert np.allclose(np.sort(lamA), 2 * N * (1 - np.cos(i * np.pi / N)), rtol=1e-12)


def test_closed_form_rejects_consistent_neumann():
    with pytest.raises(mf.MofemError) as e:
        mf.eig_p1_closed(16, 1.0, lumped=False, dirichlet=False)
    assert e.value.code == mf.E_UNSUPPORTED


def test_header_constants_match_binding():
    """Every MOFEM_PREC_* and MOFEM_TRACE_* value of include/mofem.h equals the
    binding's constant of the same name."""
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "mofem.h")).read()
    found = re.findall(r"MOFEM_((?:PREC|TRACE)_[A-Z0-9_]+)\s*=\s*(\d+)", hdr)
    assert len(found) >= 15
    for name, val in found:
        assert getattr(mf, name) == int(val), name

// Internal declarations shared by the libmofem translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

#include "../../include/mofem.h"

namespace mofem {

// ---- error handling -------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();
int fail(int code, const std::string& msg);

// ---- host threading ---------------------------------------------------------
// Run fn(begin, end) over [0, n) split into contiguous chunks on up to
// host_threads() threads (serially when n is small).
void parallel_for(long n, long min_chunk, const std::function<void(long, long)>& fn);
// threads of one host-side call: mofem_set_host_threads, or the hardware's
// (at most 16), or the calling thread's share (set_thread_share)
int host_threads();
// give the calling thread's host-side calls n threads (0: the process
// setting); returns the previous share
int set_thread_share(int n);

// ---- one-dimensional assembly (host_fem.cpp) --------------------------------
void gauss_legendre01(int nq, double* x, double* w);
void lagrange_equispaced(int k, double xi, double* val, double* der);
double eval_weight(const mofem_weight* w, double x);

// ---- dense eigen-solver (host_eigen.cpp) ------------------------------------
// Generalised symmetric-definite eigenproblem on dense row-major q x q
// matrices K, M (M SPD, banded with half-width kb used for the Cholesky).
// On success lam (ascending) and V (row-major, columns are eigenvectors with
// V^T M V = I).  Returns MOFEM_OK or MOFEM_E_NUMERIC.
int geneig_dense(int q, int kb, const double* K, const double* M, double* lam, double* V);

// Expand a DIA band (half-width kb, n rows) to a dense row-major matrix
// restricted to indices [t, n - t).
void band_to_dense(int n, int kb, const double* band, int trim, double* dense);

// ---- banded Cholesky (host_chol.cpp) ------------------------------------------
// S: q rows of 2 kb + 1 entries, S[i * (2 kb + 1) + kb + (j - i)] = S_ij, symmetric
// positive definite.  Writes Lf[i * (kb + 1) + l] = L[i][i - l] and
// Lb[i * (kb + 1) + l] = L[i + l][i] for l = 1..kb (0 outside the matrix), and
// 1 / L[i][i] at l = 0, where S = L L^T.  MOFEM_E_NUMERIC if S is not SPD.
int band_cholesky(int q, int kb, const double* S, double* Lf, double* Lb);

}  // namespace mofem

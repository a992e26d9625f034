// Banded Cholesky factorisation (host, FP64, once per preconditioner set-up).
//
// The paper's own preconditioners are products of two one-dimensional
// matrices, P(U) = S U T: eq. (80) with S = B1 and T = A + B2 for the
// elliptic problem, eq. (95) with S = M3 + c B1 and T = M + c (A + B2) per
// IMEX step.  S and T are symmetric positive definite and banded (half-width
// k for P_k), so P^{-1}(R) = S^{-1} R T^{-1} costs two banded triangular
// solves per dimension once S = L L^T and T are factorised.  The Cholesky
// factor of a band matrix keeps its half-width (no fill-in outside the band).
#include <cmath>
#include <vector>

#include "mofem_internal.h"

namespace mofem {

int band_cholesky(int q, int kb, const double* S, double* Lf, double* Lb) {
  const int w = 2 * kb + 1, c = kb + 1;
  // L[i][i - l] for l = 0..kb, row by row (column-oriented band storage)
  std::vector<double> L((size_t)q * c, 0.0);
  auto at = [&](int i, int j) -> double& { return L[(size_t)i * c + (i - j)]; };
  for (int i = 0; i < q; ++i) {
    const int j0 = i - kb < 0 ? 0 : i - kb;
    for (int j = j0; j <= i; ++j) {
      double sum = S[(size_t)i * w + kb + (j - i)];
      for (int m = j0; m < j; ++m) sum -= at(i, m) * at(j, m);  // m >= i - kb >= j - kb
      if (j == i) {
        if (!(sum > 0.0) || !std::isfinite(sum)) return MOFEM_E_NUMERIC;
        at(i, i) = std::sqrt(sum);
      } else {
        at(i, j) = sum / at(j, j);
      }
    }
  }
  for (int i = 0; i < q; ++i) {
    const double inv = 1.0 / at(i, i);
    Lf[(size_t)i * c] = inv;
    Lb[(size_t)i * c] = inv;
    for (int l = 1; l <= kb; ++l) {
      Lf[(size_t)i * c + l] = i - l >= 0 ? at(i, i - l) : 0.0;
      Lb[(size_t)i * c + l] = i + l < q ? at(i + l, i) : 0.0;
    }
  }
  return MOFEM_OK;
}

}  // namespace mofem

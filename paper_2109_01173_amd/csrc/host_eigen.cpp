// Generalised symmetric-definite eigen-decomposition on the host (FP64).
//
// The single-term preconditioner of Sec. 5 (eq. (80)) and Sec. 6 (eq. (95))
// is applied in the spectral form of Sec. 4 (eqs. (55)-(59)), which needs,
// once per geometry, the pencils (K, M) of the s and t directions
// diagonalised:  K V = M V diag(lam),  V^T M V = I.
//
// Method (textbook dense linear algebra, written out here):
//   1. banded Cholesky  M = L L^T  (L lower, half-width kb);
//   2. C = L^{-1} K L^{-T}  by banded forward substitution on rows;
//   3. Householder reduction of C to tridiagonal T = Q^T C Q;
//   4. implicit QL iteration with Wilkinson-type shifts on T; the Givens
//      rotations are recorded and then applied to the eigenvector matrix
//      in parallel over column blocks;
//   5. eigenvectors of C: Q z (reflectors applied in reverse order);
//   6. V = L^{-T} (Q z)  by banded back substitution;
//   7. ascending sort.
// Threads: steps 2, 3, 4-apply, 5 and 6 split rows/columns over the host
// threads; step 3 uses a spin barrier between its phases.
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <vector>

#include "mofem_internal.h"

namespace mofem {

namespace {

struct SpinBarrier {
  explicit SpinBarrier(int n) : n_(n), count_(0), gen_(0) {}
  void wait() {
    int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_acq_rel);
      return;
    }
    int spins = 0;
    while (gen_.load(std::memory_order_acquire) == g) {
      if (++spins > 256) std::this_thread::yield();
    }
  }
  int n_;
  std::atomic<int> count_;
  std::atomic<int> gen_;
};

int team_size() {
  cpu_set_t set;
  int n = 0;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(n, host_threads()));
}

void run_team(int nt, const std::function<void(int, int)>& body) {
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back([&body, t, nt] { body(t, nt); });
  body(0, nt);
  for (auto& x : th) x.join();
}

inline void split(long n, int t, int nt, long* b, long* e) {
  long chunk = (n + nt - 1) / nt;
  *b = std::min(n, (long)t * chunk);
  *e = std::min(n, *b + chunk);
}

// Householder tridiagonalisation of the symmetric q x q row-major matrix A
// (full storage, overwritten).  On exit d, e hold T (e[i] = T[i][i+1]) and
// the reflector vectors sit in A[k+1.., k] with factors tau[k].
void tridiagonalise(int q, double* A, double* d, double* e, double* tau) {
  int nt = q >= 256 ? team_size() : 1;
  std::vector<double> v(q), p(q), w(q);
  SpinBarrier bar(nt);
  // shared scalars for the current step
  double alpha = 0.0, t_k = 0.0;
  auto make_reflector = [&](int k) {
    // x = A[k+1 .. q-1][k]
    int r = q - k - 1;
    double xnorm2 = 0.0;
    for (int i = 1; i < r; ++i) {
      double xi = A[(size_t)(k + 1 + i) * q + k];
      xnorm2 += xi * xi;
    }
    double x0 = A[(size_t)(k + 1) * q + k];
    if (xnorm2 == 0.0) {
      alpha = x0;
      t_k = 0.0;
      return;
    }
    double nrm = std::sqrt(x0 * x0 + xnorm2);
    alpha = x0 >= 0.0 ? -nrm : nrm;
    // v = x - alpha e1, scaled so that v[0] = 1
    double v0 = x0 - alpha;
    v[0] = 1.0;
    for (int i = 1; i < r; ++i) v[i] = A[(size_t)(k + 1 + i) * q + k] / v0;
    double vtv = 1.0 + xnorm2 / (v0 * v0);
    t_k = 2.0 / vtv;
  };
  run_team(nt, [&](int tid, int nth) {
    for (int k = 0; k + 2 < q; ++k) {
      int r = q - k - 1;
      if (tid == 0) make_reflector(k);
      bar.wait();
      if (t_k == 0.0) {
        if (tid == 0) {
          d[k] = A[(size_t)k * q + k];
          e[k] = alpha;
          tau[k] = 0.0;
          for (int i = 0; i < r; ++i) A[(size_t)(k + 1 + i) * q + k] = 0.0;
        }
        bar.wait();
        continue;
      }
      // p = tau * B v over the rows this thread owns
      long b, en;
      split(r, tid, nth, &b, &en);
      for (long i = b; i < en; ++i) {
        const double* row = A + (size_t)(k + 1 + i) * q + (k + 1);
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += row[j] * v[j];
        p[i] = t_k * s;
      }
      bar.wait();
      if (tid == 0) {
        double ptv = 0.0;
        for (int i = 0; i < r; ++i) ptv += p[i] * v[i];
        double K = 0.5 * t_k * ptv;
        for (int i = 0; i < r; ++i) w[i] = p[i] - K * v[i];
      }
      bar.wait();
      for (long i = b; i < en; ++i) {
        double* row = A + (size_t)(k + 1 + i) * q + (k + 1);
        double vi = v[i], wi = w[i];
        for (int j = 0; j < r; ++j) row[j] -= vi * w[j] + wi * v[j];
      }
      bar.wait();
      if (tid == 0) {
        d[k] = A[(size_t)k * q + k];
        e[k] = alpha;
        tau[k] = t_k;
        for (int i = 0; i < r; ++i) A[(size_t)(k + 1 + i) * q + k] = v[i];
      }
      bar.wait();
    }
  });
  if (q >= 2) {
    d[q - 2] = A[(size_t)(q - 2) * q + (q - 2)];
    e[q - 2] = A[(size_t)(q - 1) * q + (q - 2)];
  }
  d[q - 1] = A[(size_t)(q - 1) * q + (q - 1)];
  if (q >= 1) e[q - 1] = 0.0;
  if (q >= 2) tau[q - 2] = 0.0;
  if (q >= 1) tau[q - 1] = 0.0;
}

struct Rot {
  int i;
  double c, s;
};

// Implicit QL on the tridiagonal (d, e); appends every Givens rotation
// (acting on eigenvector-matrix rows i, i+1) to `rots`.  Returns false if an
// eigenvalue needs more than 60 sweeps.  The sweep is the published implicit
// QL algorithm with Wilkinson-type shifts (Bowdler, Martin, Reinsch and
// Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer. Math.
// 11 (1968), as distributed in EISPACK's tql2), so its step order follows that
// algorithm.
bool ql_implicit(int n, double* d, double* e, std::vector<Rot>& rots) {
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      if (++iter > 60) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool early = false;
      for (int i = m - 1; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        rots.push_back({i, c, s});
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

}  // namespace

int geneig_dense(int q, int kb, const double* K, const double* M, double* lam, double* V) {
  if (q <= 0) return MOFEM_E_ARG;
  // 1. banded Cholesky of M: Lb[i*(kb+1) + (j - i + kb)] = L[i][j], j in [i-kb, i]
  std::vector<double> Lb((size_t)q * (kb + 1), 0.0);
  auto Lat = [&](int i, int j) -> double& { return Lb[(size_t)i * (kb + 1) + (j - i + kb)]; };
  for (int i = 0; i < q; ++i) {
    for (int j = std::max(0, i - kb); j <= i; ++j) {
      double s = M[(size_t)i * q + j];
      for (int p = std::max(0, i - kb); p < j; ++p) s -= Lat(i, p) * Lat(j, p);
      if (i == j) {
        if (!(s > 0.0)) return MOFEM_E_NUMERIC;
        Lat(i, i) = std::sqrt(s);
      } else {
        Lat(i, j) = s / Lat(j, j);
      }
    }
  }
  // 2. W = L^{-1} K (row substitution, columns in parallel); C = L^{-1} W^T
  std::vector<double> W((size_t)q * q), C((size_t)q * q);
  auto forward_rows = [&](const double* src, double* dst) {
    parallel_for(q, 64, [&](long c0, long c1) {
      for (int i = 0; i < q; ++i) {
        double* di = dst + (size_t)i * q;
        const double* si = src + (size_t)i * q;
        for (long c = c0; c < c1; ++c) di[c] = si[c];
        for (int p = std::max(0, i - kb); p < i; ++p) {
          double l = Lat(i, p);
          const double* dp = dst + (size_t)p * q;
          for (long c = c0; c < c1; ++c) di[c] -= l * dp[c];
        }
        double inv = 1.0 / Lat(i, i);
        for (long c = c0; c < c1; ++c) di[c] *= inv;
      }
    });
  };
  forward_rows(K, W.data());
  // transpose W into C's storage temporarily, then substitute into W's storage
  parallel_for(q, 16, [&](long r0, long r1) {
    for (long i = r0; i < r1; ++i)
      for (int j = 0; j < q; ++j) C[(size_t)i * q + j] = W[(size_t)j * q + i];
  });
  forward_rows(C.data(), W.data());
  // symmetrise into C
  parallel_for(q, 16, [&](long r0, long r1) {
    for (long i = r0; i < r1; ++i)
      for (int j = 0; j < q; ++j) C[(size_t)i * q + j] = 0.5 * (W[(size_t)i * q + j] + W[(size_t)j * q + i]);
  });
  W.clear();
  W.shrink_to_fit();

  // 3. tridiagonalise
  std::vector<double> d(q), e(q), tau(q);
  tridiagonalise(q, C.data(), d.data(), e.data(), tau.data());

  // 4. QL with recorded rotations; Z rows = eigenvectors of T (starts as I)
  std::vector<Rot> rots;
  rots.reserve((size_t)q * 8);
  if (!ql_implicit(q, d.data(), e.data(), rots)) return MOFEM_E_NUMERIC;
  std::vector<double> Z((size_t)q * q, 0.0);
  for (int i = 0; i < q; ++i) Z[(size_t)i * q + i] = 1.0;
  // rotation (i, c, s) acts on rows i, i+1 of Z:
  //   f = Z[i+1]; Z[i+1] = s Z[i] + c f; Z[i] = c Z[i] - s f
  // (row j of Z is the j-th eigenvector of T written in the basis of e_c)
  parallel_for(q, 32, [&](long c0, long c1) {
    for (const Rot& R : rots) {
      double* zi = Z.data() + (size_t)R.i * q;
      double* zj = zi + q;
      for (long c = c0; c < c1; ++c) {
        double f = zj[c];
        zj[c] = R.s * zi[c] + R.c * f;
        zi[c] = R.c * zi[c] - R.s * f;
      }
    }
  });
  rots.clear();
  rots.shrink_to_fit();
  // Row j of Z is eigenvector j of T (the rotations act on eigenvector pairs).
  std::vector<double>& Y = Z;

  // 5 + 6. apply reflectors H_{q-3} .. H_0, then solve L^T v = x, per eigenvector
  parallel_for(q, 8, [&](long j0, long j1) {
    std::vector<double> x(q);
    for (long j = j0; j < j1; ++j) {
      double* y = Y.data() + (size_t)j * q;
      for (int k = q - 3; k >= 0; --k) {
        if (tau[k] == 0.0) continue;
        // v stored in C[k+1 .., k]
        double s = 0.0;
        for (int i = k + 1; i < q; ++i) s += C[(size_t)i * q + k] * y[i];
        s *= tau[k];
        for (int i = k + 1; i < q; ++i) y[i] -= s * C[(size_t)i * q + k];
      }
      for (int i = q - 1; i >= 0; --i) {
        double s = y[i];
        for (int p = i + 1; p <= std::min(q - 1, i + kb); ++p) s -= Lat(p, i) * y[p];
        y[i] = s / Lat(i, i);
      }
    }
  });

  // 7. ascending order, V[i][j] = eigenvector j component i
  std::vector<int> order(q);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  for (int j = 0; j < q; ++j) {
    lam[j] = d[order[j]];
    if (!std::isfinite(lam[j])) return MOFEM_E_NUMERIC;
  }
  parallel_for(q, 16, [&](long r0, long r1) {
    for (long i = r0; i < r1; ++i)
      for (int j = 0; j < q; ++j) V[(size_t)i * q + j] = Y[(size_t)order[j] * q + i];
  });
  return MOFEM_OK;
}

}  // namespace mofem

using namespace mofem;

extern "C" int mofem_geneig_host(int n, int kb, const double* K, const double* M, int trim,
                                 double* lam, double* V) {
  clear_error();
  if (n < 1 || kb < 1 || kb > 4 || (trim != 0 && trim != 1) || n - 2 * trim < 1)
    return fail(MOFEM_E_ARG, "geneig_host: bad n/kb/trim");
  if (!K || !M || !lam || !V) return fail(MOFEM_E_ARG, "geneig_host: NULL pointer");
  int q = n - 2 * trim;
  std::vector<double> Kd((size_t)q * q), Md((size_t)q * q);
  band_to_dense(n, kb, K, trim, Kd.data());
  band_to_dense(n, kb, M, trim, Md.data());
  int rc = geneig_dense(q, kb, Kd.data(), Md.data(), lam, V);
  if (rc != MOFEM_OK) return fail(rc, "geneig_host: mass matrix not positive definite or QL did not converge");
  return MOFEM_OK;
}

// Closed-form generalised eigenpairs of uniform P1 pencils (A, M) on an
// interval of length `len` with N elements, h = len / N (Sec. 4.1: with
// Dirichlet conditions A and the consistent M are tridiagonal Toeplitz
// matrices, M = alpha A + beta I, eq. (60), so both are diagonalised by the
// sine vectors of eq. (64); their eigenvalues follow eqs. (63) and (65)).
//   Dirichlet (q = N - 1), v_i[j] = sin(i j pi / N), i, j = 1..N-1:
//     A v_i = (2 / h)(1 - cos(i pi / N)) v_i,
//     M v_i = (h / 3)(2 + cos(i pi / N)) v_i   (consistent)
//             h v_i                             (lumped: trapezoid mass h I)
//   Neumann, lumped only (q = N + 1), w_i[j] = cos(i j pi / N), i, j = 0..N:
//     A w_i = (2 / h^2)(1 - cos(i pi / N)) M0 w_i,  M0 = h diag(1/2, 1, .., 1, 1/2).
// The vectors are scaled to V^T M V = I and sorted by ascending eigenvalue
// (ascending i).
extern "C" int mofem_eig_p1_closed(int n_elem, double len, int lumped, int dirichlet, double* lam, double* V) {
  clear_error();
  if (n_elem < 2 || !(len > 0.0) || !lam || !V) return fail(MOFEM_E_ARG, "eig_p1_closed: bad n_elem/len/pointers");
  if (!dirichlet && !lumped)
    return fail(MOFEM_E_UNSUPPORTED, "eig_p1_closed: consistent mass with Neumann conditions has no closed form");
  const int N = n_elem;
  const double h = len / N, pi = 3.14159265358979323846;
  if (dirichlet) {
    const int q = N - 1;
    for (int i = 1; i <= q; ++i) {
      const double c = std::cos(i * pi / N);
      const double la = 2.0 / h * (1.0 - c);
      const double mu = lumped ? h : h / 3.0 * (2.0 + c);
      lam[i - 1] = la / mu;
      const double scale = 1.0 / std::sqrt(mu * 0.5 * N);  // sum_j sin^2 = N / 2
      for (int j = 1; j <= q; ++j) V[(size_t)(j - 1) * q + (i - 1)] = scale * std::sin((double)i * j * pi / N);
    }
  } else {
    const int q = N + 1;
    for (int i = 0; i <= N; ++i) {
      lam[i] = 2.0 / (h * h) * (1.0 - std::cos(i * pi / N));
      // sum_j D_j cos^2 = N / 2 (0 < i < N) or N (i = 0, N)
      const double scale = 1.0 / std::sqrt(h * ((i == 0 || i == N) ? N : 0.5 * N));
      for (int j = 0; j <= N; ++j) V[(size_t)j * q + i] = scale * std::cos((double)i * j * pi / N);
    }
  }
  return MOFEM_OK;
}

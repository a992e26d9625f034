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
//      in parallel over column blocks, one sweep at a time;
//   5. eigenvectors of C: Q z (reflectors applied in reverse order, to
//      blocks of eight eigenvectors at a time);
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
// (its lower triangle is read and updated; the upper one goes stale).  On
// exit d, e hold T (e[i] = T[i][i+1]) and the reflector vectors sit in
// A[k+1.., k] with factors tau[k].
// Step k reflects column k of the trailing matrix (rows and columns k+1..):
// p = tau A v, w = p - (tau / 2)(p . v) v, A -= v w^T + w v^T.  The rank-2
// update of step k and the product p of step k+1 share one pass over the
// lower triangle: the next reflector comes from the updated column k+1,
// which is formed first; every updated entry a_ij (j < i) then adds a_ij v'_j
// to row i's own p' entry and a_ij v'_i to its row chunk's partial array for
// p'_j (the chunks' partials are then summed in chunk order).  The rows are
// cut into NCH chunks of about equal triangle area, dealt to the threads in
// turn: the arithmetic does not depend on the thread count.
void tridiagonalise(int q, double* A, double* d, double* e, double* tau) {
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * q + j]; };
  if (q <= 2) {
    d[0] = at(0, 0);
    e[0] = 0.0;
    tau[0] = 0.0;
    if (q == 2) {
      d[1] = at(1, 1);
      e[0] = at(1, 0);
      e[1] = 0.0;
      tau[1] = 0.0;
    }
    return;
  }
  const int nt = q >= 256 ? team_size() : 1;
  constexpr int NCH = 64;
  std::vector<double> v(q, 0.0), vn(q, 0.0), w(q, 0.0), p(q, 0.0);
  std::vector<double> part((size_t)NCH * q, 0.0);
  SpinBarrier bar(nt);
  double alpha = 0.0, tk = 0.0, alpha_n = 0.0, tk_n = 0.0;
  // reflector I - t u u^T (u[c+1] = 1) mapping A[c+1 .., c] to al e_1; u holds
  // absolute indices c+1 .. q-1
  auto reflector = [&](int c, std::vector<double>& u, double* al, double* t) {
    const double x0 = at(c + 1, c);
    double xnorm2 = 0.0;
    for (int i = c + 2; i < q; ++i) xnorm2 += at(i, c) * at(i, c);
    u[c + 1] = 1.0;
    if (xnorm2 == 0.0) {
      *al = x0;
      *t = 0.0;
      for (int i = c + 2; i < q; ++i) u[i] = 0.0;
      return;
    }
    const double nrm = std::sqrt(x0 * x0 + xnorm2);
    *al = x0 >= 0.0 ? -nrm : nrm;
    const double u0 = x0 - *al;
    for (int i = c + 2; i < q; ++i) u[i] = at(i, c) / u0;
    *t = 2.0 / (1.0 + xnorm2 / (u0 * u0));
  };
  // rows [lo, q) split into nth ranges of about equal lower-triangle area
  auto rows_of = [&](int lo, int t, int nth, int* b, int* en) {
    const double m = q - lo, total = m * (m + 1.0) / 2.0;
    auto first = [&](int tt) {
      if (tt <= 0) return lo;
      if (tt >= nth) return q;
      const double a = total * tt / nth;
      const int r = (int)std::ceil((std::sqrt(8.0 * a + 1.0) - 1.0) / 2.0);
      return std::min(q, lo + r);
    };
    *b = first(t);
    *en = first(t + 1);
  };
  // p[i] = t (p[i] + sum over the chunks of part[c][i]) for i in [lo, q)
  auto reduce_p = [&](int lo, double t, int tid, int nth) {
    long b, en;
    split(q - lo, tid, nth, &b, &en);
    for (long ii = b; ii < en; ++ii) {
      const int i = lo + (int)ii;
      double s = p[i];
      for (int c = 0; c < NCH; ++c) s += part[(size_t)c * q + i];
      p[i] = t * s;
    }
  };
  run_team(nt, [&](int tid, int nth) {
    // step 0: reflector of column 0 and p = tau A v over rows/columns 1..
    if (tid == 0) reflector(0, v, &alpha, &tk);
    bar.wait();
    for (int c = tid; c < NCH; c += nth) {
      double* pt = part.data() + (size_t)c * q;
      int b, en;
      rows_of(1, c, NCH, &b, &en);
      std::fill(pt, pt + q, 0.0);
      for (int i = b; i < en; ++i) {
        const double* row = A + (size_t)i * q;
        const double vi = v[i];
        double sacc = 0.0;
        for (int j = 1; j < i; ++j) {
          sacc += row[j] * v[j];
          pt[j] += row[j] * vi;
        }
        p[i] = sacc + row[i] * vi;
      }
    }
    bar.wait();
    reduce_p(1, tk, tid, nth);
    bar.wait();
    for (int k = 0; k + 2 < q; ++k) {
      const bool next = k + 3 < q;  // a reflector follows this step
      if (tid == 0) {
        if (k > 0) {
          std::swap(v, vn);
          alpha = alpha_n;
          tk = tk_n;
        }
        double ptv = 0.0;
        for (int i = k + 1; i < q; ++i) ptv += p[i] * v[i];
        const double K = 0.5 * tk * ptv;
        for (int i = k + 1; i < q; ++i) w[i] = p[i] - K * v[i];
        d[k] = at(k, k);
        e[k] = alpha;
        tau[k] = tk;
        for (int i = k + 1; i < q; ++i) at(i, k) = v[i];
        // column k+1 of the updated trailing matrix, diagonal included
        for (int i = k + 1; i < q; ++i) at(i, k + 1) -= v[i] * w[k + 1] + w[i] * v[k + 1];
        if (next) reflector(k + 1, vn, &alpha_n, &tk_n);
      }
      bar.wait();
      // rows k+2.., columns k+2 .. i: the update, and the next product
      for (int c = tid; c < NCH; c += nth) {
        double* pt = part.data() + (size_t)c * q;
        int b, en;
        rows_of(k + 2, c, NCH, &b, &en);
        if (next) std::fill(pt + k + 2, pt + q, 0.0);
        for (int i = b; i < en; ++i) {
          double* row = A + (size_t)i * q;
          const double vi = v[i], wi = w[i];
          if (next) {
            const double vni = vn[i];
            double sacc = 0.0;
            for (int j = k + 2; j < i; ++j) {
              const double a = row[j] - (vi * w[j] + wi * v[j]);
              row[j] = a;
              sacc += a * vn[j];
              pt[j] += a * vni;
            }
            const double a = row[i] - (vi * wi + wi * vi);
            row[i] = a;
            p[i] = sacc + a * vni;
          } else {
            for (int j = k + 2; j <= i; ++j) row[j] -= vi * w[j] + wi * v[j];
          }
        }
      }
      bar.wait();
      if (next) {
        reduce_p(k + 2, tk_n, tid, nth);
        bar.wait();
      }
    }
  });
  d[q - 2] = at(q - 2, q - 2);
  e[q - 2] = at(q - 1, q - 2);
  d[q - 1] = at(q - 1, q - 1);
  e[q - 1] = 0.0;
  tau[q - 2] = 0.0;
  tau[q - 1] = 0.0;
}

struct Rot {
  int i;
  double c, s;
};

// Implicit QL on the tridiagonal (d, e); appends every Givens rotation
// (acting on eigenvector-matrix rows i, i+1) to `rots` and the index of each
// sweep's first rotation to `sweeps`.  Returns false if an
// eigenvalue needs more than 60 sweeps.  The sweep is the published implicit
// QL algorithm with Wilkinson-type shifts (Bowdler, Martin, Reinsch and
// Wilkinson, "The QR and QL algorithms for symmetric matrices", Numer. Math.
// 11 (1968), as distributed in EISPACK's tql2), so its step order follows that
// algorithm.
bool ql_implicit(int n, double* d, double* e, std::vector<Rot>& rots, std::vector<size_t>& sweeps) {
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
      sweeps.push_back(rots.size());  // a sweep's rotations act on rows m-1, m-2, .. in turn
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

  // 4. QL with recorded rotations; Z rows = eigenvectors of T (starts as I).
  // Z is padded to whole blocks of NB rows and NR columns (zeros stay zeros).
  std::vector<Rot> rots;
  std::vector<size_t> sweeps;
  rots.reserve((size_t)q * 8);
  if (!ql_implicit(q, d.data(), e.data(), rots, sweeps)) return MOFEM_E_NUMERIC;
  sweeps.push_back(rots.size());
  constexpr int NR = 32, NB = 8;
  const long ldz = (q + NR - 1) / NR * NR;
  const long rows = (q + NB - 1) / NB * NB;
  std::vector<double> Z((size_t)rows * ldz, 0.0);
  for (int i = 0; i < q; ++i) Z[(size_t)i * ldz + i] = 1.0;
  // (c, s) of every rotation, sweep by sweep (row indices implied)
  std::vector<double> cs(2 * rots.size() + 2);
  for (size_t r = 0; r < rots.size(); ++r) {
    cs[2 * r] = rots[r].c;
    cs[2 * r + 1] = rots[r].s;
  }
  // rotation (i, c, s) acts on rows i, i+1 of Z:
  //   f = Z[i+1]; Z[i+1] = s Z[i] + c f; Z[i] = c Z[i] - s f.
  // Within a sweep the next rotation acts on rows i-1, i, so the new row i is
  // carried in registers: one load and one store per rotation and column.
  // Columns in blocks of NR (a block of Z stays in cache while the rotation
  // list streams past), blocks in parallel.
  parallel_for(ldz / NR, 1, [&](long b0, long b1) {
    for (long cb = b0; cb < b1; ++cb) {
      double* zc = Z.data() + cb * NR;
      for (size_t w = 0; w + 1 < sweeps.size(); ++w) {
        const size_t r0 = sweeps[w], r1 = sweeps[w + 1];
        if (r0 == r1) continue;
        const int top = rots[r0].i + 1;
        double carry[NR];
        const double* zt = zc + (size_t)top * ldz;
        for (int c = 0; c < NR; ++c) carry[c] = zt[c];
        const double* rc = cs.data() + 2 * r0;
        int i = top - 1;
        for (size_t r = r0; r < r1; ++r, --i, rc += 2) {
          const double co = rc[0], si = rc[1];
          const double* __restrict__ zi = zc + (size_t)i * ldz;
          double* __restrict__ zj = zc + (size_t)(i + 1) * ldz;
          for (int c = 0; c < NR; ++c) {
            const double x = zi[c], f = carry[c];
            zj[c] = si * x + co * f;
            carry[c] = co * x - si * f;
          }
        }
        double* zb = zc + (size_t)(i + 1) * ldz;
        for (int c = 0; c < NR; ++c) zb[c] = carry[c];
      }
    }
  });
  rots.clear();
  rots.shrink_to_fit();
  cs.clear();
  cs.shrink_to_fit();
  // Row j of Z is eigenvector j of T (the rotations act on eigenvector pairs).
  std::vector<double>& Y = Z;

  // 5. reflector k (k = 0 .. q-3) packed contiguously: v_k = C[k+1 .., k]
  std::vector<size_t> off(q > 2 ? q - 2 : 1);
  size_t tot = 0;
  for (int k = 0; k + 2 < q; ++k) {
    off[k] = tot;
    tot += (size_t)(q - k - 1);
  }
  std::vector<double> Vr(tot > 0 ? tot : 1);
  parallel_for(q > 2 ? q - 2 : 0, 16, [&](long k0, long k1) {
    for (long k = k0; k < k1; ++k)
      for (int i = 0; i < q - k - 1; ++i) Vr[off[k] + i] = C[(size_t)(k + 1 + i) * q + k];
  });
  C.clear();
  C.shrink_to_fit();
  // Reflectors are applied GR at a time (k = k1, k1 - 1, .., k1 - GR + 1):
  // with d_j = v_j^T y (one pass over y for the whole group) the factors of
  // the successive reflections are s_k1 = tau_k1 d_k1 and
  //   s_j = tau_j (d_j - sum_{i > j in the group} (v_j^T v_i) s_i),
  // and y -= sum_j s_j v_j (a second pass): two passes over y per group
  // instead of two per reflector.  The Gram entries v_j^T v_i are shared by
  // every block of eigenvectors.
  constexpr int GR = 4;
  const int nref = q > 2 ? q - 2 : 0;
  const int ngroups = (nref + GR - 1) / GR;
  auto vat = [&](int j, int i) { return i >= j + 1 ? Vr[off[j] + (i - j - 1)] : 0.0; };
  // group g holds k1 = nref - 1 - g GR down to max(0, k1 - GR + 1)
  std::vector<double> gram((size_t)ngroups * GR * GR, 0.0);
  parallel_for(ngroups, 8, [&](long g0, long g1) {
    for (long g = g0; g < g1; ++g) {
      const int k1 = nref - 1 - (int)g * GR;
      for (int a = 0; a < GR; ++a)
        for (int b = 0; b < a; ++b) {
          const int ja = k1 - a, jb = k1 - b;  // ja < jb
          if (ja < 0) continue;
          double acc = 0.0;
          for (int i = jb + 1; i < q; ++i) acc += vat(ja, i) * vat(jb, i);
          gram[((size_t)g * GR + a) * GR + b] = acc;
        }
    }
  });
  // 5 + 6. per block of NB eigenvectors, interleaved (entry i of the block's
  // vectors contiguous): apply H_{q-3} .. H_0, then solve L^T v = x for each
  parallel_for(rows / NB, 1, [&](long b0, long b1) {
    std::vector<double> yt((size_t)q * NB);
    for (long jb = b0; jb < b1; ++jb) {
      double* yb = Y.data() + (size_t)jb * NB * ldz;
      for (int t = 0; t < NB; ++t)
        for (int i = 0; i < q; ++i) yt[(size_t)i * NB + t] = yb[(size_t)t * ldz + i];
      for (int g = 0; g < ngroups; ++g) {
        const int k1 = nref - 1 - g * GR;
        const int ng = std::min(GR, k1 + 1);  // reflectors k1 .. k1 - ng + 1
        const int kl = k1 - ng + 1;
        double d[GR][NB] = {};
        // head rows kl+1 .. k1 (some reflectors still zero there)
        for (int i = kl + 1; i <= k1 && i < q; ++i) {
          const double* yi = yt.data() + (size_t)i * NB;
          for (int a = 0; a < ng; ++a) {
            const double va = vat(k1 - a, i);
            for (int t = 0; t < NB; ++t) d[a][t] += va * yi[t];
          }
        }
        // bulk rows k1+1 .. q-1
        const double* vp[GR];
        for (int a = 0; a < GR; ++a) vp[a] = a < ng ? Vr.data() + off[k1 - a] + a : nullptr;
        if (ng == GR) {
          for (int i = k1 + 1; i < q; ++i) {
            const double* yi = yt.data() + (size_t)i * NB;
            const int o = i - k1 - 1;
            for (int a = 0; a < GR; ++a) {
              const double va = vp[a][o];
              for (int t = 0; t < NB; ++t) d[a][t] += va * yi[t];
            }
          }
        } else {
          for (int i = k1 + 1; i < q; ++i) {
            const double* yi = yt.data() + (size_t)i * NB;
            const int o = i - k1 - 1;
            for (int a = 0; a < ng; ++a) {
              const double va = vp[a][o];
              for (int t = 0; t < NB; ++t) d[a][t] += va * yi[t];
            }
          }
        }
        // factors of the successive reflections
        double sf[GR][NB] = {};
        for (int a = 0; a < ng; ++a) {
          const double ta = tau[k1 - a];
          for (int t = 0; t < NB; ++t) {
            double x = d[a][t];
            for (int b = 0; b < a; ++b) x -= gram[((size_t)g * GR + a) * GR + b] * sf[b][t];
            sf[a][t] = ta * x;
          }
        }
        for (int i = kl + 1; i <= k1 && i < q; ++i) {
          double* yi = yt.data() + (size_t)i * NB;
          for (int a = 0; a < ng; ++a) {
            const double va = vat(k1 - a, i);
            for (int t = 0; t < NB; ++t) yi[t] -= sf[a][t] * va;
          }
        }
        for (int i = k1 + 1; i < q; ++i) {
          double* __restrict__ yi = yt.data() + (size_t)i * NB;
          const int o = i - k1 - 1;
          for (int a = 0; a < ng; ++a) {
            const double va = vp[a][o];
            for (int t = 0; t < NB; ++t) yi[t] -= sf[a][t] * va;
          }
        }
      }
      for (int i = q - 1; i >= 0; --i) {
        double* __restrict__ yi = yt.data() + (size_t)i * NB;
        for (int p = i + 1; p <= std::min(q - 1, i + kb); ++p) {
          const double l = Lat(p, i);
          const double* yp = yt.data() + (size_t)p * NB;
          for (int t = 0; t < NB; ++t) yi[t] -= l * yp[t];
        }
        const double dii = Lat(i, i);
        for (int t = 0; t < NB; ++t) yi[t] /= dii;
      }
      for (int t = 0; t < NB; ++t)
        for (int i = 0; i < q; ++i) yb[(size_t)t * ldz + i] = yt[(size_t)i * NB + t];
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
      for (int j = 0; j < q; ++j) V[(size_t)i * q + j] = Y[(size_t)order[j] * ldz + i];
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

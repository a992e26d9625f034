// One-dimensional MO-FEM assembly on the host (FP64).
//
// Computes the weighted 1D matrices of Sec. 3.1 (eq. (23)) and Sec. 3.2
// (eqs. (29)-(31)) for P_k Lagrange elements with equispaced element nodes,
// and their lumped P1 counterparts of Sec. 3.3 (eqs. (36)-(39)), in the
// banded DIA layout of include/mofem.h.  Element integrals use Gauss-Legendre
// quadrature whose nodes are found by Newton's method on the three-term
// Legendre recurrence; lumping integrates the element-wise linear
// interpolant of the integrand, i.e. the two-point rule at the element ends.
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "mofem_internal.h"

namespace mofem {

// ---------------------------------------------------------------------------
// errors and threads
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
const char* last_error_cstr() { return g_last_error.c_str(); }

namespace {
int default_threads() {
  static int n = [] {
    unsigned h = std::thread::hardware_concurrency();
    int t = h ? (int)h : 4;
    return t > 16 ? 16 : t;
  }();
  return n;
}
std::atomic<int> g_host_threads{0};  // 0: default_threads()
thread_local int t_thread_share = 0;  // > 0: this thread's calls use that many
}  // namespace

int host_threads() {
  if (t_thread_share > 0) return t_thread_share;
  const int g = g_host_threads.load(std::memory_order_relaxed);
  return g > 0 ? g : default_threads();
}

int set_thread_share(int n) {
  const int prev = t_thread_share;
  t_thread_share = n > 0 ? n : 0;
  return prev;
}

void parallel_for(long n, long min_chunk, const std::function<void(long, long)>& fn) {
  int nt = host_threads();
  if (min_chunk < 1) min_chunk = 1;
  long max_t = (n + min_chunk - 1) / min_chunk;
  if (max_t < nt) nt = (int)max_t;
  if (nt <= 1) {
    if (n > 0) fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  long chunk = (n + nt - 1) / nt;
  for (int t = 1; t < nt; ++t) {
    long b = t * chunk, e = std::min(n, b + chunk);
    if (b < e) th.emplace_back([&fn, b, e] { fn(b, e); });
  }
  fn(0, std::min(n, chunk));
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// quadrature and basis
// ---------------------------------------------------------------------------
void gauss_legendre01(int nq, double* x, double* w) {
  // roots of P_nq on [-1, 1]: Newton from the Chebyshev-like initial guess
  for (int i = 0; i < nq; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 1; j < nq; ++j) {
        double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_nq(z), p0 = P_{nq-1}(z)
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int j = 1; j < nq; ++j) {
        double p2 = ((2.0 * j + 1.0) * z * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = nq * (z * p1 - p0) / (z * z - 1.0);
    }
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = 0.5 * (1.0 - z);  // ascending on [0, 1]
    w[i] = 0.5 * wt;
  }
}

void lagrange_equispaced(int k, double xi, double* val, double* der) {
  // psi_a(xi) = prod_{b != a} (xi - b/k) / ((a - b)/k), reference element [0, 1]
  for (int a = 0; a <= k; ++a) {
    double num = 1.0, den = 1.0, dsum = 0.0;
    for (int b = 0; b <= k; ++b) {
      if (b == a) continue;
      den *= (double)(a - b) / k;
    }
    for (int b = 0; b <= k; ++b) {
      if (b == a) continue;
      num *= xi - (double)b / k;
    }
    // derivative via the sum over the dropped factor
    for (int c = 0; c <= k; ++c) {
      if (c == a) continue;
      double t = 1.0;
      for (int b = 0; b <= k; ++b) {
        if (b == a || b == c) continue;
        t *= xi - (double)b / k;
      }
      dsum += t;
    }
    val[a] = num / den;
    der[a] = dsum / den;
  }
}

double eval_weight(const mofem_weight* w, double x) {
  if (!w) return 1.0;
  const double* p = w->p;
  switch (w->kind) {
    case MOFEM_W_ONE: return 1.0;
    case MOFEM_W_POLY: return p[0] + x * (p[1] + x * (p[2] + x * p[3]));
    case MOFEM_W_PROFILE: return p[0] + p[1] * std::sin(p[2] * x + p[3]);
    case MOFEM_W_PROFILE_D: return p[1] * p[2] * std::cos(p[2] * x + p[3]);
    case MOFEM_W_PROFILE_INV: return 1.0 / (p[0] + p[1] * std::sin(p[2] * x + p[3]));
    case MOFEM_W_PROFILE_D2L: {
      double L = p[0] + p[1] * std::sin(p[2] * x + p[3]);
      double dL = p[1] * p[2] * std::cos(p[2] * x + p[3]);
      return dL * dL / L;
    }
    case MOFEM_W_CALLBACK: return w->fn(x, w->ctx);
    case MOFEM_W_PPROFILE_D: return p[1] + x * (2.0 * p[2] + x * 3.0 * p[3]);
    case MOFEM_W_PPROFILE_INV: return 1.0 / (p[0] + x * (p[1] + x * (p[2] + x * p[3])));
    case MOFEM_W_PPROFILE_D2L: {
      double L = p[0] + x * (p[1] + x * (p[2] + x * p[3]));
      double dL = p[1] + x * (2.0 * p[2] + x * 3.0 * p[3]);
      return dL * dL / L;
    }
    default: return NAN;
  }
}

void band_to_dense(int n, int kb, const double* band, int trim, double* dense) {
  int q = n - 2 * trim;
  std::memset(dense, 0, sizeof(double) * (size_t)q * q);
  for (int i = 0; i < q; ++i) {
    int gi = i + trim;
    for (int d = 0; d <= 2 * kb; ++d) {
      int gj = gi + d - kb;
      int j = gj - trim;
      if (j < 0 || j >= q) continue;
      dense[(size_t)i * q + j] = band[(size_t)d * n + gi];
    }
  }
}

}  // namespace mofem

using namespace mofem;

extern "C" int mofem_version(void) { return 10000 * 0 + 100 * 1 + 0; }

extern "C" const char* mofem_last_error(void) { return last_error_cstr(); }

extern "C" int mofem_assemble_1d(int order, int m_elem, double x0, double x1, int di, int dj,
                                 const mofem_weight* w, int nq, double* band) {
  clear_error();
  if (order < 0 || order > 4) return fail(MOFEM_E_ARG, "assemble_1d: order must be 0..4");
  if (m_elem < 1) return fail(MOFEM_E_ARG, "assemble_1d: m_elem must be >= 1");
  if ((di != 0 && di != 1) || (dj != 0 && dj != 1))
    return fail(MOFEM_E_ARG, "assemble_1d: derivative orders must be 0 or 1");
  if (!band) return fail(MOFEM_E_ARG, "assemble_1d: band is NULL");
  if (!(x1 > x0)) return fail(MOFEM_E_ARG, "assemble_1d: need x1 > x0");
  if (nq == 0) nq = 12;
  if (nq < 1 || nq > 32) return fail(MOFEM_E_ARG, "assemble_1d: nq must be 1..32");
  if (w && (w->kind < MOFEM_W_ONE || w->kind > MOFEM_W_PPROFILE_D2L))
    return fail(MOFEM_E_ARG, "assemble_1d: unknown weight kind");
  if (w && w->kind == MOFEM_W_CALLBACK && !w->fn)
    return fail(MOFEM_E_ARG, "assemble_1d: callback weight without function");

  const bool lumped = (order == 0);
  const int k = lumped ? 1 : order;
  const int kb = k;
  const long n = (long)k * m_elem + 1;
  const double h = (x1 - x0) / m_elem;
  std::memset(band, 0, sizeof(double) * (size_t)(2 * kb + 1) * n);

  std::vector<double> xq, wq;
  if (lumped) {
    xq = {0.0, 1.0};
    wq = {0.5, 0.5};
  } else {
    xq.resize(nq);
    wq.resize(nq);
    gauss_legendre01(nq, xq.data(), wq.data());
  }
  const int npt = (int)xq.size();
  std::vector<double> val((size_t)npt * (k + 1)), der((size_t)npt * (k + 1));
  for (int p = 0; p < npt; ++p) lagrange_equispaced(k, xq[p], &val[(size_t)p * (k + 1)], &der[(size_t)p * (k + 1)]);

  std::vector<double> loc((size_t)(k + 1) * (k + 1));
  for (int e = 0; e < m_elem; ++e) {
    std::fill(loc.begin(), loc.end(), 0.0);
    for (int p = 0; p < npt; ++p) {
      double x = x0 + h * (e + xq[p]);
      double ww = eval_weight(w, x) * wq[p] * h;
      const double* v = &val[(size_t)p * (k + 1)];
      const double* dv = &der[(size_t)p * (k + 1)];
      for (int a = 0; a <= k; ++a) {
        double fa = di ? dv[a] / h : v[a];
        for (int b = 0; b <= k; ++b) {
          double fb = dj ? dv[b] / h : v[b];
          loc[(size_t)a * (k + 1) + b] += ww * fa * fb;
        }
      }
    }
    for (int a = 0; a <= k; ++a) {
      long gi = (long)e * k + a;
      for (int b = 0; b <= k; ++b) {
        long gj = (long)e * k + b;
        int d = (int)(gj - gi) + kb;
        band[(size_t)d * n + gi] += loc[(size_t)a * (k + 1) + b];
      }
    }
  }
  for (size_t i = 0; i < (size_t)(2 * kb + 1) * n; ++i)
    if (!std::isfinite(band[i])) return fail(MOFEM_E_NOTFINITE, "assemble_1d: weight produced a non-finite value");
  return MOFEM_OK;
}

extern "C" int mofem_set_host_threads(int n) {
  clear_error();
  const int prev = mofem::host_threads();
  mofem::g_host_threads.store(n > 0 ? (n > 256 ? 256 : n) : 0, std::memory_order_relaxed);
  return prev;
}

// Vector kernels of the MO-PCG recurrence (Sec. 5, eqs. (77)-(78)), FP64.
//
// Every nodal matrix of one batch item is treated as a flat contiguous array
// of n = q_s * q_t doubles.  Each item is processed by vec_blocks(n) blocks
// of 256 threads; a block owns one contiguous chunk, so its loads are
// coalesced.  Frobenius products (sum(sum(X o Y)) of eq. (77)) are reduced
// deterministically: per-block partial sums in a fixed order, then one block
// per item adds the partials in a fixed order (no floating-point atomics),
// so results are bitwise reproducible from run to run.  The scalar
// recurrence (alpha, beta) is computed on the device from those sums.
#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void chunk_of(long long n, int blk, int nblk, long long* b, long long* e) {
  long long c = (n + nblk - 1) / nblk;
  *b = (long long)blk * c;
  *e = *b + c < n ? *b + c : n;
  if (*b > n) *b = n;
}

// block-wide sum in fixed order; result valid in thread 0
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kThreads / 64];
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) t += red[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ partial, int np,
                                                          double* __restrict__ out) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) s += partial[(size_t)b * np + i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[b] = s;
}

// out[b] = beta * out[b] + alpha * sum of the item's partials (fixed order)
__global__ __launch_bounds__(kThreads) void reduce_axpy_kernel(const double* __restrict__ partial, int np,
                                                               double* __restrict__ out, double alpha,
                                                               double beta) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) s += partial[(size_t)b * np + i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[b] = (beta == 0.0 ? 0.0 : beta * out[b]) + alpha * s;
}

template <typename YT>
__global__ __launch_bounds__(kThreads) void dot_kernel(const double* __restrict__ X, const YT* __restrict__ Y,
                                                       long long n, long long stride,
                                                       double* __restrict__ partial, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const double* x = X + (size_t)b * stride;
  const YT* y = Y + (size_t)b * stride;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) s = fma(x[i], (double)y[i], s);
  s = block_sum(s);
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = s;
}


// R may alias Y (each element is read before it is written by the same thread)
__global__ __launch_bounds__(kThreads) void residual_kernel(const double* __restrict__ Rhs, const double* Y,
                                                            double* R, long long n, long long stride,
                                                            long long rhs_stride, double* __restrict__ partial,
                                                            const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const double* f = Rhs + (size_t)b * rhs_stride;
  const double* y = Y + (size_t)b * stride;
  double* r = R + (size_t)b * stride;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    double v = f[i] - y[i];
    r[i] = v;
    s = fma(v, v, s);
  }
  s = block_sum(s);
  if (threadIdx.x == 0 && partial) partial[(size_t)b * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void cg_update_kernel(double* __restrict__ U, double* __restrict__ R,
                                                             const double* __restrict__ Q, const double* __restrict__ Y,
                                                             const double* __restrict__ num, const double* __restrict__ den,
                                                             double* __restrict__ alpha_out, long long n, long long stride,
                                                             long long u_stride, double* __restrict__ partial,
                                                             const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const double alpha = num[b] / den[b];
  if (blockIdx.x == 0 && threadIdx.x == 0 && alpha_out) alpha_out[b] = alpha;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double* u = U ? U + (size_t)b * u_stride : nullptr;
  double* r = R + (size_t)b * stride;
  const double* q = Q + (size_t)b * stride;
  const double* y = Y + (size_t)b * stride;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    if (u) u[i] = fma(alpha, q[i], u[i]);
    double v = fma(-alpha, y[i], r[i]);
    r[i] = v;
    s = fma(v, v, s);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// cg_update, also writing R's padded transform operand (row length Kp):
// FP64, FP32 or split BF16 (hi, lo).  Each thread walks its elements with a
// running (row, col) so no division sits in the loop.
__global__ __launch_bounds__(kThreads) void cg_update_pad_kernel(
    double* __restrict__ U, double* __restrict__ R, const double* __restrict__ Q, const double* __restrict__ Y,
    const double* __restrict__ num, const double* __restrict__ den, double* __restrict__ alpha_out, int qt,
    long long n, long long stride, long long u_stride, double* __restrict__ partial, const int* active,
    unsigned short* __restrict__ ohi, unsigned short* __restrict__ olo, double* __restrict__ o64,
    float* __restrict__ o32, long long o_stride) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const double alpha = num[b] / den[b];
  if (blockIdx.x == 0 && threadIdx.x == 0 && alpha_out) alpha_out[b] = alpha;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double* u = U ? U + (size_t)b * u_stride : nullptr;  // null: the solution update is deferred
  double* r = R + (size_t)b * stride;
  const double* q = Q + (size_t)b * stride;
  const double* y = Y + (size_t)b * stride;
  const int Kp = pad_up(qt);
  const size_t ob = (size_t)b * o_stride;
  long long i = lo + threadIdx.x;
  long long row = i / qt;
  int col = (int)(i - row * qt);
  double s = 0.0;
  for (; i < hi; i += kThreads) {
    if (u) u[i] = fma(alpha, q[i], u[i]);
    const double v = fma(-alpha, y[i], r[i]);
    r[i] = v;
    s = fma(v, v, s);
    const size_t o = ob + (size_t)row * Kp + col;
    if (o64) {
      o64[o] = v;
    } else if (o32) {
      o32[o] = (float)v;
    } else {
      const float f = (float)v;
      const __bf16 h = (__bf16)f;
      ohi[o] = __builtin_bit_cast(unsigned short, h);
      if (olo) olo[o] = __builtin_bit_cast(unsigned short, (__bf16)(f - (float)h));
    }
    col += kThreads;
    while (col >= qt) {
      col -= qt;
      ++row;
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// <R, Z> and <Z, Y> in one pass (Z read once); Z in FP64 or FP32
template <typename ZT>
__global__ __launch_bounds__(kThreads) void zdots_kernel(const double* __restrict__ R, const ZT* __restrict__ Z,
                                                         const double* __restrict__ Y, long long n, long long stride,
                                                         double* __restrict__ p1, double* __restrict__ p2,
                                                         const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const size_t off = (size_t)b * stride;
  double s1 = 0.0, s2 = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double z = (double)Z[off + i];
    s1 = fma(R[off + i], z, s1);
    s2 = fma(z, Y[off + i], s2);
  }
  s1 = block_sum(s1);
  s2 = block_sum(s2);
  if (threadIdx.x == 0) {
    p1[(size_t)b * gridDim.x + blockIdx.x] = s1;
    p2[(size_t)b * gridDim.x + blockIdx.x] = s2;
  }
}
// The deferred solution update and the new direction in one pass, for items
// live in this iteration: U += alpha Q (every live item), then Q = Z + beta Q
// (items still active).
template <typename ZT>
__global__ __launch_bounds__(kThreads) void step_direction_kernel(double* __restrict__ Q, const ZT* __restrict__ Z,
                                                                  const double* __restrict__ beta,
                                                                  double* __restrict__ U,
                                                                  const double* __restrict__ alpha, long long n,
                                                                  long long stride, long long u_stride,
                                                                  const int* live, const int* active) {
  const int b = blockIdx.y;
  if (!live[b]) return;
  const bool act = active[b] != 0;
  const double al = alpha[b], be = act ? beta[b] : 0.0;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double* q = Q + (size_t)b * stride;
  const ZT* z = Z + (size_t)b * stride;
  double* u = U + (size_t)b * u_stride;
  if (act) {
    for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
      const double qo = q[i];
      u[i] = fma(al, qo, u[i]);
      q[i] = fma(be, qo, (double)z[i]);
    }
  } else {
    for (long long i = lo + threadIdx.x; i < hi; i += kThreads) u[i] = fma(al, q[i], u[i]);
  }
}
template <typename ZT>
__global__ __launch_bounds__(kThreads) void direction_kernel(double* __restrict__ Q, const ZT* __restrict__ Z,
                                                             const double* __restrict__ beta, long long n,
                                                             long long stride, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const double be = beta ? beta[b] : 0.0;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  double* q = Q + (size_t)b * stride;
  const ZT* z = Z + (size_t)b * stride;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) q[i] = fma(be, q[i], (double)z[i]);
}

__global__ __launch_bounds__(kThreads) void copy_kernel(const double* __restrict__ X, double* __restrict__ Y,
                                                        long long n, long long xs, long long ys) {
  const int b = blockIdx.y;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) Y[(size_t)b * ys + i] = X[(size_t)b * xs + i];
}

__global__ __launch_bounds__(kThreads) void fill_kernel(double* __restrict__ X, double v, long long n,
                                                        long long stride) {
  const int b = blockIdx.y;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) X[(size_t)b * stride + i] = v;
}

__global__ void beta_kernel(const double* __restrict__ rz_new, double* __restrict__ rz_old,
                            const double* __restrict__ zy, const double* __restrict__ alpha,
                            double* __restrict__ beta, int flexible, int batch, const int* active) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  if (active && !active[b]) return;
  double bt = flexible ? (-alpha[b] * zy[b] / rz_old[b]) : (rz_new[b] / rz_old[b]);
  beta[b] = bt;
  rz_old[b] = rz_new[b];
}

// ---- device-side control of the MO-PCG iteration ---------------------------
// Per item: active (iterating), claim (its recurrence residual passed the
// target: confirm on the true residual), restart (the true residual did
// not: continue from it with a fresh direction), status, iteration count.
// The host only reads `active` every few iterations.
constexpr int kStatusOk = 0, kStatusBreakdown = -4, kStatusMaxit = -5, kStatusNotFinite = -7;

__global__ void pcg_init_kernel(const double* __restrict__ rhs2, const double* __restrict__ rr,
                                double* __restrict__ target2, int* __restrict__ active, int* __restrict__ claim,
                                int* __restrict__ restart, int* __restrict__ status, int* __restrict__ iters,
                                double tol2, int tau_stop, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double r = rr[b], f = rhs2[b];
  claim[b] = 0;
  restart[b] = 0;
  iters[b] = 0;
  if (!isfinite(r) || !isfinite(f)) {
    status[b] = kStatusNotFinite;
    active[b] = 0;
    target2[b] = 0.0;
    return;
  }
  status[b] = kStatusOk;
  const double t = tol2 * (tau_stop ? r : f);
  target2[b] = t;
  active[b] = (f == 0.0 || r <= t) ? 0 : 1;
}


// The per-iteration control kernels run one block per item: they first add
// the item's partial sums in the fixed order of reduce_kernel (so the result
// is the same), then thread 0 takes the item's decision.
__device__ __forceinline__ double item_sum(const double* __restrict__ partial, int np, int b) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kThreads) s += partial[(size_t)b * np + i];
  return block_sum(s);  // valid in thread 0
}

// rr_b = ||R_b||^2 from the CG update's partials; breakdown / non-finite
// checks; claim of convergence when rr_b <= target2_b.  live[b]: this
// iteration's step alpha Q is valid and still to be added to U (by the
// direction pass, which runs for live items); not set on breakdown, so U
// keeps the last valid iterate.
__global__ __launch_bounds__(kThreads) void check_kernel(const double* __restrict__ part, int np,
                                                         double* __restrict__ rr, const double* __restrict__ qy,
                                                         const double* __restrict__ target2, int* __restrict__ active,
                                                         int* __restrict__ claim, int* __restrict__ status,
                                                         int* __restrict__ iters, int* __restrict__ live) {
  const int b = blockIdx.x;
  if (!active[b]) {
    if (threadIdx.x == 0) {
      claim[b] = 0;
      if (live) live[b] = 0;
    }
    return;
  }
  const double r = item_sum(part, np, b);
  if (threadIdx.x != 0) return;
  rr[b] = r;
  claim[b] = 0;
  if (live) live[b] = 0;
  iters[b] += 1;
  const double a = qy[b];
  if (!isfinite(a) || !(a > 0.0)) {
    status[b] = kStatusBreakdown;
    active[b] = 0;
  } else if (!isfinite(r)) {
    status[b] = kStatusNotFinite;
    active[b] = 0;
  } else {
    if (live) live[b] = 1;
    if (r <= target2[b]) claim[b] = 1;
  }
}
// tr_b = true residual ||Rhs - L(U)||^2 of a claiming item: converged, or
// restart from the true residual
__global__ __launch_bounds__(kThreads) void confirm_kernel(const double* __restrict__ part, int np,
                                                           double* __restrict__ tr,
                                                           const double* __restrict__ target2,
                                                           int* __restrict__ active, const int* __restrict__ claim,
                                                           int* __restrict__ restart) {
  const int b = blockIdx.x;
  if (!claim[b]) return;
  const double t = item_sum(part, np, b);
  if (threadIdx.x != 0) return;
  tr[b] = t;
  if (t <= target2[b]) active[b] = 0;
  else restart[b] = 1;  // the recurrence drifted: continue from the true residual
}
// rz_new = <R, Z>, zy = <Z, Y> from the two-dot partials; beta (0 after a
// restart): standard rz_new / rz_old or flexible -alpha zy / rz_old
__global__ __launch_bounds__(kThreads) void beta_kernel(const double* __restrict__ part_rz,
                                                        const double* __restrict__ part_zy, int np,
                                                        double* __restrict__ rz_new, double* __restrict__ zy,
                                                        double* __restrict__ rz_old, const double* __restrict__ alpha,
                                                        double* __restrict__ beta, int* __restrict__ restart,
                                                        int flexible, const int* __restrict__ active) {
  const int b = blockIdx.x;
  if (!active[b]) return;
  const double s1 = item_sum(part_rz, np, b);
  const double s2 = item_sum(part_zy, np, b);
  if (threadIdx.x != 0) return;
  rz_new[b] = s1;
  zy[b] = s2;
  double bt = flexible ? (-alpha[b] * s2 / rz_old[b]) : (s1 / rz_old[b]);
  if (restart[b]) {
    bt = 0.0;
    restart[b] = 0;
  }
  beta[b] = bt;
  rz_old[b] = s1;
}
// R = Rhs - LU - alpha_b Y: the residual of U + alpha Q with Y = L(Q)
__global__ __launch_bounds__(kThreads) void residual_step_kernel(const double* __restrict__ Rhs, const double* LU,
                                                                 const double* __restrict__ Y,
                                                                 const double* __restrict__ alpha, double* R,
                                                                 long long n, long long stride, long long rhs_stride,
                                                                 double* __restrict__ partial, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const double al = alpha[b];
  const double* f = Rhs + (size_t)b * rhs_stride;
  const double* ly = LU + (size_t)b * stride;
  const double* y = Y + (size_t)b * stride;
  double* r = R + (size_t)b * stride;
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double v = fma(-al, y[i], f[i] - ly[i]);
    r[i] = v;
    s = fma(v, v, s);
  }
  s = block_sum(s);
  if (threadIdx.x == 0 && partial) partial[(size_t)b * gridDim.x + blockIdx.x] = s;
}

// per-item result of a solve: iterations, status (MAXIT if the final true
// residual misses the item's target), relative true residual
__global__ void pcg_final_kernel(const double* __restrict__ tr, const double* __restrict__ rhs2,
                                 const double* __restrict__ target2, const int* __restrict__ status,
                                 const int* __restrict__ iters, int* __restrict__ iters_out,
                                 int* __restrict__ status_out, double* __restrict__ relres_out, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double t = tr[b], f = rhs2[b];
  int st = status[b];
  if (st == kStatusOk && !(t <= target2[b] || (f == 0.0 && t == 0.0))) st = kStatusMaxit;
  const int it = iters[b];
  iters_out[b] = it;
  status_out[b] = st;
  relres_out[b] = f > 0.0 ? sqrt(t / f) : sqrt(t);
}

// beta of the next direction; zero (a fresh direction) for restarted items

__global__ __launch_bounds__(kThreads) void copy_masked_kernel(const double* __restrict__ X, double* __restrict__ Y,
                                                               long long n, long long xs, long long ys,
                                                               const int* __restrict__ mask) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) Y[(size_t)b * ys + i] = X[(size_t)b * xs + i];
}

__global__ void scale_items_kernel(double* __restrict__ x, const double* __restrict__ f, int batch) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) x[b] *= f[b];
}

// DIB kinetics, Sec. 7, eqs. (99)-(100); kin = rho, A1, A2, B, C, D, alpha, gamma, k2, k3
__global__ __launch_bounds__(kThreads) void dib_source_kernel(const double* __restrict__ U, const double* __restrict__ V,
                                                              double* __restrict__ TU, double* __restrict__ TV,
                                                              long long n, long long stride, double rho, double A1,
                                                              double A2, double Bc, double Cc, double Dc,
                                                              double al, double ga, double k2, double k3,
                                                              double tau) {
  const int b = blockIdx.y;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const size_t off = (size_t)b * stride;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double e = U[off + i], th = V[off + i];
    const double f = A1 * (1.0 - th) * e - A2 * e * e * e - Bc * (th - al);
    const double g = Cc * (1.0 + k2 * e) * (1.0 - th) * (1.0 - ga * (1.0 - th)) -
                     Dc * th * (1.0 + ga * th) * (1.0 + k3 * e);
    TU[off + i] = fma(tau * rho, f, e);
    TV[off + i] = fma(tau * rho, g, th);
  }
}

// Adjoint of the explicit DIB kinetics (eqs. (99)-(100)) in one IMEX step:
//   LU = NU + tau rho (f_u NU + g_u NV),  LV = NV + tau rho (f_v NU + g_v NV),
// partial derivatives at the step's input state (U, V).
__global__ __launch_bounds__(kThreads) void dib_adjoint_kernel(const double* __restrict__ U, const double* __restrict__ V,
                                                               const double* __restrict__ NU,
                                                               const double* __restrict__ NV, double* __restrict__ LU,
                                                               double* __restrict__ LV, long long n, long long stride,
                                                               double rho, double A1, double A2, double Bc, double Cc,
                                                               double Dc, double ga, double k2, double k3,
                                                               double tau) {
  const int b = blockIdx.y;
  long long lo, hi;
  chunk_of(n, blockIdx.x, gridDim.x, &lo, &hi);
  const size_t off = (size_t)b * stride;
  const double r = tau * rho;
  for (long long i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double e = U[off + i], th = V[off + i];
    const double nu = NU[off + i], nv = NV[off + i];
    const double f_e = A1 * (1.0 - th) - 3.0 * A2 * e * e;
    const double f_t = -A1 * e - Bc;
    const double g_e = Cc * k2 * (1.0 - th) * (1.0 - ga * (1.0 - th)) - Dc * k3 * th * (1.0 + ga * th);
    const double g_t = Cc * (1.0 + k2 * e) * (2.0 * ga * (1.0 - th) - 1.0) - Dc * (1.0 + k3 * e) * (1.0 + 2.0 * ga * th);
    LU[off + i] = nu + r * (f_e * nu + g_e * nv);
    LV[off + i] = nv + r * (f_t * nu + g_t * nv);
  }
}

}  // namespace

#define CHECK_LAUNCH() return hipGetLastError() == hipSuccess ? 0 : -1

int launch_reduce(const double* partial, int n_partial, double* out, int batch, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(batch), dim3(kThreads), 0, s, partial, n_partial, out);
  CHECK_LAUNCH();
}
int launch_reduce_axpy(const double* partial, int n_partial, double* out, double alpha, double beta, int batch,
                       hipStream_t s) {
  hipLaunchKernelGGL(reduce_axpy_kernel, dim3(batch), dim3(kThreads), 0, s, partial, n_partial, out, alpha, beta);
  CHECK_LAUNCH();
}
int launch_dib_adjoint(const double* U, const double* V, const double* NU, const double* NV, double* LU, double* LV,
                       long long n, long long stride, int batch, const double* k, double tau, hipStream_t s) {
  hipLaunchKernelGGL(dib_adjoint_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, U, V, NU, NV, LU, LV, n,
                     stride, k[0], k[1], k[2], k[3], k[4], k[5], k[7], k[8], k[9], tau);
  CHECK_LAUNCH();
}
int launch_dot_partial(const double* X, const double* Y, long long n, long long stride, int batch,
                       double* partial, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel<double>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, X, Y, n, stride, partial,
                     active);
  CHECK_LAUNCH();
}
int launch_residual(const double* Rhs, const double* Y, double* R, long long n, long long stride,
                    long long rhs_stride, int batch, double* partial, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Rhs, Y, R, n, stride,
                     rhs_stride, partial, active);
  CHECK_LAUNCH();
}
int launch_cg_update(double* U, double* R, const double* Q, const double* Y, const double* num, const double* den,
                     double* alpha_out, long long n, long long stride, long long u_stride, int batch,
                     double* partial, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(cg_update_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, U, R, Q, Y, num, den,
                     alpha_out, n, stride, u_stride, partial, active);
  CHECK_LAUNCH();
}
int launch_cg_update_pad(double* U, double* R, const double* Q, const double* Y, const double* num,
                         const double* den, double* alpha_out, int qs, int qt, long long stride,
                         long long u_stride, int batch, double* partial, const int* active, unsigned short* ohi,
                         unsigned short* olo, double* o64, float* o32, long long o_stride, hipStream_t s) {
  if (!ohi && !o64 && !o32)  // no transform operand wanted
    return launch_cg_update(U, R, Q, Y, num, den, alpha_out, (long long)qs * qt, stride, u_stride, batch, partial,
                            active, s);
  hipLaunchKernelGGL(cg_update_pad_kernel, dim3(vec_blocks((long long)qs * qt), batch), dim3(kThreads), 0, s, U, R, Q, Y, num, den,
                     alpha_out, qt, (long long)qs * qt, stride, u_stride, partial, active, ohi, olo, o64, o32,
                     o_stride);
  CHECK_LAUNCH();
}
int launch_direction(double* Q, const double* Z, const double* beta, long long n, long long stride, int batch,
                     const int* active, hipStream_t s) {
  hipLaunchKernelGGL(direction_kernel<double>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Q, Z, beta, n, stride,
                     active);
  CHECK_LAUNCH();
}
int launch_step_direction(double* Q, const double* Z, const double* beta, double* U, const double* alpha,
                          long long n, long long stride, long long u_stride, int batch, const int* live,
                          const int* active, hipStream_t s) {
  hipLaunchKernelGGL(step_direction_kernel<double>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Q, Z, beta, U,
                     alpha, n, stride, u_stride, live, active);
  CHECK_LAUNCH();
}
int launch_step_direction(double* Q, const float* Z, const double* beta, double* U, const double* alpha,
                          long long n, long long stride, long long u_stride, int batch, const int* live,
                          const int* active, hipStream_t s) {
  hipLaunchKernelGGL(step_direction_kernel<float>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Q, Z, beta, U,
                     alpha, n, stride, u_stride, live, active);
  CHECK_LAUNCH();
}
int launch_residual_step(const double* Rhs, const double* LU, const double* Y, const double* alpha, double* R,
                         long long n, long long stride, long long rhs_stride, int batch, double* partial,
                         const int* active, hipStream_t s) {
  hipLaunchKernelGGL(residual_step_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Rhs, LU, Y, alpha, R, n,
                     stride, rhs_stride, partial, active);
  CHECK_LAUNCH();
}
int launch_direction(double* Q, const float* Z, const double* beta, long long n, long long stride, int batch,
                     const int* active, hipStream_t s) {
  hipLaunchKernelGGL(direction_kernel<float>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, Q, Z, beta, n, stride,
                     active);
  CHECK_LAUNCH();
}
int launch_dot_partial(const double* X, const float* Y, long long n, long long stride, int batch, double* partial,
                       const int* active, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel<float>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, X, Y, n, stride, partial,
                     active);
  CHECK_LAUNCH();
}
int launch_zdots_partial(const double* R, const double* Z, const double* Y, long long n, long long stride, int batch,
                         double* p1, double* p2, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(zdots_kernel<double>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, R, Z, Y, n, stride, p1, p2,
                     active);
  CHECK_LAUNCH();
}
int launch_zdots_partial(const double* R, const float* Z, const double* Y, long long n, long long stride, int batch,
                         double* p1, double* p2, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(zdots_kernel<float>, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, R, Z, Y, n, stride, p1, p2,
                     active);
  CHECK_LAUNCH();
}
int launch_copy(const double* X, double* Y, long long n, long long xs, long long ys, int batch, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, X, Y, n, xs, ys);
  CHECK_LAUNCH();
}
int launch_fill(double* X, double v, long long n, long long stride, int batch, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, X, v, n, stride);
  CHECK_LAUNCH();
}
int launch_beta(const double* rz_new, double* rz_old, const double* zy, const double* alpha, double* beta,
                int flexible, int batch, const int* active, hipStream_t s) {
  hipLaunchKernelGGL(beta_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, rz_new, rz_old, zy, alpha, beta,
                     flexible, batch, active);
  CHECK_LAUNCH();
}
int launch_pcg_init(const double* rhs2, const double* rr, double* target2, int* active, int* claim, int* restart,
                    int* status, int* iters, double tol2, int tau_stop, int batch, hipStream_t s) {
  hipLaunchKernelGGL(pcg_init_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, rhs2, rr, target2, active, claim,
                     restart, status, iters, tol2, tau_stop, batch);
  CHECK_LAUNCH();
}
int launch_pcg_final(const double* tr, const double* rhs2, const double* target2, const int* status,
                     const int* iters, int* iters_out, int* status_out, double* relres_out, int batch,
                     hipStream_t s) {
  hipLaunchKernelGGL(pcg_final_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, tr, rhs2, target2, status, iters,
                     iters_out, status_out, relres_out, batch);
  CHECK_LAUNCH();
}
int launch_check(const double* part, int np, double* rr, const double* qy, const double* target2, int* active,
                 int* claim, int* status, int* iters, int* live, int batch, hipStream_t s) {
  hipLaunchKernelGGL(check_kernel, dim3(batch), dim3(kThreads), 0, s, part, np, rr, qy, target2, active, claim,
                     status, iters, live);
  CHECK_LAUNCH();
}
int launch_confirm(const double* part, int np, double* tr, const double* target2, int* active, const int* claim,
                   int* restart, int batch, hipStream_t s) {
  hipLaunchKernelGGL(confirm_kernel, dim3(batch), dim3(kThreads), 0, s, part, np, tr, target2, active, claim,
                     restart);
  CHECK_LAUNCH();
}
int launch_beta(const double* part_rz, const double* part_zy, int np, double* rz_new, double* zy, double* rz_old,
                const double* alpha, double* beta, int* restart, int flexible, const int* active, int batch,
                hipStream_t s) {
  hipLaunchKernelGGL(beta_kernel, dim3(batch), dim3(kThreads), 0, s, part_rz, part_zy, np, rz_new, zy, rz_old,
                     alpha, beta, restart, flexible, active);
  CHECK_LAUNCH();
}
int launch_copy_masked(const double* X, double* Y, long long n, long long xs, long long ys, int batch,
                       const int* mask, hipStream_t s) {
  hipLaunchKernelGGL(copy_masked_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, X, Y, n, xs, ys, mask);
  CHECK_LAUNCH();
}
int launch_scale_items(double* x, const double* f, int batch, hipStream_t s) {
  hipLaunchKernelGGL(scale_items_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, x, f, batch);
  CHECK_LAUNCH();
}
int launch_dib_source(const double* U, const double* V, double* TU, double* TV, long long n, long long stride,
                      int batch, const double* k, double tau, hipStream_t s) {
  hipLaunchKernelGGL(dib_source_kernel, dim3(vec_blocks(n), batch), dim3(kThreads), 0, s, U, V, TU, TV, n, stride,
                     k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8], k[9], tau);
  CHECK_LAUNCH();
}

}  // namespace mofem

// Banded Cholesky solves of the paper's product preconditioners.
//
// P(U) = S U T with S, T symmetric positive definite and banded (Sec. 5,
// eq. (80): S = B1, T = A + B2; Sec. 6, eq. (95): S = M3 + c B1,
// T = M + c (A + B2)).  With S = L L^T factorised on the host,
//     P^{-1}(R) = S^{-1} R T^{-1}
// is two launches of one kernel that solves along the leading index of its
// input for every column and writes the result transposed:
//     launch 1: X = R    (q_s x q_t) -> (S^{-1} R)^T            (q_t x q_s)
//     launch 2: X = that (q_t x q_s) -> (T^{-1} (S^{-1} R)^T)^T  (q_s x q_t)
// and the second output is S^{-1} R T^{-1} because T is symmetric.
//
// One thread per column: the forward substitution L w = x runs down the
// column and stores w in a scratch item, the back substitution L^T y = w
// runs up the column.  Each row's coefficients are the same for every column,
// so they are wave-uniform loads.  The column data stream through registers
// CH rows at a time, the next chunk in flight while the current one is
// solved (the recurrence itself is kb fused multiply-adds per row).  The back
// substitution collects 64 rows x 64 columns in LDS and stores them as 64
// contiguous pieces of rows of the transposed output.
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

namespace {
constexpr int kCols = 64;  // columns per block (one wave)
constexpr int kCh = 16;    // rows per register chunk (a divisor of kCols)

// index of the factor pair whose scale equals the item's scale, -1 if none
__device__ __forceinline__ int factor_set(const BcholArgs& a, int b) {
  const double s = a.item_scale ? a.item_scale[b] : 1.0;
  for (int j = 0; j < a.n_sets; ++j)
    if (a.scales[j] == s) return j;
  return -1;
}
}  // namespace

template <int KB>
__global__ __launch_bounds__(kCols) void bchol_kernel(BcholArgs a) {
  __shared__ double tile[kCols][kCols + 1];
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
  const int n = a.n_rows;
  // an item whose scale has no factor pair gets a NaN result (the solve then
  // stops with MOFEM_E_NOTFINITE) instead of another pair's preconditioner
  const int found = factor_set(a, b);
  const bool unmatched = found < 0;
  const int set = unmatched ? 0 : found;
  const double* __restrict__ Lf = a.Lf + (size_t)set * n * (KB + 1);
  const double* __restrict__ Lb = a.Lb + (size_t)set * n * (KB + 1);
  const int lane = threadIdx.x;
  const int col0 = blockIdx.x * kCols;
  const int col = col0 + lane;
  const bool in = col < a.n_cols;
  const int cc = in ? col : a.n_cols - 1;  // clamped: loads stay in bounds
  const double* __restrict__ x = a.X + (size_t)b * a.x_stride + cc;
  double* __restrict__ w = a.W + (size_t)b * a.w_stride + cc;

  // ---- forward substitution: w_i = (x_i - sum_l L[i][i-l] w_{i-l}) / L[i][i]
  double h[KB];
#pragma unroll
  for (int l = 0; l < KB; ++l) h[l] = 0.0;  // h[l] = w_{i-1-l}
  double cur[kCh], nxt[kCh];
#pragma unroll
  for (int r = 0; r < kCh; ++r) cur[r] = x[(size_t)min(r, n - 1) * a.ld_x];
  for (int i0 = 0; i0 < n; i0 += kCh) {
#pragma unroll
    for (int r = 0; r < kCh; ++r) nxt[r] = x[(size_t)min(i0 + kCh + r, n - 1) * a.ld_x];
#pragma unroll
    for (int r = 0; r < kCh; ++r) {
      const int i = i0 + r;
      if (i < n) {
        const double* c = Lf + (size_t)i * (KB + 1);
        double acc = cur[r];
#pragma unroll
        for (int l = KB; l >= 1; --l) acc = fma(-c[l], h[l - 1], acc);
        const double v = acc * c[0];
#pragma unroll
        for (int l = KB - 1; l >= 1; --l) h[l] = h[l - 1];
        h[0] = v;
        if (in) w[(size_t)i * a.n_cols] = v;
      }
    }
#pragma unroll
    for (int r = 0; r < kCh; ++r) cur[r] = nxt[r];
  }

  // ---- back substitution: y_i = (w_i - sum_l L[i+l][i] y_{i+l}) / L[i][i],
  // row blocks of 64 from the bottom; each block leaves through LDS as rows
  // of the transposed output
  double g[KB];
#pragma unroll
  for (int l = 0; l < KB; ++l) g[l] = 0.0;  // g[l] = y_{i+1+l}
  double* __restrict__ out = a.Out + (size_t)b * a.o_stride;
  const int top = n - 1;
#pragma unroll
  for (int r = 0; r < kCh; ++r) cur[r] = w[(size_t)max(top - r, 0) * a.n_cols];
  int i = top;
  for (int rb = top / kCols; rb >= 0; --rb) {
    const int r0 = rb * kCols;
    // rows i .. r0 of this block, in chunks of kCh (the chunk boundaries follow
    // i, which steps down by one per row from the top)
    while (i >= r0) {
#pragma unroll
      for (int r = 0; r < kCh; ++r) nxt[r] = w[(size_t)max(i - kCh - r, 0) * a.n_cols];
#pragma unroll
      for (int r = 0; r < kCh; ++r) {
        const int ii = i - r;
        if (ii >= r0) {
          const double* c = Lb + (size_t)ii * (KB + 1);
          double acc = cur[r];
#pragma unroll
          for (int l = KB; l >= 1; --l) acc = fma(-c[l], g[l - 1], acc);
          const double v = acc * c[0];
#pragma unroll
          for (int l = KB - 1; l >= 1; --l) g[l] = g[l - 1];
          g[0] = v;
          tile[ii - r0][lane] = v;
        }
      }
      // rows consumed in this chunk: all kCh, or up to the block's first row
      const int used = min(kCh, i - r0 + 1);
      if (used == kCh) {
#pragma unroll
        for (int r = 0; r < kCh; ++r) cur[r] = nxt[r];
      } else {
        // the chunk straddles the block boundary: realign the register chunk
        // at the next row to solve (i - used) and refetch it
#pragma unroll
        for (int r = 0; r < kCh; ++r) cur[r] = w[(size_t)max(i - used - r, 0) * a.n_cols];
      }
      i -= used;
    }
    __syncthreads();
    // rows r0 .. r0 + 63 of columns col0 .. col0 + 63  ->  out[col][r0 + lane]
    const int row = r0 + lane;
    if (row < n) {
      for (int c = 0; c < kCols && col0 + c < a.n_cols; ++c)
        out[(size_t)(col0 + c) * a.ld_o + row] = unmatched ? __builtin_nan("") : tile[lane][c];
    }
    __syncthreads();
  }
}

int launch_bchol(const BcholArgs& a, int kb, int batch, hipStream_t s) {
  if (a.n_rows < 1 || a.n_cols < 1 || batch < 1) return 0;
  const dim3 grid((a.n_cols + kCols - 1) / kCols, batch);
  switch (kb) {
    case 1: hipLaunchKernelGGL(bchol_kernel<1>, grid, dim3(kCols), 0, s, a); break;
    case 2: hipLaunchKernelGGL(bchol_kernel<2>, grid, dim3(kCols), 0, s, a); break;
    case 3: hipLaunchKernelGGL(bchol_kernel<3>, grid, dim3(kCols), 0, s, a); break;
    case 4: hipLaunchKernelGGL(bchol_kernel<4>, grid, dim3(kCols), 0, s, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mofem

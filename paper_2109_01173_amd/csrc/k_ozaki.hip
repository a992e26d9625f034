// FP64-accurate spectral transforms on INT8 matrix cores (error-free slices).
//
// The four products of the preconditioner inverse of Sec. 4 (eqs. (55)-(59)),
//     Z = V_s ((V_s^T R V_t) ./ D) V_t^T,
// in the same "NT" form as k_gemm.hip, C[m][n] = sum_k A[m][k] B[n][k], but
// evaluated from exact integer products: the error-free splitting of matrix
// products by Ozaki, Ogita, Oishi and Rump (Numer. Algorithms 59 (2012)),
// with 8-bit integer slices as Ootomo, Ozaki and Yokota adapted it to integer
// matrix units (Int. J. High Perform. Comput. Appl. 38 (2024)).
//
// Slices.  Every row x of an operand (both operands are contiguous along k)
// gets the smallest exponent e with max_k |x_k| <= (127/128) 2^e (0 for a
// zero row); x' = x 2^-e is cut into S signed base-128 digits, each the
// nearest integer (ties to even) to 128 times the remainder so far:
// d_p = rint(2^7 x'_{p-1}), x'_p = 2^7 x'_{p-1} - d_p, so |d_1| <= 127,
// |d_p| <= 64 after it, every step is exact in FP64, and
// x = 2^e (sum_p d_p 2^-7p + r) with |r| <= 2^-7S / 2 (nearest digits leave
// unbiased remainders: 6-8x less error than truncated ones).
// Product.  With A's digits a_p and B's digits b_q,
//     C[m][n] ~ 2^(ea_m + eb_n) sum_{p + q <= S + 1} 2^-7(p+q) (a_p b_q^T)[m][n],
// every a_p b_q^T is an exact int32 product on v_mfma_i32_16x16x64_i8, and
// the products of one diagonal p + q = d share the scale 2^-7d, so they are
// summed in one int32 accumulator per diagonal (at most S K 127^2 < 2^31 for
// K <= 16384 with S = 7).  The truncation error per entry is below
// (S + 1) 2^-7S K 2^(ea_m + eb_n) (2^-46 K 2^(ea + eb) for S = 7; about
// 2e-14 of the largest entry for random operands with K = 2048); the
// epilogue converts the S diagonal sums to FP64, adds them from the smallest
// scale up, applies 2^(ea_m + eb_n), and divides by D like the FP64 kernel.
//
// Layout: the slices of an item are [S][pad_up(rows)][pad_up(K)] bytes (row
// length pad_up(K), zeros in the padding), the exponents [pad_up(rows)]
// ints.  Block tile 64 x 64 (4 waves of 32 x 32, 2 x 2 MFMA tiles), k tile
// 64 (one MFMA step), all 2 S slice tiles of a k tile in one LDS stage
// (2 S x 4 KB) filled by direct global -> LDS loads and reloaded once every
// wave holds the current tile's fragments in registers (as the BF16
// kernel); the products of the first A digit are issued before that
// barrier, so they overlap the other waves' fragment reads (7 % faster
// than issuing every product after it).  LDS rows of 64 bytes with their
// 16-byte chunks XOR-swizzled by ((row / 2) ^ (row / 4)) % 4: any 8
// consecutive rows of a fragment read cover a 128-byte bank window once and
// any 16 a 256-byte window (rocprofv3 SQ_LDS_BANK_CONFLICT: none; the swizzle
// (row / 4) % 4 conflicted in half the LDS-active cycles).  Within an MFMA
// the hardware's assignment of k to lanes is the same for both operands, and
// integer sums do not depend on their order, so the fragments are read with
// any common k order.
#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

typedef int i4_t __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ void lds_load16(const signed char* src, signed char* dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// One block per (padded) row of an item: exponent, then S digit planes.  Rows
// of at most 2048 padded entries are read once into registers (eight per
// thread, 16-byte loads where the row start allows) and leave as one 8-byte
// store per digit plane and thread; longer rows take two passes.
template <int S>
__global__ __launch_bounds__(256) void slice_rows_kernel(const double* __restrict__ X, long long xs, int ld, int M,
                                                         int K, signed char* __restrict__ out, long long os,
                                                         int* __restrict__ ex, long long es, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int row = blockIdx.x, tid = threadIdx.x;
  const int Kp = pad_up(K), Mp = pad_up(M);
  const bool live = row < M;
  const double* __restrict__ x = X + (size_t)b * xs + (size_t)(live ? row : 0) * ld;
  // rows of at most 2048 (padded) entries stay in registers: eight
  // consecutive entries per thread, read once with 16-byte loads
  __shared__ double wmax[4];
  if (Kp <= 2048) {
    double v[8];
    const int k8 = 8 * tid;
    const bool al = (((size_t)x) % 16) == 0;  // the row start (uniform in the block)
    double mx = 0.0;
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      const int k = k8 + u;
      if (live && al && k + 1 < K) {
        const double2 w = *reinterpret_cast<const double2*>(x + k);
        v[u] = w.x;
        v[u + 1] = w.y;
      } else {
        v[u] = (live && k < K) ? x[k] : 0.0;
        v[u + 1] = (live && k + 1 < K) ? x[k + 1] : 0.0;
      }
      mx = fmax(mx, fmax(fabs(v[u]), fabs(v[u + 1])));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) wmax[tid >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    int e = 0;
    if (mx > 0.0) {
      const double f = frexp(mx, &e);
      if (f > 127.0 / 128.0) ++e;
    }
    if (tid == 0) ex[(size_t)b * es + row] = e;
    if (k8 >= Kp) return;
    signed char* __restrict__ o = out + (size_t)b * os + (size_t)row * Kp;
    const size_t plane = (size_t)Mp * Kp;
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ldexp(v[u], -e);
#pragma unroll
    for (int p = 0; p < S; ++p) {
      unsigned long long w = 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double y = v[u] * 128.0;
        const double d = rint(y);
        v[u] = y - d;
        w |= ((unsigned long long)((unsigned)(int)d & 0xFFu)) << (8 * u);
      }
      *reinterpret_cast<unsigned long long*>(o + p * plane + k8) = w;
    }
    return;
  }
  // 1. row maximum of |x|
  double mx = 0.0;
  if (live)
    for (int k = tid; k < K; k += 256) mx = fmax(mx, fabs(x[k]));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((tid & 63) == 0) wmax[tid >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  int e = 0;
  if (mx > 0.0) {
    const double f = frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
    if (f > 127.0 / 128.0) ++e;      // so that |2^7 x 2^-e| <= 127
  }
  if (tid == 0) ex[(size_t)b * es + row] = e;
  // 2. digits, four consecutive k per thread and plane (one 32-bit store each)
  signed char* __restrict__ o = out + (size_t)b * os + (size_t)row * Kp;
  const size_t plane = (size_t)Mp * Kp;
  for (int k4 = 4 * tid; k4 < Kp; k4 += 1024) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (live && k4 + u < K) ? ldexp(x[k4 + u], -e) : 0.0;
#pragma unroll
    for (int p = 0; p < S; ++p) {
      unsigned w = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double y = v[u] * 128.0;
        const double d = rint(y);
        v[u] = y - d;
        w |= ((unsigned)(int)d & 0xFFu) << (8 * u);
      }
      *reinterpret_cast<unsigned*>(o + p * plane + k4) = w;
    }
  }
}

template <int S, int OMODE>
__global__ __launch_bounds__(256, 2) void gemm_i8_kernel(GemmArgs g) {
  constexpr int TB = 64, BK = 64;
  constexpr int TILE = TB * BK;  // bytes of one slice tile
  __shared__ __attribute__((aligned(16))) signed char lds[2 * S * TILE];

  const int b = blockIdx.y;
  if (g.active && !g.active[b]) return;
  const int Mp = pad_up(g.M), Np = pad_up(g.N), Kp = pad_up(g.K);
  const int tm = Mp / TB, tn = Np / TB;
  int tr, tc;
  grouped_tile(blockIdx.x, tm, tn, 8, &tr, &tc);
  const int m0 = tr * TB, n0 = tc * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int wv = __builtin_amdgcn_readfirstlane(wave);

  const signed char* __restrict__ Ag = g.a_item ? (const signed char*)g.a_item[b] : g.a_i8 + (size_t)b * g.a_stride;
  const signed char* __restrict__ Bg = g.b_item ? (const signed char*)g.b_item[b] : g.b_i8 + (size_t)b * g.b_stride;
  const size_t a_plane = (size_t)Mp * Kp, b_plane = (size_t)Np * Kp;

  // One wave instruction moves 16 rows x 64 bytes of one slice tile: wave w
  // loads rows 16 w .. 16 w + 15 of all 2 S slice tiles.  Lane (row, slot)
  // fetches the global chunk that the swizzle places in that slot (the
  // swizzle of row 16 w + lrow depends on lrow only).
  const int lrow = lane >> 2;
  const int lchunk = (lane & 3) ^ (((lrow >> 1) ^ (lrow >> 2)) & 3);
  const unsigned a_off = (unsigned)((m0 + 16 * wv + lrow) * Kp + lchunk * 16);
  const unsigned b_off = (unsigned)((n0 + 16 * wv + lrow) * Kp + lchunk * 16);
  signed char* const lds_w = lds + wv * 16 * BK;
  auto dma = [&](int k0) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) {
      lds_load16(Ag + sl * a_plane + k0 + a_off, lds_w + sl * TILE);
      lds_load16(Bg + sl * b_plane + k0 + b_off, lds_w + (S + sl) * TILE);
    }
  };
  // fragment of tile row block rb (16 rows from rb) of a slice tile
  auto frag = [&](const signed char* tile, int rb) {
    const int r = rb + (lane & 15);
    const int c = (lane >> 4) ^ (((r >> 1) ^ (r >> 2)) & 3);
    return *reinterpret_cast<const i4_t*>(tile + r * BK + c * 16);
  };

  i4_t acc[S][2][2];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[d][i][j] = (i4_t){0, 0, 0, 0};

  const int nk = Kp / BK;
  dma(0);
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // this wave's loads of tile kt landed
    __syncthreads();                          // and every wave's
    i4_t fa[S][2], fb[S][2];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[q][j] = frag(lds + (S + q) * TILE, wn * 32 + j * 16);
#pragma unroll
    for (int p = 0; p < S; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[p][i] = frag(lds + p * TILE, wm * 32 + i * 16);
    // the products of the first A digit run before the stage is released
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[q][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[0][i], fb[q][j], acc[q][i][j], 0, 0, 0);
    __syncthreads();  // every wave holds its fragments: the stage is free
    if (kt + 1 < nk) dma((kt + 1) * BK);
#pragma unroll
    for (int p = 1; p < S; ++p)
#pragma unroll
      for (int q = 0; q < S - p; ++q)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[p + q][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[p][i], fb[q][j], acc[p + q][i][j], 0, 0, 0);
  }

  // epilogue: acc[d][i][j][r] = diagonal p + q = d + 2 of C[row][col],
  // row = 4 (lane / 16) + r, col = lane % 16 within the 16 x 16 tile
  const double s = g.item_scale ? g.item_scale[b] : 1.0;
  const int* __restrict__ ea = g.a_exp_item ? g.a_exp_item[b] : g.a_exp + (size_t)b * g.a_exp_stride;
  const int* __restrict__ eb = g.b_exp_item ? g.b_exp_item[b] : g.b_exp + (size_t)b * g.b_exp_stride;
  const double* __restrict__ lam = g.lam_item ? g.lam_item[b] : g.lam;
  const double* __restrict__ mu = g.mu_item ? g.mu_item[b] : g.mu;
  double* __restrict__ C = g.c64 + (size_t)b * g.c_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
        const bool in = row < g.M && col < g.N;
        double v = 0.0;
#pragma unroll
        for (int d = S - 1; d >= 0; --d) v += (double)acc[d][i][j][r] * __builtin_ldexp(1.0, -7 * (d + 2));
        v = ldexp(v, ea[row] + eb[col]);
        v *= g.out_scale;
        if (g.divide) {
          const double l = lam[min(row, g.M - 1)], m = mu[min(col, g.N - 1)];
          v /= g.alpha + s * (g.beta_s * l + g.beta_t * m + g.delta * l * m);
        }
        if (!in) v = 0.0;
        if (OMODE == O_PAD_T) C[(size_t)col * Mp + row] = v;
        else if (OMODE == O_PAD_N) C[(size_t)row * Np + col] = v;
        else if (in) C[(size_t)row * g.N + col] = v;
      }
}

}  // namespace

int launch_slice_rows(const double* X, long long xs, int ld, int M, int K, signed char* out, long long os, int* ex,
                      long long es, int batch, const int* active, hipStream_t s) {
  if (M < 1 || K < 1 || ld < K || pad_up(K) > kOzMaxK) return -1;
  hipLaunchKernelGGL((slice_rows_kernel<kOzSlices>), dim3(pad_up(M), batch), dim3(256), 0, s, X, xs, ld, M, K, out,
                     os, ex, es, active);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_gemm_i8(const GemmArgs& g, int omode, int batch, hipStream_t s) {
  if (pad_up(g.K) > kOzMaxK) return -1;
  dim3 grid((pad_up(g.M) / 64) * (pad_up(g.N) / 64), batch);
  if (omode == O_PAD_T)
    hipLaunchKernelGGL((gemm_i8_kernel<kOzSlices, O_PAD_T>), grid, dim3(256), 0, s, g);
  else if (omode == O_PAD_N)
    hipLaunchKernelGGL((gemm_i8_kernel<kOzSlices, O_PAD_N>), grid, dim3(256), 0, s, g);
  else if (omode == O_F64_RAW)
    hipLaunchKernelGGL((gemm_i8_kernel<kOzSlices, O_F64_RAW>), grid, dim3(256), 0, s, g);
  else
    return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mofem

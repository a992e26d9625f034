// Dense two-sided spectral transforms of the preconditioner on MFMA.
//
// The preconditioner inverse of Sec. 4 (eqs. (55)-(59)), used as the
// single-term preconditioner of Sec. 5 (eq. (80)) and Sec. 6 (eq. (95)),
//     Z = V_s ((V_s^T R V_t) ./ D) V_t^T,
// is evaluated as four "NT" products C[m][n] = sum_k A[m][k] B[n][k] whose
// operands are all contiguous along k:
//     T' = (R V_t)^T       A = R (padded copy)  B = V_t^T   out transposed
//     S' = (V_s^T T ./ D)^T A = V_s^T   B = T'      out transposed, divide by D
//     W  = V_s S            A = V_s      B = S'      out row-major
//     Z  = W V_t^T          A = W        B = V_t     out FP64 (the caller's R/Z layout)
// so neither operand ever needs a transpose in LDS.  D is formed in the
// epilogue from the eigenvalue vectors (never stored).
//
// Precisions:
//   GEMM_F64     v_mfma_f64_16x16x4_f64, FP64 operands and accumulation.
//   GEMM_F32     v_mfma_f32_16x16x4_f32, FP32 operands and accumulation.
//   GEMM_BF16X3  v_mfma_f32_16x16x32_bf16 with split operands x = hi + lo
//                (hi = bf16(x), lo = bf16(x - hi)); A B ~ Ah Bh + Ah Bl + Al Bh,
//                FP32 accumulation, FP32-level accuracy.
//   GEMM_BF16X2  one operand split, the other taken in BF16: two products.
//                The data operand split with the eigenbasis exactly
//                representable in BF16 (the preconditioner is defined with
//                the BF16-rounded basis), or the eigenbasis split with plain
//                BF16 data (the first back transform of the forward-BF16
//                variant that rounds S).
//   GEMM_BF16    the hi * hi product only.
// A transform writes the lo half of a split output only when its consumer
// reads it (c_lo set).
// LDS operand rows hold BK values with their 16-byte chunks XOR-swizzled by
// row, so the 16 rows read by one ds_read_b128 fall on distinct banks.
// Tiling: 256 threads = 4 waves, block tile 128 x 128, each wave 64 x 64
// (4 x 4 MFMA tiles of 16 x 16), or 64 x 64 blocks of 32 x 32 wave tiles for
// grids too small to fill the chip (picked per shape, see mofem_prec_tune);
// k tiles of 16 (FP64), 32 (FP32), 64 (BF16).
// The loads of the next k tile overlap the MFMAs of the current one (BF16:
// direct global -> LDS loads issued once the current tile's fragments are in
// registers; FP32 and FP64: through registers); in the split products the
// three passes run one after the other over all 16 accumulators, so
// back-to-back MFMAs are independent.
// Block order is XCD-aware: each XCD takes a compact block of tiles of one
// item, about four (128 tiles) or eight (64 tiles) tile rows high; the BF16
// products with 128 tiles take 8 x 8 blocks where the grid splits evenly.
// Intermediates are padded to multiples of 128 in both dimensions and the
// epilogue writes zeros into the padding, so consumers read whole tiles
// without bounds checks.
#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned short us8_t __attribute__((ext_vector_type(8)));


__device__ __forceinline__ unsigned short bf16_bits(float x) {
  __bf16 h = (__bf16)x;   // round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_to_f(unsigned short u) {
  return __uint_as_float(((unsigned)u) << 16);
}
__device__ __forceinline__ void split_bf16(float x, unsigned short* hi, unsigned short* lo) {
  unsigned short h = bf16_bits(x);
  *hi = h;
  *lo = bf16_bits(x - bf16_to_f(h));
}


// ------------------------------------------------------------------------------
// FP64
// ------------------------------------------------------------------------------
template <int OMODE, int BK = 16, int WT = 4>
__global__ __launch_bounds__(256, 2) void gemm_f64_kernel(GemmArgs g) {
  constexpr int TB = 32 * WT;  // block tile TB x TB: 4 waves of WT x WT MFMA tiles
  constexpr int LDS_K = BK + 1;
  __shared__ double As[TB][LDS_K];
  __shared__ double Bs[TB][LDS_K];

  const int b = blockIdx.y;
  if (g.active && !g.active[b]) return;
  // tiles cover the padded extent, so every padded output entry is written
  const int tm = pad_up(g.M) / TB, tn = pad_up(g.N) / TB;
  int tr, tc;
  grouped_tile(blockIdx.x, tm, tn, TB == 128 ? 4 : 8, &tr, &tc);
  const int m0 = tr * TB, n0 = tc * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int lda = pad_up(g.K);
  const int ldb = pad_up(g.K);
  const double* __restrict__ A = g.a_item ? (const double*)g.a_item[b] : g.a64 + (size_t)b * g.a_stride;
  const double* __restrict__ B = g.b_item ? (const double*)g.b_item[b] : g.b64 + (size_t)b * g.b_stride;
  const double* __restrict__ lam = g.lam_item ? g.lam_item[b] : g.lam;
  const double* __restrict__ mu = g.mu_item ? g.mu_item[b] : g.mu;

  // global -> register staging: TPR threads per tile row, HK values each
  constexpr int TPR = 256 / TB;
  constexpr int HK = BK / TPR;
  const int lrow = tid / TPR, lk = (tid % TPR) * HK;
  double ra[HK], rb[HK];
  auto load_tile = [&](int k0) {
    const int arow = m0 + lrow;
#pragma unroll
    for (int e = 0; e < HK; ++e) {
      const int kk = k0 + lk + e;
      ra[e] = A[(size_t)arow * lda + kk];
      rb[e] = B[(size_t)(n0 + lrow) * ldb + kk];
    }
  };

  d4_t acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = (d4_t){0.0, 0.0, 0.0, 0.0};

  const int nk = (g.K + BK - 1) / BK;
  load_tile(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < HK; ++e) {
      As[lrow][lk + e] = ra[e];
      Bs[lrow][lk + e] = rb[e];
    }
    __syncthreads();
    if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      double av[WT], bv[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) av[i] = As[wm * (16 * WT) + i * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < WT; ++j) bv[j] = Bs[wn * (16 * WT) + j * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: acc[i][j][r] = C[row][col], row = 4 r + lane/16, col = lane%16 (per 16x16 tile)
  const double s = g.item_scale ? g.item_scale[b] : 1.0;
  double* __restrict__ C = g.c64 + (size_t)b * g.c_stride;
  const int Mp = pad_up(g.M), Np = pad_up(g.N);
  // eigenvalues of the lane's rows and columns, loaded together before the
  // stores (indices clamped; padding entries are zeroed below)
  double el[WT][4], em[WT];
  if (g.divide) {
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) el[i][r] = lam[min(m0 + wm * (16 * WT) + i * 16 + 4 * r + (lane >> 4), g.M - 1)];
#pragma unroll
    for (int j = 0; j < WT; ++j) em[j] = mu[min(n0 + wn * (16 * WT) + j * 16 + (lane & 15), g.N - 1)];
  }
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (16 * WT) + i * 16 + 4 * r + (lane >> 4);
        const int col = n0 + wn * (16 * WT) + j * 16 + (lane & 15);
        const bool in = row < g.M && col < g.N;
        double v = acc[i][j][r] * g.out_scale;
        if (g.divide) {
          const double l = el[i][r], m = em[j];
          v /= g.alpha + s * (g.beta_s * l + g.beta_t * m + g.delta * l * m);
        }
        if (!in) v = 0.0;
        if (OMODE == O_PAD_T) C[(size_t)col * Mp + row] = v;
        else if (OMODE == O_PAD_N) C[(size_t)row * Np + col] = v;
        else if (in) C[(size_t)row * g.N + col] = v;
      }
}

// ------------------------------------------------------------------------------
// FP32: v_mfma_f32_16x16x4_f32, FP32 operands and accumulation
// ------------------------------------------------------------------------------
template <int OMODE, int WT = 4>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmArgs g) {
  constexpr int TB = 32 * WT;  // block tile TB x TB: 4 waves of WT x WT MFMA tiles
  constexpr int BK = 32;
  constexpr int LDS_K = BK + 1;
  __shared__ float As[TB][LDS_K];
  __shared__ float Bs[TB][LDS_K];

  const int b = blockIdx.y;
  if (g.active && !g.active[b]) return;
  // tiles cover the padded extent, so every padded output entry is written
  const int tm = pad_up(g.M) / TB, tn = pad_up(g.N) / TB;
  int tr, tc;
  grouped_tile(blockIdx.x, tm, tn, TB == 128 ? 4 : 8, &tr, &tc);
  const int m0 = tr * TB, n0 = tc * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int Kp = pad_up(g.K);
  const float* __restrict__ A = g.a_item ? (const float*)g.a_item[b] : (const float*)g.a_hi + (size_t)b * g.a_stride;
  const float* __restrict__ B = g.b_item ? (const float*)g.b_item[b] : (const float*)g.b_hi + (size_t)b * g.b_stride;
  const double* __restrict__ lam = g.lam_item ? g.lam_item[b] : g.lam;
  const double* __restrict__ mu = g.mu_item ? g.mu_item[b] : g.mu;

  // global -> register staging: TPR threads per tile row, NV 16-byte loads each
  constexpr int TPR = 256 / TB;
  constexpr int NV = BK / TPR / 4;
  const int lrow = tid / TPR, lk = (tid % TPR) * (BK / TPR);
  f4_t ra[NV], rb[NV];
  auto load_tile = [&](int k0) {
    const f4_t* pa = (const f4_t*)(A + (size_t)(m0 + lrow) * Kp + k0 + lk);
    const f4_t* pb = (const f4_t*)(B + (size_t)(n0 + lrow) * Kp + k0 + lk);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ra[v] = pa[v];
      rb[v] = pb[v];
    }
  };

  f4_t acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};

  const int nk = (g.K + BK - 1) / BK;
  load_tile(0);
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        As[lrow][lk + 4 * v + e] = ra[v][e];
        Bs[lrow][lk + 4 * v + e] = rb[v][e];
      }
    __syncthreads();
    if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      float av[WT], bv[WT];
#pragma unroll
      for (int i = 0; i < WT; ++i) av[i] = As[wm * (16 * WT) + i * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < WT; ++j) bv[j] = Bs[wn * (16 * WT) + j * 16 + (lane & 15)][ks * 4 + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }

  // epilogue: acc[i][j][r] = C[row][col], row = 4*(lane/16) + r, col = lane%16
  const double s = g.item_scale ? g.item_scale[b] : 1.0;
  // divisor D(row, col) = da(row) + db(row) mu(col), da = alpha + s beta_s lam,
  // db = s (beta_t + delta lam), in FP32 like the accumulators; the lane's
  // factors are loaded together before the stores (indices clamped; padding
  // entries are zeroed below)
  float da[WT][4], db[WT][4], dm[WT];
  if (g.divide) {
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double l = lam[min(m0 + wm * (16 * WT) + i * 16 + 4 * (lane >> 4) + r, g.M - 1)];
        da[i][r] = (float)(g.alpha + s * g.beta_s * l);
        db[i][r] = (float)(s * (g.beta_t + g.delta * l));
      }
#pragma unroll
    for (int j = 0; j < WT; ++j) dm[j] = (float)mu[min(n0 + wn * (16 * WT) + j * 16 + (lane & 15), g.N - 1)];
  }
  const float osc = (float)g.out_scale;
  const int Mp = pad_up(g.M), Np = pad_up(g.N);
  float* __restrict__ C32 = (float*)g.c_hi + (size_t)b * g.c_stride;
  double* __restrict__ C64 = g.c64 + (size_t)b * g.c_stride;
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (16 * WT) + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * (16 * WT) + j * 16 + (lane & 15);
        const bool in = row < g.M && col < g.N;
        float v = acc[i][j][r] * osc;
        if (g.divide) v *= __builtin_amdgcn_rcpf(fmaf(db[i][r], dm[j], da[i][r]));
        if (!in) v = 0.f;
        if (OMODE == O_F64_RAW) {
          if (in) C64[(size_t)row * g.N + col] = (double)v;
        } else if (OMODE == O_F32_RAW) {
          if (in) C32[(size_t)row * g.N + col] = v;
        } else {
          const size_t idx = (OMODE == O_PAD_T) ? (size_t)col * Mp + row : (size_t)row * Np + col;
          C32[idx] = v;
        }
      }
}

// ------------------------------------------------------------------------------
// split BF16 (NPROD = 3) and plain BF16 (NPROD = 1), FP32 accumulation
// ------------------------------------------------------------------------------
// MODE: BF_HH   plain BF16                    A_h B_h
//       BF_X3   both operands split            A_l B_h + A_h B_l + A_h B_h
//       BF_X2A  A split, B exact in BF16       A_l B_h + A_h B_h
//       BF_X2B  B split, A exact in BF16       A_h B_l + A_h B_h
enum { BF_HH = 0, BF_X3 = 1, BF_X2A = 2, BF_X2B = 3 };

__device__ __forceinline__ void lds_load16(const unsigned short* src, unsigned short* dst) {
  __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// k tiles reach LDS by direct global -> LDS loads (global_load_lds_dwordx4)
// into one LDS stage; the loads of tile kt + 1 start as soon as every wave
// holds tile kt's fragments in registers and run under its MFMAs.  Whole
// 128-byte row pieces per load (k tile 64): a k tile of 32 with two stages
// (64-byte pieces) doubled the L2 requests, kept the texture addresser 72 %
// busy and was 12 % slower; register staging was 7-21 % slower.
template <int MODE, int OMODE, int BK = 64, int MINW = 2, int WT = 4>
__global__ __launch_bounds__(256, MINW) void gemm_bf16_kernel(GemmArgs g) {
  // block tile TB x TB: 4 waves in 2 x 2, each WT x WT MFMA tiles of 16 x 16
  constexpr int TB = 32 * WT;
  // operand rows of BK values, 16-byte chunks XOR-swizzled by row (see sw)
  constexpr int LDS_K = BK;
  static_assert(BK == 64, "the swizzle and the staging assume rows of 64 values");
  constexpr bool ALO = (MODE == BF_X3 || MODE == BF_X2A);
  constexpr bool BLO = (MODE == BF_X3 || MODE == BF_X2B);
  // One LDS buffer: the operand tiles of the main loop, then (padded output)
  // the staging tile of the epilogue, so the output leaves in whole rows.
  constexpr int SLD = TB + 8;  // staging row length (16-byte aligned)
  constexpr int NOP = 2 + (ALO ? 1 : 0) + (BLO ? 1 : 0);
  constexpr int MAIN = NOP * TB * LDS_K;
  constexpr bool RAW = (OMODE == O_F64_RAW || OMODE == O_F32_RAW);
  constexpr int STAGE = RAW ? 0 : TB * SLD;
  __shared__ __attribute__((aligned(16))) unsigned short lds[MAIN > STAGE ? MAIN : STAGE];
  typedef unsigned short Row[LDS_K];
  Row* Ah = reinterpret_cast<Row*>(lds);
  Row* Bh = Ah + TB;
  Row* Al = Bh + TB;                 // used when ALO
  Row* Bl = Al + (ALO ? TB : 0);     // used when BLO
  // element offset of the 16-byte chunk holding k (a multiple of 8) in row r:
  // chunk index XOR (r / 2) % 8 (rocprofv3 SQ_LDS_BANK_CONFLICT: none)
  auto sw = [](int r, int k) { return (((k >> 3) ^ ((r >> 1) % (BK / 8))) << 3); };

  // tiles cover the padded extent, so every padded output entry is written
  const int tm = pad_up(g.M) / TB, tn = pad_up(g.N) / TB;
  // 128-row tiles: 8 x 8 tile blocks per XCD (1-3 % faster than 4 x 8 blocks
  // of two items per XCD, at the same fetched bytes)
  int b, tr, tc;
  item_tile(blockIdx.x, blockIdx.y, tm, tn, TB == 128 ? 4 : 8, TB == 128, &b, &tr, &tc);
  if (g.active && !g.active[b]) return;
  const int m0 = tr * TB, n0 = tc * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int Kp = pad_up(g.K);
  const unsigned short* __restrict__ Ahg =
      g.a_item ? (const unsigned short*)g.a_item[b] : (const unsigned short*)g.a_hi + (size_t)b * g.a_stride;
  const unsigned short* __restrict__ Alg =
      g.a_item ? (const unsigned short*)g.a_item_lo[b] : (const unsigned short*)g.a_lo + (size_t)b * g.a_stride;
  const unsigned short* __restrict__ Bhg =
      g.b_item ? (const unsigned short*)g.b_item[b] : (const unsigned short*)g.b_hi + (size_t)b * g.b_stride;
  const unsigned short* __restrict__ Blg =
      g.b_item ? (const unsigned short*)g.b_item_lo[b] : (const unsigned short*)g.b_lo + (size_t)b * g.b_stride;
  const double* __restrict__ lam = g.lam_item ? g.lam_item[b] : g.lam;
  const double* __restrict__ mu = g.mu_item ? g.mu_item[b] : g.mu;

  constexpr int CPR = BK / 8;  // 16-byte chunks per row

  f4_t acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = (f4_t){0.f, 0.f, 0.f, 0.f};

  const int nk = (g.K + BK - 1) / BK;
  // One wave instruction moves 64 x 16 bytes into RPI consecutive LDS rows;
  // lane (row, slot) fetches the global chunk that the swizzle places in
  // that slot.
  constexpr int TILE = TB * LDS_K;
  constexpr int RPI = 64 / CPR;
  constexpr int IPW = TB / RPI / 4;
  constexpr int KS = BK / 32;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const int irow = lane / CPR, islot = lane % CPR;
  auto dma = [&](int k0) {
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
      const int r0 = (wv * IPW + j) * RPI;
      const int r = r0 + irow;
      const int c = islot ^ ((r >> 1) % CPR);
      const size_t ao = (size_t)(m0 + r) * Kp + k0 + c * 8;
      const size_t bo = (size_t)(n0 + r) * Kp + k0 + c * 8;
      lds_load16(Ahg + ao, lds + r0 * LDS_K);
      lds_load16(Bhg + bo, lds + TILE + r0 * LDS_K);
      if (ALO) lds_load16(Alg + ao, lds + 2 * TILE + r0 * LDS_K);
      if (BLO) lds_load16(Blg + bo, lds + (ALO ? 3 : 2) * TILE + r0 * LDS_K);
    }
  };
  bf8_t fa[KS][WT], fb[KS][WT], fal[KS][WT], fbl[KS][WT];
  auto read = [&]() {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int kq = ks * 32 + (lane >> 4) * 8;
#pragma unroll
      for (int i = 0; i < WT; ++i) {
        const int r = wm * (16 * WT) + i * 16 + (lane & 15);
        fa[ks][i] = __builtin_bit_cast(bf8_t, *(const us8_t*)&Ah[r][sw(r, kq)]);
        if (ALO) fal[ks][i] = __builtin_bit_cast(bf8_t, *(const us8_t*)&Al[r][sw(r, kq)]);
      }
#pragma unroll
      for (int j = 0; j < WT; ++j) {
        const int r = wn * (16 * WT) + j * 16 + (lane & 15);
        fb[ks][j] = __builtin_bit_cast(bf8_t, *(const us8_t*)&Bh[r][sw(r, kq)]);
        if (BLO) fbl[ks][j] = __builtin_bit_cast(bf8_t, *(const us8_t*)&Bl[r][sw(r, kq)]);
      }
    }
  };
  auto mma = [&]() {
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ALO) {
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[ks][i], fb[ks][j], acc[i][j], 0, 0, 0);
      }
      if (BLO) {
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[ks][i], fbl[ks][j], acc[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[ks][i], fb[ks][j], acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_s_setprio(0);
  };
  dma(0);
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);  // this wave's loads of tile kt landed
    __syncthreads();                     // and every wave's
    read();
    __syncthreads();                     // every wave holds its fragments: the stage is free
    if (kt + 1 < nk) dma((kt + 1) * BK);
    mma();
  }

  // epilogue: acc[i][j][r] = C[row][col], row = 4*(lane/16) + r, col = lane%16
  const double s = g.item_scale ? g.item_scale[b] : 1.0;
  // divisor D(row, col) = da(row) + db(row) mu(col), da = alpha + s beta_s lam,
  // db = s (beta_t + delta lam), in FP32 like the accumulators; the lane's
  // factors are loaded together before the stores (indices clamped; padding
  // entries are zeroed below)
  float da[WT][4], db[WT][4], dm[WT];
  if (g.divide) {
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double l = lam[min(m0 + wm * (16 * WT) + i * 16 + 4 * (lane >> 4) + r, g.M - 1)];
        da[i][r] = (float)(g.alpha + s * g.beta_s * l);
        db[i][r] = (float)(s * (g.beta_t + g.delta * l));
      }
#pragma unroll
    for (int j = 0; j < WT; ++j) dm[j] = (float)mu[min(n0 + wn * (16 * WT) + j * 16 + (lane & 15), g.N - 1)];
  }
  const float osc = (float)g.out_scale;
  double* __restrict__ C64 = g.c64 + (size_t)b * g.c_stride;
  float* __restrict__ C32r = (float*)g.c_hi + (size_t)b * g.c_stride;  // O_F32_RAW
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (16 * WT) + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * (16 * WT) + j * 16 + (lane & 15);
        const bool in = row < g.M && col < g.N;
        float v = acc[i][j][r] * osc;
        if (g.divide) v *= __builtin_amdgcn_rcpf(fmaf(db[i][r], dm[j], da[i][r]));
        if (!in) v = 0.f;
        if (OMODE == O_F64_RAW) {
          if (in) C64[(size_t)row * g.N + col] = (double)v;
        } else if (OMODE == O_F32_RAW) {
          if (in) C32r[(size_t)row * g.N + col] = v;
        } else {
          acc[i][j][r] = v;  // the FP32 value to split
        }
      }
  if constexpr (!RAW) {
    // Padded split output through LDS: pass 0 writes hi, pass 1 lo.  In
    // LDS the tile is laid out as the output rows (C^T rows for O_PAD_T),
    // then every thread stores whole 16-byte pieces of those rows.
    const int Mp = pad_up(g.M), Np = pad_up(g.N);
    unsigned short* __restrict__ Cg[2] = {(unsigned short*)g.c_hi + (size_t)b * g.c_stride,
                                          (unsigned short*)g.c_lo + (size_t)b * g.c_stride};
    __syncthreads();  // every wave is done with the operand tiles
    // the lo half is written when the consumer reads it (c_lo set)
    const int passes = g.c_lo ? 2 : 1;
    for (int pass = 0; pass < passes; ++pass) {
#pragma unroll
      for (int i = 0; i < WT; ++i)
#pragma unroll
        for (int j = 0; j < WT; ++j) {
          const int rl = wm * (16 * WT) + i * 16 + 4 * (lane >> 4);  // first of 4 consecutive tile rows
          const int cl = wn * (16 * WT) + j * 16 + (lane & 15);
          unsigned short u[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float f = acc[i][j][r];
            const unsigned short h = bf16_bits(f);
            u[r] = pass == 0 ? h : bf16_bits(f - bf16_to_f(h));
          }
          if (OMODE == O_PAD_T) {
            // C^T row cl holds C[rl .. rl+3][cl] contiguously: one 8-byte write
            const unsigned long long packed = (unsigned long long)u[0] | ((unsigned long long)u[1] << 16) |
                                              ((unsigned long long)u[2] << 32) | ((unsigned long long)u[3] << 48);
            *reinterpret_cast<unsigned long long*>(&lds[cl * SLD + rl]) = packed;
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[(rl + r) * SLD + cl] = u[r];
          }
        }
      __syncthreads();
      // TB rows of TB values in 16-byte pieces, TB * TB / 2048 per thread
      unsigned short* __restrict__ C = Cg[pass];
#pragma unroll
      for (int v = 0; v < TB * TB / 2048; ++v) {
        const int idx = tid + 256 * v;
        const int sr = idx / (TB / 8), ch = (idx % (TB / 8)) * 8;
        const us8_t val = *reinterpret_cast<const us8_t*>(&lds[sr * SLD + ch]);
        const size_t o = (OMODE == O_PAD_T) ? (size_t)(n0 + sr) * Mp + m0 + ch : (size_t)(m0 + sr) * Np + n0 + ch;
        *reinterpret_cast<us8_t*>(C + o) = val;
      }
      __syncthreads();  // before the next pass overwrites the staging tile
    }
  }
}

template <int OMODE, int WT>
static void launch_mode(const GemmArgs& g, int prec, int batch, hipStream_t s) {
  constexpr int TB = 32 * WT;
  dim3 grid((pad_up(g.M) / TB) * (pad_up(g.N) / TB), batch);
  if (prec == GEMM_F64) {
    if constexpr (OMODE != O_F32_RAW) hipLaunchKernelGGL((gemm_f64_kernel<OMODE, 16, WT>), grid, dim3(256), 0, s, g);
  } else if (prec == GEMM_F32)
    hipLaunchKernelGGL((gemm_f32_kernel<OMODE, WT>), grid, dim3(256), 0, s, g);
  else if (prec == GEMM_BF16X3)
    hipLaunchKernelGGL((gemm_bf16_kernel<BF_X3, OMODE, 64, 2, WT>), grid, dim3(256), 0, s, g);
  else if (prec == GEMM_BF16X2 && g.split_a)
    hipLaunchKernelGGL((gemm_bf16_kernel<BF_X2A, OMODE, 64, 2, WT>), grid, dim3(256), 0, s, g);
  else if (prec == GEMM_BF16X2)
    hipLaunchKernelGGL((gemm_bf16_kernel<BF_X2B, OMODE, 64, 2, WT>), grid, dim3(256), 0, s, g);
  else
    // three waves per SIMD (at most 168 VGPRs): measured 15-20 % faster than two
    hipLaunchKernelGGL((gemm_bf16_kernel<BF_HH, OMODE, 64, 3, WT>), grid, dim3(256), 0, s, g);
}

int launch_gemm(const GemmArgs& g, int prec, int omode, int batch, int tile, hipStream_t s) {
  if (prec != GEMM_F64 && prec != GEMM_F32 && prec != GEMM_BF16 && prec != GEMM_BF16X3 && prec != GEMM_BF16X2)
    return -1;
  if (tile != 64 && tile != 128) return -1;
  const bool big = tile == 128;
  if (omode == O_PAD_T) big ? launch_mode<O_PAD_T, 4>(g, prec, batch, s) : launch_mode<O_PAD_T, 2>(g, prec, batch, s);
  else if (omode == O_PAD_N) big ? launch_mode<O_PAD_N, 4>(g, prec, batch, s) : launch_mode<O_PAD_N, 2>(g, prec, batch, s);
  else if (omode == O_F64_RAW) big ? launch_mode<O_F64_RAW, 4>(g, prec, batch, s) : launch_mode<O_F64_RAW, 2>(g, prec, batch, s);
  else if (omode == O_F32_RAW && prec != GEMM_F64)
    big ? launch_mode<O_F32_RAW, 4>(g, prec, batch, s) : launch_mode<O_F32_RAW, 2>(g, prec, batch, s);
  else return -1;
  return 0;
}

// Raw FP64 items (M x K, row length K) -> padded operand (pad(M) x pad(K)),
// FP64, FP32 or split BF16 (hi, and lo unless olo is null), zeros in the padding.  One block per padded
// row; consecutive threads take consecutive columns (coalesced both ways).
__global__ __launch_bounds__(256) void pad_operand_kernel(const double* __restrict__ A, long long a_stride, int M,
                                                          int K, double* __restrict__ o64, float* __restrict__ o32,
                                                          unsigned short* __restrict__ ohi,
                                                          unsigned short* __restrict__ olo, long long o_stride,
                                                          int split, const int* active) {
  const int b = blockIdx.y;
  if (active && !active[b]) return;
  const int row = blockIdx.x;
  const int Kp = pad_up(K);
  const double* a = A + (size_t)b * a_stride;
  const size_t obase = (size_t)b * o_stride + (size_t)row * Kp;
  for (int c = threadIdx.x; c < Kp; c += 256) {
    const double x = (row < M && c < K) ? a[(size_t)row * K + c] : 0.0;
    if (split) {
      unsigned short hi, lo;
      split_bf16((float)x, &hi, &lo);
      ohi[obase + c] = hi;
      if (olo) olo[obase + c] = lo;
    } else if (o32) {
      o32[obase + c] = (float)x;
    } else {
      o64[obase + c] = x;
    }
  }
}

int launch_pad_operand(const double* A, long long a_stride, int M, int K, double* o64, float* o32,
                       unsigned short* ohi, unsigned short* olo, long long o_stride, int split, int batch,
                       const int* active, hipStream_t s) {
  hipLaunchKernelGGL(pad_operand_kernel, dim3(pad_up(M), batch), dim3(256), 0, s, A, a_stride, M, K, o64, o32, ohi,
                     olo, o_stride, split, active);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mofem

// Multiterm banded operator apply  Y = sum_t c_t L_t X R_t  (FP64).
//
// This is the matrix-oriented operator of Sec. 5, eq. (73) (lumped: eq.
// (75); IMEX: eqs. (91)-(92); right-hand side: eqs. (74), (93)), applied to
// dense q_s x q_t nodal matrices with banded one-dimensional factors of
// half-width KB.  It reads X once and writes Y once: HBM-bound for small KB.
//
// Design (gfx950, wave64), "scatter" order along the rows:
//  * a block of 4 waves covers 4 adjacent strips of 64 columns (64 - 2 KB
//    outputs each) and TI rows; lanes run along the contiguous t direction,
//    so every row load and store is one coalesced 512-byte access;
//  * an input row x = X(r, :) is read once; the 2 KB neighbouring columns of
//    a lane come from the neighbours' registers through DPP wave shifts, and
//    the right products w_t = (x R_t)_j of every term are formed at once with
//    the lane's column of every right band (NT (2KB+1) values held in
//    registers for the whole block);
//  * each w_t is then scattered into the 2 KB + 1 output rows r - KB .. r + KB
//    it feeds, y_i += L_t[i][r] w_t, kept in a register window of 2 KB + 1
//    partial sums; output row r - KB is complete after input row r and
//    leaves with one coalesced store.  Registers per lane: NT (2KB+1) right
//    coefficients + 2KB+1 partial sums + the prefetch queue (the gather
//    order, which keeps NT (2KB+1) right products per lane, needs about 100
//    more VGPRs at KB = 2 and runs at two waves per SIMD);
//  * the left coefficients L_t[r + e][r] of the block's input rows (the
//    columns of the left bands, laid out transposed on the host) are staged
//    once in LDS and read back as wave-uniform (broadcast) reads;
//  * rows are processed in groups of U = KB (2KB+1) rows, after which the
//    window's rotation, the prefetch slot and the row's position inside its
//    element repeat, so inside a group everything is compile-time (the window
//    moves by register renaming); for P_k element matrices (k >= 2) a column
//    of a left band has only k + 1 (interior node) or 2k + 1 (element
//    vertex) structural non-zeros, and only those are touched;
//  * row loads run PF rows ahead into a register ring; each loaded row keeps
//    its register until it is overwritten (no copies across the loop's back
//    edge, which would force waits on the loads in flight); loads and stores
//    are buffer accesses with a scalar row offset and a fixed per-lane
//    column offset; rows are clamped to the matrix (rows and columns outside
//    it only ever meet zero band coefficients) and the halo lanes' stores
//    carry an out-of-range offset that the hardware drops, as do the stores
//    of output rows outside the matrix (whose coefficients are zero), so the
//    row body has no branches;
//  * an optional fused Frobenius product <X, Y> per item (eq. (77)) is
//    reduced per block and written to a partial-sum array (a second, fixed
//    order pass makes it deterministic);
//  * a later pass of an operator with more terms than one launch takes adds
//    its result to Y (accumulate).
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

constexpr int kBandWaves = 4;

// Rows per unrolled group (a multiple of U = KB (2KB+1), the period of the
// window rotation and of the element phase) and the length of the register
// ring of loaded rows (a divisor of the group, so that every ring slot is a
// compile-time index).  A loaded row stays in its slot until the load of the
// row NQ further overwrites it, PF = NQ - KB - 1 rows ahead: the current row
// and the KB rows before it (the X values of the output rows completing now)
// are always still there, so no value ever has to move between registers.
template <int KB> struct BandRing;
template <> struct BandRing<1> { static constexpr int UG = 12, NQ = 12; };
template <> struct BandRing<2> { static constexpr int UG = 10, NQ = 10; };
template <> struct BandRing<3> { static constexpr int UG = 42, NQ = 14; };
template <> struct BandRing<4> { static constexpr int UG = 36, NQ = 12; };

// Tile configuration.  GG: row groups per block (TI = GG UG rows); zero
// selects the default.
template <int KB, int NT, int GG = 0>
struct BandCfg {
  static constexpr int W = 2 * KB + 1;
  static constexpr int U = KB * W;   // period of window rotation and element phase
  static constexpr int UG = BandRing<KB>::UG;
  static constexpr int NQ = BandRing<KB>::NQ;
  static constexpr int PF = NQ - KB - 1;
  static constexpr int RC = NT * W;  // left coefficients per input row
  // default: about 160 rows per block, at most 36 KB of staged coefficients
  // (four blocks per compute unit fit the LDS)
  static constexpr int G_ROWS = 160 / UG;
  static constexpr int G_LDS = (36 * 1024 / 8 / RC - 2 * KB) / UG;
  static constexpr int G_MIN = G_ROWS < G_LDS ? G_ROWS : G_LDS;
  static constexpr int G = GG > 0 ? GG : (G_MIN < 1 ? 1 : G_MIN);
  static constexpr int TI = G * UG;         // output rows per block
  static constexpr int NR = TI + 2 * KB;    // input rows per block
  static constexpr int SW = 64 - 2 * KB;
  // waves per SIMD the register budget is compiled for (measured register
  // use of the difference-form kernel: one item per lane at most 128 VGPRs up
  // to 5 terms for KB <= 2, 2 (KB = 3) or 1 (KB = 4) terms, at most 168 up to
  // 4 (KB = 3) or 3 (KB = 4) terms; two items per lane up to 168 with 4 terms
  // at KB <= 2, more with 5 or 6; more terms at KB >= 3 run as several passes)
  static constexpr int MINW = (KB <= 2) ? (NT <= 5 ? 4 : 3)
                              : (KB == 3) ? (NT <= 2 ? 4 : 3)
                                          : (NT <= 1 ? 4 : (NT <= 3 ? 3 : 2));
  static constexpr int MINW2 = (KB <= 2 && NT <= 4) ? 3 : 2;
  static_assert(UG % U == 0 && UG % NQ == 0 && PF >= 1, "ring must divide the group period");
  static_assert(NR * RC * 8 <= 64 * 1024, "staged coefficients exceed 64 KB");
};

typedef int i32x2_t __attribute__((ext_vector_type(2)));
// buffer resource over [base, base + bytes): out-of-range offsets read 0 and
// drop stores (word 3: the raw-buffer format of gfx9-family GPUs)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t band_rsrc(const void* base, long long bytes) {
  const int n = bytes > 0x7fffffffLL ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}
__device__ __forceinline__ double band_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void band_store(double v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2_t, v), r, voff, soff, 0);
}
constexpr int kBandDrop = 0x7fffffff;  // a byte offset past every item: the store is dropped

// Telescoped left products.  For an output row i with band coefficients c_k
// on its input rows r_k = i - KB + k (k = 0 .. 2KB) and first possibly
// non-zero k_lo,  sum_k c_k w(r_k) = S_klo w(r_klo) + sum_{k > k_lo} S_k (w(r_k)
// - w(r_{k-1}))  with the suffix sums S_k = sum_{k' >= k} c_k'.  For the
// stiffness-like bands the terms c_k w(r_k) nearly cancel, while the
// differences of the smooth w are small and exact: the rounding error of the
// sum falls from eps sum |c_k w| to about eps sum |S_k (w_k - w_k-1)|.  In the
// scatter order input row s = r_k reaches output i through slot e = 2KB - k;
// k_lo is 0 for element vertices (and general bands) and KB - ph for an
// interior node of element phase ph, whose row couples only its own element.
// Returns whether slot e of an input row of element phase `phase` is the
// first contribution to its output (which takes w itself, the others w - w_prev).
template <int KB, bool PAT>
__device__ constexpr bool first_of(int phase, int e) {
  const int ph_out = (phase + e) % KB;  // element phase of the output row
  const int klo = (!PAT || ph_out == 0) ? 0 : KB - ph_out;
  return e == 2 * KB - klo;
}

// The arrays are separate __restrict__ kernel arguments (not struct members)
// so that the compiler can order the loads freely around the stores to Y.
// IPL items per lane: with IPL = 2 a lane serves the same column of two batch
// items (items 2y and 2y + 1 of block row y), which share the operator, so
// every staged left coefficient read from LDS and every right coefficient in
// registers serves two outputs (the per-item scale must then be 1 for all
// items or absent: it is folded into the shared right coefficients).
template <int KB, int NT, bool PAT, bool ACC, int IPL, int GG>
__global__ __launch_bounds__(64 * kBandWaves, (IPL == 1 ? BandCfg<KB, NT, GG>::MINW : BandCfg<KB, NT, GG>::MINW2))
void band_apply_kernel(
    BandArgs a, const double* __restrict__ X, double* __restrict__ Y, const double* __restrict__ leftT,
    const double* __restrict__ right) {
  using C = BandCfg<KB, NT, GG>;
  constexpr int W = C::W, RC = C::RC, TI = C::TI, NR = C::NR, PF = C::PF, NQ = C::NQ, UG = C::UG;
  __shared__ double lcol[NR * RC];
  __shared__ double dsum[IPL][kBandWaves];

  // the items of this block; an item past the batch or masked off is carried
  // as a copy of a live one whose stores are dropped and whose <X, Y> is not
  // written
  int bi[IPL];
  bool live[IPL];
  int any = -1;
#pragma unroll
  for (int i = 0; i < IPL; ++i) {
    bi[i] = blockIdx.y * IPL + i;
    live[i] = bi[i] < a.batch && !(a.active && !a.active[bi[i]]);
    if (live[i] && any < 0) any = bi[i];
  }
  if (any < 0) return;
#pragma unroll
  for (int i = 0; i < IPL; ++i)
    if (!live[i]) bi[i] = any;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n_sb = (a.qt + kBandWaves * C::SW - 1) / (kBandWaves * C::SW);
  const int n_tiles = n_sb * a.n_rowblk;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  const int sb = tile / a.n_rowblk;
  const int rb = tile - sb * a.n_rowblk;

  const int j = (sb * kBandWaves + wave) * C::SW + lane - KB;  // output column of this lane
  const bool own = (lane >= KB) && (lane < 64 - KB) && (j < a.qt);
  int bcol = j + a.off_t;                                        // input column this lane loads
  bcol = bcol < 0 ? 0 : (bcol >= a.nt_in ? a.nt_in - 1 : bcol);  // clamped: meets zero coefficients

  const int g0 = rb * TI;                         // first output node row of this block
  const int i0 = g0 - a.ph_s;                     // output row of m = 0
  const int a0 = g0 - KB + a.off_s - a.ph_s;      // input row of p = 0

  // stage the left-band columns of the block's NR input rows
  for (int e = threadIdx.x; e < NR * RC; e += 64 * kBandWaves) {
    const int ar = a0 + e / RC;
    lcol[e] = (ar >= 0 && ar < a.ns_in) ? leftT[(size_t)a0 * RC + e] : 0.0;
  }

  // right coefficients of column j, with the per-item scale folded in
  // (unconditional loads from a clamped column, zeroed outside the matrix)
  const double scale = (IPL == 1 && a.item_scale) ? a.item_scale[bi[0]] : 1.0;
  const bool jvalid = (j >= 0) && (j < a.qt);
  const int jc = j < 0 ? 0 : (j >= a.qt ? a.qt - 1 : j);
  double rc[NT][W];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double s = jvalid ? (((a.scaled_mask >> t) & 1) ? scale : 1.0) : 0.0;
#pragma unroll
    for (int d = 0; d < W; ++d) rc[t][d] = s * right[((size_t)t * W + d) * a.qt + jc];
  }

  // one buffer resource per item: rows by a scalar byte offset, the lane's
  // column by a fixed per-lane offset (no per-row address arithmetic)
  __amdgpu_buffer_rsrc_t xr[IPL], yr[IPL];
  int yoff[IPL];
#pragma unroll
  for (int i = 0; i < IPL; ++i) {
    xr[i] = band_rsrc(X + (size_t)bi[i] * a.in_stride, (long long)a.ns_in * a.ld_x * 8);
    yr[i] = band_rsrc(Y + (size_t)bi[i] * a.out_stride, (long long)a.qs * a.ld_y * 8);
    yoff[i] = (own && live[i]) ? j * 8 : kBandDrop;
  }
  const int xoff = bcol * 8;
  const int last_row = a.ns_in - 1;
  const int xrow = a.ld_x * 8, yrow = a.ld_y * 8;
  // rows outside the matrix read as zero (an out-of-range offset): the
  // difference form below needs exact zeros there, not copies of edge rows
  auto load_row = [&](int p, int i) -> double {
    const int r = a0 + p;
    int off = __builtin_amdgcn_readfirstlane(((unsigned)r <= (unsigned)last_row) ? r * xrow : kBandDrop);
    __asm__ volatile("" : "+s"(off));  // formed here, not hoisted for a whole group
    return band_load(xr[i], xoff, off);
  };

  double acc[IPL][W];   // acc[i][e]: partial sum of output m = p - 2KB + e (p = current input row)
  double xq[IPL][NQ];   // loaded rows, slot = p mod NQ, filled PF rows ahead
  double wprev[IPL][NT];  // right products of the previous input row
  double dot[IPL];
#pragma unroll
  for (int i = 0; i < IPL; ++i) {
    dot[i] = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) wprev[i][t] = 0.0;
#pragma unroll
    for (int d = 0; d < W; ++d) acc[i][d] = 0.0;
#pragma unroll
    for (int d = 0; d < NQ; ++d) xq[i][d] = 0.0;
  }
  // prologue: rows 0 .. PF-1 in flight
  StaticFor<0, PF>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
#pragma unroll
    for (int i = 0; i < IPL; ++i) xq[i][p % NQ] = load_row(p, i);
  });
  __syncthreads();  // staged coefficients visible to all four waves

  // input row p (node row g0 - KB + p, element phase p mod KB, ring slot
  // p mod NQ): right products, their scatter into outputs m = p - 2KB + e for
  // e in [max(ELO, dlo), dhi], then the window moves on by one row
  auto input_row = [&](int p, auto q_c, auto ph_c, auto elo_c, double* done) {
    constexpr int qslot = decltype(q_c)::value;
    constexpr int phase = decltype(ph_c)::value;
    constexpr int ELO = decltype(elo_c)::value;
    constexpr int dlo = (!PAT || phase == 0) ? 0 : KB - phase;
    constexpr int dhi = (!PAT || phase == 0) ? 2 * KB : 2 * KB - phase;
    constexpr int elo = dlo > ELO ? dlo : ELO;
    int lofs = __builtin_amdgcn_readfirstlane(p * RC);
    __asm__ volatile("" : "+s"(lofs));  // this row's LDS base, formed here
    const double* lc = lcol + lofs;
    double nb[IPL][W];
#pragma unroll
    for (int i = 0; i < IPL; ++i) {
      // the slot PF rows ahead held row p + PF - NQ = p - KB - 1, no longer needed
      xq[i][(qslot + PF) % NQ] = load_row(p + PF, i);  // clamped: rows past the end are harmless
      nb[i][KB] = xq[i][qslot];
#pragma unroll
      for (int d = KB + 1; d < W; ++d) nb[i][d] = wave_shl1(nb[i][d - 1]);
#pragma unroll
      for (int d = KB - 1; d >= 0; --d) nb[i][d] = wave_shr1(nb[i][d + 1]);
    }
    // neighbour differences: exact for smooth data (close values subtract
    // exactly), so the stiffness-like right products lose no digits
#pragma unroll
    for (int i = 0; i < IPL; ++i)
#pragma unroll
      for (int d = 0; d < W; ++d)
        if (d != KB) nb[i][d] -= nb[i][KB];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      // this term's left coefficients of the row: read once, used by every item
      double cf[W];
#pragma unroll
      for (int e = elo; e <= dhi; ++e) cf[e] = lc[t * W + e];
#pragma unroll
      for (int i = 0; i < IPL; ++i) {
        // w = sum_d R[d] x[d] = sum_{d != KB} R[d] (x[d] - x[KB]) + (sum_d R[d]) x[KB]
        // (the column sum sits in the centre slot)
        double w = rc[t][KB] * nb[i][KB];
#pragma unroll
        for (int d = 0; d < W; ++d)
          if (d != KB) w = fma(rc[t][d], nb[i][d], w);
        // telescoped left product: an output's first input row brings w, every
        // later one w - w_prev, weighted by the suffix sums of the output's row
        const double dw = w - wprev[i][t];
        wprev[i][t] = w;
#pragma unroll
        for (int e = elo; e <= dhi; ++e)
          acc[i][e] = fma(cf[e], first_of<KB, PAT>(phase, e) ? w : dw, acc[i][e]);
      }
    }
#pragma unroll
    for (int i = 0; i < IPL; ++i) {
#pragma unroll
      for (int t = 0; t < NT; ++t) __asm__ volatile("" : "+v"(wprev[i][t]));
      // materialise this row's partial sums here: left free, the compiler
      // sinks the chains of several rows towards their stores and keeps every
      // row's products alive in registers meanwhile
#pragma unroll
      for (int e = 0; e < W; ++e) __asm__ volatile("" : "+v"(acc[i][e]));
      // move the window: acc[i][0] (output p - 2KB) is complete
      done[i] = acc[i][0];
#pragma unroll
      for (int e = 0; e < W - 1; ++e) acc[i][e] = acc[i][e + 1];
      acc[i][W - 1] = 0.0;
    }
  };
  // Each row's work stays together (a scheduling barrier after it): moving
  // the next row's ring load above this row's last read of that slot, or
  // interleaving rows, would hold several rows' values in registers at once.

  // warm-up: input rows 0 .. 2KB-1 feed only outputs m >= 0 (e >= 2KB - p)
  StaticFor<0, 2 * KB>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    double done[IPL];
    input_row(p, std::integral_constant<int, p % NQ>{}, std::integral_constant<int, p % KB>{},
              std::integral_constant<int, 2 * KB - p>{}, done);
    __builtin_amdgcn_sched_barrier(0);
  });

  // main loop: input row p = 2KB + m completes output m (node row g0 + m);
  // output rows outside the matrix (first and last row block) have zero
  // coefficients, so y = 0 there, and their store and load get an
  // out-of-range offset
#pragma unroll 1
  for (int grp = 0; grp < TI / UG; ++grp) {  // (never unrolled: the group body is large)
    StaticFor<0, UG>::run([&](auto pc) {
      constexpr int P = decltype(pc)::value;
      constexpr int p_mod = (2 * KB + P) % NQ;
      const int m = grp * UG + P;
      double y[IPL];
      input_row(2 * KB + m, std::integral_constant<int, p_mod>{}, std::integral_constant<int, P % KB>{},
                std::integral_constant<int, 0>{}, y);
      const int i = i0 + m;
      int yrow_off = __builtin_amdgcn_readfirstlane(((unsigned)i < (unsigned)a.qs) ? i * yrow : kBandDrop);
      __asm__ volatile("" : "+s"(yrow_off));  // one compare, no branch
#pragma unroll
      for (int it = 0; it < IPL; ++it) {
        if constexpr (ACC) y[it] += band_load(yr[it], yoff[it], yrow_off);
        band_store(y[it], yr[it], yoff[it], yrow_off);
        // X of output row i (square operators) is input row p - KB; every lane
        // accumulates, the halo lanes' sums are discarded once at the end
        dot[it] = fma(y[it], xq[it][(p_mod + NQ - KB) % NQ], dot[it]);
      }
      __builtin_amdgcn_sched_barrier(0);
    });
  }

  if (a.dot_partial) {
#pragma unroll
    for (int it = 0; it < IPL; ++it) {
      const double dw = wave_sum(own ? dot[it] : 0.0);
      if (lane == 0) dsum[it][wave] = dw;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IPL; ++it) {
      if (threadIdx.x == 0 && live[it]) {
        double t = 0.0;
        for (int w = 0; w < kBandWaves; ++w) t += dsum[it][w];
        a.dot_partial[(size_t)bi[it] * a.n_partial + tile] = t;
      }
    }
  }
}

template <int KB, int NT, bool ACC, int IPL, int GG = 0>
void launch_kb_nt(const BandArgs& a, int batch, bool pat, hipStream_t s) {
  using C = BandCfg<KB, NT, GG>;
  const int n_sb = (a.qt + kBandWaves * C::SW - 1) / (kBandWaves * C::SW);
  dim3 grid(n_sb * a.n_rowblk, (batch + IPL - 1) / IPL);
  if (pat && KB >= 2)
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, (KB >= 2), ACC, IPL, GG>), grid, dim3(64 * kBandWaves), 0, s, a,
                       a.X, a.Y, a.left, a.right);
  else
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, false, ACC, IPL, GG>), grid, dim3(64 * kBandWaves), 0, s, a, a.X,
                       a.Y, a.left, a.right);
}

// Row groups per block of the small-block variant (a quarter of the default
// rows) for band widths up to 2; launches whose default grid would leave
// compute units idle (few items, small q) take it.  0 where none is compiled
// (KB >= 3, where smaller row blocks measured slower).
template <int KB>
constexpr int band_small_groups() {
  return KB <= 2 ? ((160 / BandRing<KB>::UG) / 4 > 0 ? (160 / BandRing<KB>::UG) / 4 : 1) : 0;
}

// Terms one launch takes for band half-width KB (more run as several passes,
// the later ones accumulating): up to 6 for KB <= 2; up to 4 for KB >= 3,
// where 5 or 6 terms in one launch need more than 256 registers per lane.
constexpr int band_max_pass_terms(int kb) { return kb <= 2 ? 6 : 4; }

// One translation unit per band width compiles these (k_band_kb*.hip); the
// accumulating variants serve the later passes (5 and 6 terms split as
// 3 + 2 and 3 + 3 at KB >= 3; 7 and 8 terms as 4 + 3 and 4 + 4).
#define MOFEM_BAND_INSTANTIATE_NT(KB, NT)                                                 \
  template void launch_kb_nt<KB, NT, false, 1>(const BandArgs&, int, bool, hipStream_t);  \
  template void launch_kb_nt<KB, NT, false, 2>(const BandArgs&, int, bool, hipStream_t);
#define MOFEM_BAND_INSTANTIATE_COMMON(KB)                                                 \
  MOFEM_BAND_INSTANTIATE_NT(KB, 1)                                                        \
  MOFEM_BAND_INSTANTIATE_NT(KB, 2)                                                        \
  MOFEM_BAND_INSTANTIATE_NT(KB, 3)                                                        \
  MOFEM_BAND_INSTANTIATE_NT(KB, 4)                                                        \
  template void launch_kb_nt<KB, 2, true, 1>(const BandArgs&, int, bool, hipStream_t);    \
  template void launch_kb_nt<KB, 3, true, 1>(const BandArgs&, int, bool, hipStream_t);    \
  template void launch_kb_nt<KB, 4, true, 1>(const BandArgs&, int, bool, hipStream_t);
#define MOFEM_BAND_INSTANTIATE_WIDE(KB)                                                   \
  MOFEM_BAND_INSTANTIATE_NT(KB, 5)                                                        \
  MOFEM_BAND_INSTANTIATE_NT(KB, 6)
// the small-block variants (band widths 1 and 2)
#define MOFEM_BAND_SMALL_NT(KB, NT, ACC, IPL) \
  launch_kb_nt<KB, NT, ACC, IPL, band_small_groups<KB>()>(const BandArgs&, int, bool, hipStream_t);
#define MOFEM_BAND_SMALL_LIST(P, KB)                                                                      \
  P MOFEM_BAND_SMALL_NT(KB, 1, false, 1) P MOFEM_BAND_SMALL_NT(KB, 1, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 2, false, 1) P MOFEM_BAND_SMALL_NT(KB, 2, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 3, false, 1) P MOFEM_BAND_SMALL_NT(KB, 3, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 4, false, 1) P MOFEM_BAND_SMALL_NT(KB, 4, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 5, false, 1) P MOFEM_BAND_SMALL_NT(KB, 5, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 6, false, 1) P MOFEM_BAND_SMALL_NT(KB, 6, false, 2)                          \
  P MOFEM_BAND_SMALL_NT(KB, 2, true, 1) P MOFEM_BAND_SMALL_NT(KB, 3, true, 1)                            \
  P MOFEM_BAND_SMALL_NT(KB, 4, true, 1)
#define MOFEM_BAND_INSTANTIATE_SMALL(KB) MOFEM_BAND_SMALL_LIST(template void, KB)

}  // namespace mofem

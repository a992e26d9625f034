// Multiterm banded operator apply  Y = sum_t c_t L_t X R_t  (FP64).
//
// This is the matrix-oriented operator of Sec. 5, eq. (73) (lumped: eq.
// (75); IMEX: eqs. (91)-(92); right-hand side: eqs. (74), (93)), applied to
// dense q_s x q_t nodal matrices with banded one-dimensional factors of
// half-width KB.  It reads X once and writes Y once: HBM-bound.
//
// Design (gfx950, wave64):
//  * a block of 4 waves covers 4 adjacent strips of 64 columns (64 - 2 KB
//    outputs each) and TI rows; lanes run along the contiguous t direction,
//    so every row load and store is one coalesced 512-byte access;
//  * the right products W_t = X R_t need the 2 KB neighbouring columns of a
//    lane: they come from the neighbours' registers through DPP wave shifts;
//  * the lane's column of every right band (NT x (2KB+1) values) sits in
//    registers for the whole block; the products W_t of the last 2KB+1 rows
//    form a register ring; the left coefficients of the block's rows are
//    staged once in LDS (shared by the 4 waves) and read back as
//    wave-uniform (broadcast) reads;
//  * rows are processed in groups of U = KB (2KB+1) rows, after which the
//    ring slot, the row's position inside its element and the prefetch slot
//    repeat, so inside a group everything is compile-time; for P_k element
//    matrices (k >= 2) the left product then touches only the k + 1
//    (interior node) or 2k + 1 (element vertex) structural non-zeros;
//  * row loads run PF rows ahead in a register queue; they read clamped,
//    in-range addresses unconditionally (rows and columns outside the
//    matrix only ever meet zero band coefficients), so the row body has no
//    branches except the output-row check of the first and last row block;
//  * an optional fused Frobenius product <X, Y> per item (eq. (77)) is
//    reduced per block and written to a partial-sum array (a second, fixed
//    order pass makes it deterministic).
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

constexpr int kBandWaves = 4;

// Tile configuration.  GG: row groups per block (TI = GG U rows), SS: groups
// unrolled per loop iteration, PFX: rows in flight per lane (a divisor of
// SS U, so that every queue slot is a compile-time index).  Zero selects the
// default.
template <int KB, int NT, int GG = 0, int SS = 0, int PFX = 0>
struct BandCfg {
  static constexpr int W = 2 * KB + 1;
  static constexpr int U = KB * W;   // period of ring slot and element phase
  static constexpr int RC = NT * W;  // left coefficients per output row
  // default: about 160 rows per block, at most 48 KB of staged coefficients
  static constexpr int G_ROWS = 160 / U;
  static constexpr int G_LDS = (48 * 1024 / 8) / (RC * U);
  static constexpr int G_MIN = G_ROWS < G_LDS ? G_ROWS : G_LDS;
  static constexpr int G_DEF = G_MIN < 1 ? 1 : G_MIN;
  static constexpr int S = SS > 0 ? SS : 1;
  static constexpr int G = GG > 0 ? GG : (G_DEF / S > 0 ? G_DEF / S * S : S);
  static constexpr int TI = G * U;
  static constexpr int SU = S * U;
  // prefetch distance: the largest divisor of S U not above 12 by default
  static constexpr int pf(int d) { return (SU % d == 0) ? d : pf(d - 1); }
  static constexpr int PF = PFX > 0 ? PFX : pf(12);
  static constexpr int SW = 64 - 2 * KB;
  static_assert(G % S == 0, "groups per block must be a multiple of the unroll");
  static_assert(SU % PF == 0, "prefetch distance must divide the unrolled period");
  static_assert(TI * RC * 8 <= 64 * 1024, "staged coefficients exceed 64 KB");
};

// The arrays are separate __restrict__ kernel arguments (not struct members)
// so that the compiler can order the loads freely around the stores to Y.
template <int KB, int NT, bool PAT, int GG, int SS, int PFX>
__global__ __launch_bounds__(256) void band_apply_kernel(BandArgs a, const double* __restrict__ X,
                                                         double* __restrict__ Y, const double* __restrict__ left,
                                                         const double* __restrict__ right) {
  using C = BandCfg<KB, NT, GG, SS, PFX>;
  constexpr int W = C::W, RC = C::RC, TI = C::TI, PF = C::PF, SU = C::SU;
  __shared__ double lcoef[TI * RC];
  __shared__ double dsum[kBandWaves];

  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;
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

  const int g0 = rb * TI;              // first output node row of this block
  const int delta = a.off_s - a.ph_s;  // input row = node row + delta
  const int i0 = g0 - a.ph_s;          // output row of m = 0

  // stage the left coefficients of the block's TI output rows
  for (int e = threadIdx.x; e < TI * RC; e += 64 * kBandWaves) {
    const int i = i0 + e / RC;
    lcoef[e] = (i >= 0 && i < a.qs) ? left[(size_t)i0 * RC + e] : 0.0;
  }

  // right coefficients of column j, with the per-item scale folded in
  const double scale = a.item_scale ? a.item_scale[b] : 1.0;
  const bool jvalid = (j >= 0) && (j < a.qt);
  double rc[NT][W];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double s = ((a.scaled_mask >> t) & 1) ? scale : 1.0;
#pragma unroll
    for (int d = 0; d < W; ++d) rc[t][d] = jvalid ? s * right[((size_t)t * W + d) * a.qt + j] : 0.0;
  }

  const double* Xb = X + (size_t)b * a.in_stride + bcol;
  double* Yb = Y + (size_t)b * a.out_stride + (own ? j : 0);
  const int last_row = a.ns_in - 1;
  auto load_row = [&](int p) -> double {
    int r = g0 - KB + p + delta;
    r = r < 0 ? 0 : (r > last_row ? last_row : r);
    return Xb[(size_t)r * a.ld_x];
  };

  double ring[NT][W];  // W_t of the last W node rows, slot = node mod W
  double xs[W];        // the lane's own X value of the last W node rows
  double xq[PF];       // prefetched rows, slot = p mod PF
  double dot = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int d = 0; d < W; ++d) ring[t][d] = 0.0;
#pragma unroll
  for (int d = 0; d < W; ++d) xs[d] = 0.0;
  // prologue: rows 0 .. PF-1 in flight
  StaticFor<0, PF>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    xq[p % PF] = load_row(p);
  });
  __syncthreads();  // staged coefficients visible to all four waves

  // consume row p (node row g0 - KB + p): right products into its ring slot
  auto right_row = [&](int p, auto slot_c, auto q_c) {
    constexpr int slot = decltype(slot_c)::value;
    constexpr int qslot = decltype(q_c)::value;
    const double xv = xq[qslot];
    xq[qslot] = load_row(p + PF);  // clamped: rows past the end are harmless
    double nb[W];
    nb[KB] = xv;
#pragma unroll
    for (int d = KB + 1; d < W; ++d) nb[d] = wave_shl1(nb[d - 1]);
#pragma unroll
    for (int d = KB - 1; d >= 0; --d) nb[d] = wave_shr1(nb[d + 1]);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d) s = fma(rc[t][d], nb[d], s);
      ring[t][slot] = s;
    }
    xs[slot] = xv;
  };

  // warm-up: node rows g0 - KB .. g0 + KB - 1
  StaticFor<0, 2 * KB>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    right_row(p, std::integral_constant<int, ((p - KB) % W + W) % W>{}, std::integral_constant<int, p % PF>{});
  });

  // main loop: row p = 2KB + grp SU + P completes output node row g = g0 + grp SU + P
  auto group = [&](int grp, auto check_c) {
    constexpr bool CHECK = decltype(check_c)::value;
    StaticFor<0, SU>::run([&](auto pc) {
      constexpr int P = decltype(pc)::value;
      constexpr int slot = (KB + P) % W;
      constexpr int qslot = (2 * KB + P) % PF;
      constexpr int phase = P % KB;
      constexpr int dlo = (!PAT || phase == 0) ? 0 : KB - phase;
      constexpr int dhi = (!PAT || phase == 0) ? 2 * KB : 2 * KB - phase;
      const int m = grp * SU + P;
      right_row(2 * KB + m, std::integral_constant<int, slot>{}, std::integral_constant<int, qslot>{});
      const int i = i0 + m;
      if (!CHECK || (i >= 0 && i < a.qs)) {
        const double* li = lcoef + m * RC;
        // one partial sum per term: short independent FMA chains
        double part[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          part[t] = 0.0;
#pragma unroll
          for (int d = dlo; d <= dhi; ++d) part[t] = fma(li[t * W + d], ring[t][(P + d - KB + W) % W], part[t]);
        }
        double acc = part[0];
#pragma unroll
        for (int t = 1; t < NT; ++t) acc += part[t];
        if (own) Yb[(size_t)i * a.ld_y] = acc;
        dot = fma(own ? acc : 0.0, xs[P % W], dot);
      }
    });
  };
  const bool interior = (i0 >= 0) && (i0 + TI <= a.qs);
  if (interior) {
    for (int grp = 0; grp < C::G / C::S; ++grp) group(grp, std::false_type{});
  } else {
    for (int grp = 0; grp < C::G / C::S; ++grp) group(grp, std::true_type{});
  }

  if (a.dot_partial) {
    dot = wave_sum(dot);
    if (lane == 0) dsum[wave] = dot;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kBandWaves; ++w) t += dsum[w];
      a.dot_partial[(size_t)b * a.n_partial + tile] = t;
    }
  }
}

template <int KB, int NT, int GG = 0, int SS = 0, int PFX = 0>
void launch_kb_nt(const BandArgs& a, int batch, bool pat, hipStream_t s) {
  using C = BandCfg<KB, NT, GG, SS, PFX>;
  const int n_sb = (a.qt + kBandWaves * C::SW - 1) / (kBandWaves * C::SW);
  dim3 grid(n_sb * a.n_rowblk, batch);
  if (pat && KB >= 2)
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, (KB >= 2), GG, SS, PFX>), grid, dim3(64 * kBandWaves), 0, s, a,
                       a.X, a.Y, a.left, a.right);
  else
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, false, GG, SS, PFX>), grid, dim3(64 * kBandWaves), 0, s, a, a.X,
                       a.Y, a.left, a.right);
}

// One translation unit per band width compiles these (k_band_kb*.hip).
#define MOFEM_BAND_INSTANTIATE(KB)                                                   \
  template void launch_kb_nt<KB, 1>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 2>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 3>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 5>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 6>(const BandArgs&, int, bool, hipStream_t);

}  // namespace mofem

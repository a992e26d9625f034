// Multiterm banded operator apply  Y = sum_t c_t L_t X R_t  (FP64).
//
// This is the matrix-oriented operator of Sec. 5, eq. (73) (lumped: eq.
// (75); IMEX: eqs. (91)-(92); right-hand side: eqs. (74), (93)), applied to
// dense q_s x q_t nodal matrices with banded one-dimensional factors of
// half-width KB.  It reads X once and writes Y once: HBM-bound.
//
// Design (gfx950, wave64):
//  * one wave owns a strip of 64 columns (64 - 2 KB outputs) and a block of
//    TI rows; lanes run along the contiguous t direction, so every row load
//    and store is one coalesced 512-byte access;
//  * the right products W_t = X R_t need the 2 KB neighbouring columns of a
//    lane: they come from the neighbours' registers through DPP wave shifts,
//    no LDS and no barriers;
//  * the lane's column of every right band (NT x (2KB+1) values) sits in
//    registers for the whole block; the products W_t of the last 2KB+1 rows
//    form a register ring; the left products combine the ring with the
//    row's left coefficients, which are uniform across the wave and come
//    through the scalar cache;
//  * the row loop is fully unrolled so every ring slot is a compile-time
//    register, and, for P_k element matrices (k >= 2), each row's position
//    inside its element is known at compile time: the left product then
//    touches only the k + 1 (interior node) or 2k + 1 (element vertex)
//    structural non-zeros;
//  * an optional fused Frobenius product <X, Y> per item (eq. (77)) is
//    reduced per wave and written to a partial-sum array (a second, fixed
//    order pass makes it deterministic).
#pragma once

#include "device_common.h"
#include "kernels.h"
#include "mofem_internal.h"

namespace mofem {

template <int KB>
struct BandTile {
  static constexpr int W = 2 * KB + 1;
  static constexpr int U = KB * W;  // rows after which ring slot and element phase repeat
  static constexpr int TI = (KB == 1) ? 48 : (KB == 2) ? 50 : (KB == 3) ? 42 : 36;
  static constexpr int SW = 64 - 2 * KB;  // output columns per wave
  static_assert(TI % U == 0, "row block must be a whole number of periods");
};

template <int KB, int NT, bool PAT>
__global__ __launch_bounds__(64) void band_apply_kernel(BandArgs a) {
  using T = BandTile<KB>;
  constexpr int W = T::W;
  constexpr int TI = T::TI;
  constexpr int NROWS = TI + 2 * KB;

  const int lane = threadIdx.x;
  const int n_strips = (a.qt + T::SW - 1) / T::SW;
  const int n_tiles = n_strips * a.n_rowblk;
  const int tile = xcd_tile(blockIdx.x, n_tiles);
  const int strip = tile / a.n_rowblk;
  const int rb = tile - strip * a.n_rowblk;
  const int b = blockIdx.y;
  if (a.active && !a.active[b]) return;

  const int j = strip * T::SW + lane - KB;  // output column of this lane
  const bool own = (lane >= KB) && (lane < 64 - KB) && (j < a.qt);
  const int bcol = j + a.off_t;             // input column this lane loads
  const bool in_col = (bcol >= 0) && (bcol < a.nt_in);

  const double scale = a.item_scale ? a.item_scale[b] : 1.0;

  // right coefficients of column j, with the per-item scale folded in
  double rc[NT][W];
  const bool jvalid = (j >= 0) && (j < a.qt);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double s = ((a.scaled_mask >> t) & 1) ? scale : 1.0;
#pragma unroll
    for (int d = 0; d < W; ++d)
      rc[t][d] = jvalid ? s * a.right[((size_t)t * W + d) * a.qt + j] : 0.0;
  }

  const double* __restrict__ Xb = a.X + (size_t)b * a.in_stride + (in_col ? bcol : 0);
  double* __restrict__ Yb = a.Y + (size_t)b * a.out_stride + (own ? j : 0);
  const double* __restrict__ Lc = a.left;

  const int g0 = rb * TI;           // first output node row of this block
  const int delta = a.off_s - a.ph_s;  // input row = node row + delta

  double ring[NT][W];   // W_t of the last W node rows, slot = node mod W
  double xs[W];         // the lane's own X value of the last W node rows
  double dot = 0.0;

#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int d = 0; d < W; ++d) ring[t][d] = 0.0;

  StaticFor<0, NROWS>::run([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    // node row h = g0 - KB + p ; its ring slot is (p - KB) mod W (g0 = 0 mod W)
    constexpr int slot = ((p - KB) % W + W) % W;
    const int h = g0 - KB + p;
    const int arow = h + delta;
    double xv = 0.0;
    if (in_col && arow >= 0 && arow < a.ns_in) xv = Xb[(size_t)arow * a.ld_x];
    // neighbours: nb[d] = value at lane + d - KB
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
    if constexpr (p >= 2 * KB) {
      // output node row g = h - KB = g0 + m
      constexpr int m = p - 2 * KB;
      constexpr int phase = m % KB;
      constexpr int dlo = (!PAT || phase == 0) ? 0 : KB - phase;
      constexpr int dhi = (!PAT || phase == 0) ? 2 * KB : 2 * KB - phase;
      const int g = g0 + m;
      const int i = g - a.ph_s;
      if (i >= 0 && i < a.qs) {
        const double* li = Lc + (size_t)i * (NT * W);
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int d = dlo; d <= dhi; ++d) {
            acc = fma(li[t * W + d], ring[t][((m + d - KB) % W + W) % W], acc);
          }
        }
        if (own) {
          Yb[(size_t)i * a.ld_y] = acc;
          dot = fma(acc, xs[(m % W + W) % W], dot);
        }
      }
    }
  });

  if (a.dot_partial) {
    dot = wave_sum(dot);
    if (lane == 0) a.dot_partial[(size_t)b * a.n_partial + tile] = dot;
  }
}

template <int KB, int NT>
void launch_kb_nt(const BandArgs& a, int batch, bool pat, hipStream_t s) {
  int n_strips = (a.qt + BandTile<KB>::SW - 1) / BandTile<KB>::SW;
  dim3 grid(n_strips * a.n_rowblk, batch);
  if (pat && KB >= 2)
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, (KB >= 2)>), grid, dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((band_apply_kernel<KB, NT, false>), grid, dim3(64), 0, s, a);
}

// One translation unit per band width compiles these (k_band_kb*.hip).
#define MOFEM_BAND_INSTANTIATE(KB)                                                   \
  template void launch_kb_nt<KB, 1>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 2>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 3>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 5>(const BandArgs&, int, bool, hipStream_t);        \
  template void launch_kb_nt<KB, 6>(const BandArgs&, int, bool, hipStream_t);

}  // namespace mofem

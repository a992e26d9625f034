// Device-side helpers shared by the libmofem kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mofem {

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(F&& f) {
    f(std::integral_constant<int, B>{});
    StaticFor<B + 1, E>::run(f);
  }
};
template <int E>
struct StaticFor<E, E> {
  template <class F>
  __device__ __forceinline__ static void run(F&&) {}
};

// Whole-wave lane shifts through DPP (wave_shl:1 / wave_shr:1).  Lane l
// receives the value of lane l+1 (shl) or l-1 (shr); the lane shifted in
// from outside the wave receives 0.
__device__ __forceinline__ double wave_shl1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Immediate of s_waitcnt on gfx9-family GPUs such as gfx950: vmcnt in bits
// 3:0 and 15:14, expcnt in bits 6:4, lgkmcnt in bits 11:8; a field at its
// maximum (63, 7, 15) does not wait.  Other GPU families encode these fields
// differently, so device code using it builds for gfx950 only.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(__gfx950__)
#error "s_waitcnt immediates below are encoded for gfx950"
#endif
constexpr unsigned waitcnt_imm(unsigned vmcnt, unsigned expcnt, unsigned lgkmcnt) {
  return (vmcnt & 0xFu) | (((vmcnt >> 4) & 0x3u) << 14) | ((expcnt & 0x7u) << 4) | ((lgkmcnt & 0xFu) << 8);
}
// wait until this wave's vector memory operations (loads, stores and direct
// global -> LDS loads) have completed; LDS and export counters unconstrained
constexpr unsigned kWaitVmcnt0 = waitcnt_imm(0, 7, 15);
static_assert(kWaitVmcnt0 == 0x0F70u, "vmcnt(0), expcnt(7), lgkmcnt(15)");

// Sum over the 64 lanes of a wave (every lane receives the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// XCD-aware tile order.  Work-groups are dealt round-robin to the 8 XCDs of
// an MI355X (dispatch id % 8).  Map dispatch id -> tile so that each XCD
// receives one contiguous range of tiles (neighbouring tiles share halo data
// through that XCD's L2).  Bijective for any tile count n.
__device__ __forceinline__ int xcd_tile(int id, int n) {
  const int nx = 8;
  int q = n / nx, r = n % nx;
  int x = id % nx, slot = id / nx;
  return (x < r) ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// Tile (row, column) of a tm x tn tile grid for dispatch id `id`.  Tile numbers
// run down bands of G tile rows, column by column, and each XCD takes one
// contiguous range of numbers (xcd_tile), so an XCD's share is a compact block
// of about G rows: it reads fewer operand strips into its L2 than whole tile
// rows would need.  Bijective for any tm, tn >= 1.
__device__ __forceinline__ void grouped_tile(int id, int tm, int tn, int G, int* tr, int* tc) {
  const int t = xcd_tile(id, tm * tn);
  const int band = t / (G * tn);
  const int first = band * G;
  const int rows = min(G, tm - first);
  const int w = t - band * G * tn;
  *tr = first + w % rows;
  *tc = w / rows;
}

// Item b and tile (row, column) of dispatch (bx, by) of a grid of tm x tn
// tiles per item and gridDim.y items.  When the grid splits evenly (tm a
// multiple of 8, tm tn of 64, all tiles of 512), the dispatches an XCD receives
// in turn (every eighth) take consecutive 8 x 8 blocks of one item's tiles,
// and the eight XCDs hold eight such blocks of two items at a time; otherwise
// b = by and the tile comes from grouped_tile with bands of G rows.  Bijective.
__device__ __forceinline__ void item_tile(int bx, int by, int tm, int tn, int G, bool blocks8, int* b, int* tr,
                                          int* tc) {
  const int nti = tm * tn;
  if (blocks8 && tm % 8 == 0 && nti % 64 == 0 && (nti * (int)gridDim.y) % 512 == 0) {
    const int L = bx + nti * by;
    const int x = L % 8, slot = L / 8;
    const int T = ((slot / 64) * 8 + x) * 64 + slot % 64;  // chunk (slot / 64, x), then its tile
    *b = T / nti;
    const int t = T - *b * nti;
    const int band = t / (8 * tn);
    const int w = t - band * 8 * tn;
    *tr = band * 8 + w % 8;
    *tc = w / 8;
  } else {
    *b = by;
    grouped_tile(bx, tm, tn, G, tr, tc);
  }
}

}  // namespace mofem

// Dispatch of the multiterm banded operator apply (kernel in band_kernel.inl;
// its instantiations live in k_band_kb1..4.hip so they compile in parallel).
#include "band_kernel.inl"

namespace mofem {

#define MOFEM_BAND_EXTERN_NT(KB, NT)                                                             \
  extern template void launch_kb_nt<KB, NT, false, 1>(const BandArgs&, int, bool, hipStream_t);  \
  extern template void launch_kb_nt<KB, NT, false, 2>(const BandArgs&, int, bool, hipStream_t);
#define MOFEM_BAND_EXTERN_COMMON(KB)                                                            \
  MOFEM_BAND_EXTERN_NT(KB, 1)                                                                   \
  MOFEM_BAND_EXTERN_NT(KB, 2)                                                                   \
  MOFEM_BAND_EXTERN_NT(KB, 3)                                                                   \
  MOFEM_BAND_EXTERN_NT(KB, 4)                                                                   \
  extern template void launch_kb_nt<KB, 2, true, 1>(const BandArgs&, int, bool, hipStream_t);   \
  extern template void launch_kb_nt<KB, 3, true, 1>(const BandArgs&, int, bool, hipStream_t);   \
  extern template void launch_kb_nt<KB, 4, true, 1>(const BandArgs&, int, bool, hipStream_t);
#define MOFEM_BAND_EXTERN_WIDE(KB) \
  MOFEM_BAND_EXTERN_NT(KB, 5)      \
  MOFEM_BAND_EXTERN_NT(KB, 6)
MOFEM_BAND_EXTERN_COMMON(1)
MOFEM_BAND_EXTERN_COMMON(2)
MOFEM_BAND_EXTERN_COMMON(3)
MOFEM_BAND_EXTERN_COMMON(4)
MOFEM_BAND_EXTERN_WIDE(1)
MOFEM_BAND_EXTERN_WIDE(2)
MOFEM_BAND_SMALL_LIST(extern template void, 1)
MOFEM_BAND_SMALL_LIST(extern template void, 2)

template <int KB>
static int rows_kb(int nt) {
  switch (nt) {
    case 1: return BandCfg<KB, 1>::TI;
    case 2: return BandCfg<KB, 2>::TI;
    case 3: return BandCfg<KB, 3>::TI;
    case 4: return BandCfg<KB, 4>::TI;
    case 5: return BandCfg<KB, 5>::TI;
    default: return BandCfg<KB, 6>::TI;  // (layout only; KB >= 3 runs at most 4 terms per launch)
  }
}
int band_rows_per_block(int kb, int nt, int small) {
  if (small && band_has_small(kb))
    return kb == 1 ? band_small_groups<1>() * BandRing<1>::UG : band_small_groups<2>() * BandRing<2>::UG;
  switch (kb) {
    case 1: return rows_kb<1>(nt);
    case 2: return rows_kb<2>(nt);
    case 3: return rows_kb<3>(nt);
    default: return rows_kb<4>(nt);
  }
}
int band_has_small(int kb) {
  switch (kb) {
    case 1: return band_small_groups<1>() > 0;
    case 2: return band_small_groups<2>() > 0;
    default: return 0;
  }
}
int band_cols_per_block(int kb) { return kBandWaves * (64 - 2 * kb); }
int band_pass_terms(int kb) { return band_max_pass_terms(kb); }

template <int KB, int IPL, int GG>
static int launch_kb_ipl(const BandArgs& a, int nt, int batch, bool pat, hipStream_t s) {
  switch (nt) {
    case 1: launch_kb_nt<KB, 1, false, IPL, GG>(a, batch, pat, s); return 0;
    case 2: launch_kb_nt<KB, 2, false, IPL, GG>(a, batch, pat, s); return 0;
    case 3: launch_kb_nt<KB, 3, false, IPL, GG>(a, batch, pat, s); return 0;
    case 4: launch_kb_nt<KB, 4, false, IPL, GG>(a, batch, pat, s); return 0;
    default: break;
  }
  if constexpr (KB <= 2) {
    switch (nt) {
      case 5: launch_kb_nt<KB, 5, false, IPL, GG>(a, batch, pat, s); return 0;
      case 6: launch_kb_nt<KB, 6, false, IPL, GG>(a, batch, pat, s); return 0;
      default: break;
    }
  }
  return -1;
}

// Two items per lane when the batch has at least two items and every item
// sees the same operator (no per-item scale on a scaled term).
template <int KB, int GG>
static int launch_kb_gg(const BandArgs& a, int nt, int batch, bool pat, hipStream_t s) {
  if (a.accumulate) {
    switch (nt) {
      case 2: launch_kb_nt<KB, 2, true, 1, GG>(a, batch, pat, s); return 0;
      case 3: launch_kb_nt<KB, 3, true, 1, GG>(a, batch, pat, s); return 0;
      case 4: launch_kb_nt<KB, 4, true, 1, GG>(a, batch, pat, s); return 0;
      default: return -1;
    }
  }
  const bool shared = batch >= 2 && (a.scaled_mask == 0 || a.item_scale == nullptr);
  return shared ? launch_kb_ipl<KB, 2, GG>(a, nt, batch, pat, s) : launch_kb_ipl<KB, 1, GG>(a, nt, batch, pat, s);
}

template <int KB>
static int launch_kb(const BandArgs& a, int nt, int batch, bool pat, int small, hipStream_t s) {
  if (nt > band_max_pass_terms(KB)) return -1;
  if constexpr (band_small_groups<KB>() > 0) {
    if (small) return launch_kb_gg<KB, band_small_groups<KB>()>(a, nt, batch, pat, s);
  }
  return launch_kb_gg<KB, 0>(a, nt, batch, pat, s);
}

int launch_band_apply(const BandArgs& a, int kb, int nt, int batch, bool pattern, int small, hipStream_t s) {
  switch (kb) {
    case 1: return launch_kb<1>(a, nt, batch, false, small, s);
    case 2: return launch_kb<2>(a, nt, batch, pattern, small, s);
    case 3: return launch_kb<3>(a, nt, batch, pattern, small, s);
    case 4: return launch_kb<4>(a, nt, batch, pattern, small, s);
    default: return -1;
  }
}

}  // namespace mofem

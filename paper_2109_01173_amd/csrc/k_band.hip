// Dispatch of the multiterm banded operator apply (kernel in band_kernel.inl;
// its instantiations live in k_band_kb1..4.hip so they compile in parallel).
#include "band_kernel.inl"

namespace mofem {

#define MOFEM_BAND_EXTERN(KB)                                                         \
  extern template void launch_kb_nt<KB, 1>(const BandArgs&, int, bool, hipStream_t); \
  extern template void launch_kb_nt<KB, 2>(const BandArgs&, int, bool, hipStream_t); \
  extern template void launch_kb_nt<KB, 3>(const BandArgs&, int, bool, hipStream_t); \
  extern template void launch_kb_nt<KB, 5>(const BandArgs&, int, bool, hipStream_t); \
  extern template void launch_kb_nt<KB, 6>(const BandArgs&, int, bool, hipStream_t);
MOFEM_BAND_EXTERN(1)
MOFEM_BAND_EXTERN(2)
MOFEM_BAND_EXTERN(3)
MOFEM_BAND_EXTERN(4)

template <int KB>
static int rows_kb(int nt) {
  switch (nt) {
    case 1: return BandCfg<KB, 1>::TI;
    case 2: return BandCfg<KB, 2>::TI;
    case 3: return BandCfg<KB, 3>::TI;
    case 5: return BandCfg<KB, 5>::TI;
    default: return BandCfg<KB, 6>::TI;
  }
}
int band_rows_per_block(int kb, int nt) {
  switch (kb) {
    case 1: return rows_kb<1>(nt);
    case 2: return rows_kb<2>(nt);
    case 3: return rows_kb<3>(nt);
    default: return rows_kb<4>(nt);
  }
}
int band_cols_per_block(int kb) { return kBandWaves * (64 - 2 * kb); }
int band_supported_terms(int nt) { return nt == 1 || nt == 2 || nt == 3 || nt == 5 || nt == 6; }

template <int KB>
static int launch_kb(const BandArgs& a, int nt, int batch, bool pat, hipStream_t s) {
  switch (nt) {
    case 1: launch_kb_nt<KB, 1>(a, batch, pat, s); return 0;
    case 2: launch_kb_nt<KB, 2>(a, batch, pat, s); return 0;
    case 3: launch_kb_nt<KB, 3>(a, batch, pat, s); return 0;
    case 5: launch_kb_nt<KB, 5>(a, batch, pat, s); return 0;
    case 6: launch_kb_nt<KB, 6>(a, batch, pat, s); return 0;
    default: return -1;
  }
}

int launch_band_apply(const BandArgs& a, int kb, int nt, int batch, bool pattern, hipStream_t s) {
  switch (kb) {
    case 1: return launch_kb<1>(a, nt, batch, false, s);
    case 2: return launch_kb<2>(a, nt, batch, pattern, s);
    case 3: return launch_kb<3>(a, nt, batch, pattern, s);
    case 4: return launch_kb<4>(a, nt, batch, pattern, s);
    default: return -1;
  }
}

}  // namespace mofem

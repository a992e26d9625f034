// Band-width 1 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE_COMMON(1)
MOFEM_BAND_INSTANTIATE_WIDE(1)
MOFEM_BAND_INSTANTIATE_SMALL(1)
}  // namespace mofem

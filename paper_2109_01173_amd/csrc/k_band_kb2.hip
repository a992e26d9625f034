// Band-width 2 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE_COMMON(2)
MOFEM_BAND_INSTANTIATE_WIDE(2)
MOFEM_BAND_INSTANTIATE_SMALL(2)
}  // namespace mofem

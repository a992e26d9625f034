// Band-width 4 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE_COMMON(4)

}  // namespace mofem

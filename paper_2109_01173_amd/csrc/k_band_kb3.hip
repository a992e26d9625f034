// Band-width 3 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE_COMMON(3)

}  // namespace mofem

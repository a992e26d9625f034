// Band-width 2 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE(2)
}  // namespace mofem

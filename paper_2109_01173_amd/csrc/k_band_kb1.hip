// Band-width 1 instantiations of the multiterm operator kernel.
#include "band_kernel.inl"

namespace mofem {
MOFEM_BAND_INSTANTIATE(1)
}  // namespace mofem

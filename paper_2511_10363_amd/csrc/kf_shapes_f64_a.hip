// Launch code of the small shapes for precision policy PrecF64.
#include "kf_inst.hpp"

namespace kfs {
KFS_INSTANTIATE(1, 1, PrecF64)
KFS_INSTANTIATE(2, 1, PrecF64)
KFS_INSTANTIATE(2, 2, PrecF64)
KFS_INSTANTIATE(3, 1, PrecF64)
KFS_INSTANTIATE(3, 2, PrecF64)
KFS_INSTANTIATE(4, 1, PrecF64)
}  // namespace kfs

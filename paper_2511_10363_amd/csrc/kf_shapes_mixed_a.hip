// Launch code of the small shapes for precision policy PrecMixed.
#include "kf_inst.hpp"

namespace kfs {
KFS_INSTANTIATE(1, 1, PrecMixed)
KFS_INSTANTIATE(2, 1, PrecMixed)
KFS_INSTANTIATE(2, 2, PrecMixed)
KFS_INSTANTIATE(3, 1, PrecMixed)
KFS_INSTANTIATE(3, 2, PrecMixed)
KFS_INSTANTIATE(4, 1, PrecMixed)
}  // namespace kfs

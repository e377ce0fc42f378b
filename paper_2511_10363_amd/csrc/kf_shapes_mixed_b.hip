// Launch code of the nx = 4 shapes with ny = 2, 4 for precision policy PrecMixed.
#include "kf_inst.hpp"

namespace kfs {
KFS_INSTANTIATE(4, 2, PrecMixed)
KFS_INSTANTIATE(4, 4, PrecMixed)
}  // namespace kfs

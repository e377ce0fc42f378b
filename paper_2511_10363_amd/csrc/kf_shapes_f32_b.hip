// Launch code of the nx = 4 shapes with ny = 2, 4 for precision policy PrecF32.
#include "kf_inst.hpp"

namespace kfs {
KFS_INSTANTIATE(4, 2, PrecF32)
KFS_INSTANTIATE(4, 4, PrecF32)
}  // namespace kfs

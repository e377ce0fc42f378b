// Launch code of the nx = 4 shapes with ny = 2, 4 for precision policy PrecF64.
#include "kf_inst.hpp"

namespace kfs {
KFS_INSTANTIATE(4, 2, PrecF64)
KFS_INSTANTIATE(4, 4, PrecF64)
}  // namespace kfs

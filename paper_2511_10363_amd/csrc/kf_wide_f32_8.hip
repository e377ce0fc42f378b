// Launch code of the nx = 8 group scans for precision policy PrecF32.
#include "kf_inst.hpp"

namespace kfs {
KFS_WIDE_INSTANTIATE(8, 4, PrecF32)
}  // namespace kfs

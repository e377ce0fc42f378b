// Launch code of the nx = 16 group scans for precision policy PrecF64.
#include "kf_inst.hpp"

namespace kfs {
KFS_WIDE_INSTANTIATE(16, 8, PrecF64)
}  // namespace kfs

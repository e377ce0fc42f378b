// Launch code of the nx = 8 group scans for precision policy PrecF64.
#include "kf_inst.hpp"

namespace kfs {
KFS_WIDE_INSTANTIATE(8, 4, PrecF64)
}  // namespace kfs

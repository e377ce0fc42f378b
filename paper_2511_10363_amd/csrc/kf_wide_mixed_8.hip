// Launch code of the nx = 8 group scans for precision policy PrecMixed.
#include "kf_inst.hpp"

namespace kfs {
KFS_WIDE_INSTANTIATE(8, 4, PrecMixed)
}  // namespace kfs

// Kernel instantiations for precision policy PrecF32.
#include "kf_inst.hpp"

namespace kfs {
kf_status run_f32(Op op, const kf_problem& p, char* ws, const Layout& L, hipStream_t st) {
  return run_prec<PrecF32>(op, p, ws, L, st);
}
}  // namespace kfs

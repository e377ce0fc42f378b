// Shape dispatch for precision policy PrecF32.
#include "kf_inst.hpp"

namespace kfs {
kf_status run_f32(Op op, int stages, const Job& p, char* ws, const Layout& L,
                  hipStream_t st) {
  return run_prec<PrecF32>(op, stages, p, ws, L, st);
}
}  // namespace kfs

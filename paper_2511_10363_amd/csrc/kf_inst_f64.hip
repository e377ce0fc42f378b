// Shape dispatch for precision policy PrecF64.
#include "kf_inst.hpp"

namespace kfs {
kf_status run_f64(Op op, int stages, const Job& p, char* ws, const Layout& L,
                  hipStream_t st) {
  return run_prec<PrecF64>(op, stages, p, ws, L, st);
}
}  // namespace kfs

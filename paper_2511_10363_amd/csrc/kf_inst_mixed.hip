// Shape dispatch for precision policy PrecMixed.
#include "kf_inst.hpp"

namespace kfs {
kf_status run_mixed(Op op, int stages, const Job& p, char* ws, const Layout& L,
                  hipStream_t st) {
  return run_prec<PrecMixed>(op, stages, p, ws, L, st);
}
}  // namespace kfs

// kf_plan.hpp -- host-side launch plan and workspace layout, shared by the
// C-ABI entry points and the per-precision kernel instantiations.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/kfscan.h"

namespace kfs {

constexpr int kBlock = 256;

// Time steps each thread owns: in the scans over full elements, and in the
// time-invariant scans whose per-thread fold is a linear map of the
// measurements (so a thread can own more steps).
constexpr int items_per_thread(int nx) { return nx <= 2 ? 16 : (nx <= 4 ? 8 : 4); }
constexpr int items_ti(int nx) { return nx <= 4 ? 16 : 8; }
constexpr int items_min(int nx) {
  return items_per_thread(nx) < items_ti(nx) ? items_per_thread(nx) : items_ti(nx);
}

inline size_t word_bytes(int precision) { return precision == KF_PREC_F64 ? 8 : 4; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace regions (byte offsets from the workspace base).  The control
// words (tile tickets, timeout flags and look-back status words of both scan
// slots) come first and are zeroed by the preparation kernel at the start of
// every call, so a workspace needs no initialisation and carries no state
// from one call to the next.
struct Layout {
  size_t ctr[2];              // [0] tile ticket, [1] finished blocks, [2] timeout flag
  size_t flags[2];            // look-back status words, slot 0 forward, slot 1 backward
  size_t ctrl_words;          // 32-bit words of the control region at offset 0
  size_t cst;                 // derived model quantities
  size_t agg[2];              // published tile aggregates
  size_t pre[2];              // published anchored prefixes
  long max_tiles;             // tiles per sequence at the smallest tile size
  size_t total;
};

inline long ntiles_for(long T, int items) {
  const long tile = (long)kBlock * items;
  return (T + tile - 1) / tile;
}

inline Layout make_layout(int nx, int ny, int precision, long T, long nseq) {
  const size_t w = word_bytes(precision);
  const long n = nx, m = ny;
  Layout L{};
  L.max_tiles = ntiles_for(T, items_min(nx));
  const size_t nt = (size_t)L.max_tiles * (size_t)nseq;
  const size_t cst_words =                               // CL<N, M, L>::SIZE
      10 * n * n + 4 * n * m + m * m + 2 * n + 2 * (size_t)items_ti(nx) * n * m;
  const size_t elem_words = 3 * n * n + 2 * n;           // largest element (filtering)
  const size_t pre_words = n + n * n;
  L.ctr[0] = 0;
  L.ctr[1] = 4 * sizeof(unsigned);
  L.flags[0] = 8 * sizeof(unsigned);
  L.flags[1] = L.flags[0] + nt * sizeof(int);
  L.ctrl_words = (L.flags[1] + nt * sizeof(int)) / 4;
  size_t off = align256(L.ctrl_words * 4);
  L.cst = off;
  off = align256(off + cst_words * w);
  for (int s = 0; s < 2; ++s) {
    L.agg[s] = off;
    off = align256(off + nt * elem_words * w);
    L.pre[s] = off;
    off = align256(off + nt * pre_words * w);
  }
  L.total = off;
  return L;
}

enum Op { OP_FILTER = 0, OP_RTS = 1, OP_TWOFILTER = 2 };

// Which kernels of an operation to enqueue.
enum Stage { ST_PREPARE = 1, ST_FORWARD = 2, ST_BACKWARD = 4, ST_ALL = 7 };

// Implemented once per precision (kf_inst_*.hip).
kf_status run_f64(Op op, int stages, const kf_problem& p, char* ws, const Layout& L,
                  hipStream_t st);
kf_status run_f32(Op op, int stages, const kf_problem& p, char* ws, const Layout& L,
                  hipStream_t st);
kf_status run_mixed(Op op, int stages, const kf_problem& p, char* ws, const Layout& L,
                    hipStream_t st);
bool shape_built(int nx, int ny);

}  // namespace kfs

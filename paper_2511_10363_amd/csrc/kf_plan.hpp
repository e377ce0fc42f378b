// kf_plan.hpp -- host-side launch plan and workspace layout, shared by the
// C-ABI entry points and the per-precision kernel instantiations.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/kfscan.h"

namespace kfs {

constexpr int kBlock = 256;

// Time steps each thread owns (L), at most: in the scans over full elements,
// and in the time-invariant filter, whose per-thread fold is a linear map of
// the measurements (so a thread can own more steps).  The launch takes the
// largest power of two L <= the maximum (and >= 2) that still gives a target
// number of tiles.  The time-invariant filter aims at 256 tiles, one per CU,
// since its fold is cheap and its wavefront totals become anchors early.  The
// full-element scans keep the longest tiles unless a sequence would have fewer
// than 4: their tile aggregates must be long to underflow into anchors (see
// decay_is_zero), and a short-tile look-back over non-anchored aggregates
// costs more than the parallelism gained.
constexpr int items_per_thread(int nx) { return nx <= 2 ? 16 : (nx <= 4 ? 8 : 4); }
constexpr int items_ti(int nx) { return nx <= 4 ? 16 : 8; }
constexpr long kTilesTi = 256, kTilesScan = 4;

inline long ntiles_for(long T, int items) {
  const long tile = (long)kBlock * items;
  return (T + tile - 1) / tile;
}

inline int choose_items(long T, long nseq, int lmax, long target) {
  int L = lmax;
  while (L > 2 && nseq * ntiles_for(T, L) < target) L /= 2;
  return L;
}

inline size_t word_bytes(int precision) { return precision == KF_PREC_F64 ? 8 : 4; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace regions (byte offsets from the workspace base).  The control
// region -- tile tickets, epochs, timeout flags, look-back status words and
// the tagged look-back payloads of both scan slots -- comes first and is
// zeroed by the preparation kernel at the start of every call, so a workspace
// needs no initialisation and carries no state from one call to the next.
struct Layout {
  size_t ctr[2];              // [0] tile ticket, [1] finished blocks, [2] timeout flag, [3] epoch
  size_t flags[2];            // look-back status words, slot 0 forward, slot 1 backward
  size_t agg[2];              // published tile aggregates (tagged 64-bit words)
  size_t pre[2];              // published anchored prefixes (tagged 64-bit words)
  size_t ctrl_words;          // 32-bit words of the control region at offset 0
  size_t cst;                 // derived model quantities
  size_t tree[2];             // element buffers of the tree scans (Hillis-Steele: both)
  long tree_positions;        // scan positions per sequence of the tree scans
  int items[2];               // steps per thread of the forward and backward scans
  long ntiles[2];             // tiles per sequence of the forward and backward scans
  size_t total;
};

// Tiles per thread in a look-back window: one window of 256*G tiles reaches
// back over a whole sequence of up to 1024 tiles.
inline int lookback_group(long ntiles) {
  const long g = (ntiles + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 4 ? 4 : g));
}

inline bool is_tree_scan(int scan) {
  return scan == KF_SCAN_BLELLOCH || scan == KF_SCAN_HILLIS_STEELE;
}

inline long tree_positions_for(int scan, long T) {
  if (scan == KF_SCAN_HILLIS_STEELE) return T;
  long p = 1;
  while (p < T) p <<= 1;
  return p;
}

inline Layout make_layout(int nx, int ny, int precision, int scan, long T, long nseq) {
  const size_t w = word_bytes(precision);
  const size_t halves = w / 4;                           // tagged words per scalar
  const long n = nx, m = ny;
  Layout L{};
  L.items[0] = (scan == KF_SCAN_LOOKBACK_GENERIC)
                   ? choose_items(T, nseq, items_per_thread(nx), kTilesScan)
                   : choose_items(T, nseq, items_ti(nx), kTilesTi);
  L.items[1] = choose_items(T, nseq, items_per_thread(nx), kTilesScan);
  L.ntiles[0] = ntiles_for(T, L.items[0]);
  L.ntiles[1] = ntiles_for(T, L.items[1]);
  const size_t ntf[2] = {(size_t)L.ntiles[0] * (size_t)nseq, (size_t)L.ntiles[1] * (size_t)nseq};
  const size_t cst_words =                               // CL<N, M, L>::SIZE
      10 * n * n + 4 * n * m + m * m + 2 * n + 2 * (size_t)items_ti(nx) * n * m;
  const size_t elem_words = 3 * n * n + 2 * n;           // largest element (filtering)
  const size_t pre_words = n + n * n;
  size_t off = 0;
  for (int s = 0; s < 2; ++s) {
    L.ctr[s] = off;
    off += 4 * sizeof(unsigned);
  }
  for (int s = 0; s < 2; ++s) {
    L.flags[s] = off;
    off += ntf[s] * sizeof(int);
  }
  off = (off + 7) & ~size_t(7);
  for (int s = 0; s < 2; ++s) {
    L.agg[s] = off;
    off += ntf[s] * elem_words * halves * 8;
    L.pre[s] = off;
    off += ntf[s] * pre_words * halves * 8;
  }
  L.ctrl_words = off / 4;
  off = align256(off);
  L.cst = off;
  off = align256(off + cst_words * w);
  L.tree[0] = L.tree[1] = off;
  if (is_tree_scan(scan)) {
    L.tree_positions = tree_positions_for(scan, T);
    const size_t buf = (size_t)nseq * elem_words * (size_t)L.tree_positions * w;
    L.tree[0] = off;
    off = align256(off + buf);
    L.tree[1] = off;
    if (scan == KF_SCAN_HILLIS_STEELE) off = align256(off + buf);
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

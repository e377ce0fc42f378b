// kf_plan.hpp -- host-side launch plan and workspace layout, shared by the
// C-ABI entry points and the per-precision kernel instantiations.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/kfscan.h"

namespace kfs {

constexpr int kBlock = 256;
constexpr size_t kEpochOffset = 128;  // bytes: the epoch words of the two scan slots

// Time steps each thread owns (L), at most: in the scans over full elements,
// and in the time-invariant filter, whose per-thread fold is a linear map of
// the measurements (so a thread can own more steps).  The launch takes the
// largest power of two L <= the maximum (and >= 2) that still gives a target
// number of tiles.  The time-invariant filter aims at 256 tiles, one per CU,
// since its fold is cheap and its wavefront totals become anchors early.  The
// backward scans (RTS, two-filter) aim at 256 tiles too: at T = 2^18 their
// 8-step tiles would leave half the CUs idle (measured on MI355X, 4-step
// tiles: RTS 47.6 -> 37.5 us in FP32, two-filter 87.6 -> 63.4 us in the mixed
// mode), while at T = 2^20 the 8-step tiles already give two per CU.  The
// generic forward scan keeps the longest tiles unless a sequence would have
// fewer than 4: its tile aggregates must be long to underflow into anchors
// (see decay_is_zero), and a short-tile look-back over non-anchored
// aggregates costs more than the parallelism gained.
constexpr int items_per_thread(int nx) { return nx <= 2 ? 16 : (nx <= 4 ? 8 : 4); }
constexpr int items_ti(int nx) { return nx <= 4 ? 16 : 8; }
constexpr long kTilesTi = 256, kTilesScan = 4, kTilesBack = 256;

inline long ntiles_for(long T, int items) {
  const long tile = (long)kBlock * items;
  return (T + tile - 1) / tile;
}

// States wider than nx = 4 are scanned by groups of nx lanes (kf_wide.hpp):
// workgroups of wide_block(nx) threads, each group owning wide_items(nx)
// steps, so a tile holds wide_block(nx) / nx * wide_items(nx) steps: 256
// threads at nx = 8 (32 groups, 512-step tiles) and a single wavefront at
// nx = 16 (4 groups, 64-step tiles).  The nx = 16 kernels spill registers to
// per-lane scratch memory, and a workgroup of several wavefronts can then be
// started wavefront by wavefront as scratch frees up: a tile whose
// workgroup is only partly running would hold up every later tile waiting
// for it, while those waiting workgroups hold the scratch it needs.  A
// one-wavefront workgroup is running in full as soon as it takes its tile.
inline bool is_wide(int nx) { return nx > 4; }
constexpr int wide_block(int nx) { return nx <= 8 ? 256 : 64; }
constexpr int wide_items(int) { return 16; }
inline long wide_tile(int nx) { return (long)(wide_block(nx) / nx) * wide_items(nx); }

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
  size_t ctr[2];              // [0] tile ticket, [1] finished blocks, [2] timeout flag
  size_t epoch[2];            // the pass epoch of each slot, a cache line away from the tickets
  size_t flags[2];            // look-back status words, slot 0 forward, slot 1 backward
  size_t agg[2];              // published tile aggregates (tagged 64-bit words)
  size_t pre[2];              // published anchored prefixes (tagged 64-bit words)
  size_t ctrl_words;          // 32-bit words of the control region at offset 0
  size_t cst;                 // derived model quantities
  size_t tree[2];             // element buffers of the tree scans (HS, Sengupta: both)
  long tree_positions;        // scan positions per sequence of the tree scans
  int items[2];               // steps per thread of the forward and backward scans
  long ntiles[2];             // tiles per sequence (equal-length sequences)
  long grid[2];               // blocks of the forward and backward scans
  long tile[2];               // steps per tile of the forward and backward scans
  long cst_stride;            // scalars per model in the cst region
  size_t tile_start[2];       // ragged batch: first tile ticket of each sequence, int64 [nseq+1]
  size_t tile_map[2];         // ragged batch: sequence of each ticket, int32 [grid]
  size_t total;
};

// One call, equal-length sequences (kf_problem) or a ragged batch (kf_batch).
struct Job {
  int nx, ny, precision, scan;
  long T;                     // steps per sequence (ragged batch: the mean, for tiling)
  long nseq;
  bool batch;
  long nmodels;               // 1, or nseq in a batch with a model per sequence
  long total_steps;           // rows of y and of the outputs
  const int64_t* len;         // ragged batch, device [nseq]
  const int64_t* row;         // ragged batch, device [nseq]
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  void *m_filt, *P_filt, *m_smooth, *P_smooth;
  bool tv;                    // F, Q, H, R, u, d are per-step arrays
  const void *u, *d;          // time-varying model: may be null
  uint32_t* status;           // per-sequence status words, device [nseq], or null
  int items;                  // requested steps per thread (0 = the library's choice)
};

// The scans with one kernel launch per tree level (kf_tree.hpp).
inline bool is_tree_scan(int scan) {
  return scan == KF_SCAN_BLELLOCH || scan == KF_SCAN_HILLIS_STEELE ||
         scan == KF_SCAN_LADNER_FISCHER || scan == KF_SCAN_SENGUPTA_A ||
         scan == KF_SCAN_SENGUPTA_B;
}

inline Job job_of(const kf_problem& p) {
  Job j{};
  j.nx = p.nx;
  j.ny = p.ny;
  j.precision = p.precision;
  j.scan = p.scan;
  j.T = p.T;
  j.nseq = p.nseq;
  j.batch = false;
  j.nmodels = 1;
  j.total_steps = p.T * p.nseq;
  j.F = p.F; j.Q = p.Q; j.H = p.H; j.R = p.R; j.m0 = p.m0; j.P0 = p.P0;
  j.y = p.y;
  j.m_filt = p.m_filt; j.P_filt = p.P_filt; j.m_smooth = p.m_smooth; j.P_smooth = p.P_smooth;
  j.status = p.status;
  j.items = p.items;
  return j;
}

inline Job job_of(const kf_tv_problem& p) {
  Job j{};
  j.nx = p.nx;
  j.ny = p.ny;
  j.precision = p.precision;
  // the per-step elements are folded by the look-back scans over full elements
  j.scan = (p.scan == KF_SCAN_SEQUENTIAL || is_tree_scan(p.scan)) ? p.scan
                                                                  : KF_SCAN_LOOKBACK_GENERIC;
  j.T = p.T;
  j.nseq = p.nseq;
  j.batch = false;
  j.nmodels = 1;
  j.total_steps = p.T * p.nseq;
  j.F = p.F; j.Q = p.Q; j.H = p.H; j.R = p.R; j.m0 = p.m0; j.P0 = p.P0;
  j.u = p.u; j.d = p.d;
  j.tv = true;
  j.y = p.y;
  j.m_filt = p.m_filt; j.P_filt = p.P_filt; j.m_smooth = p.m_smooth; j.P_smooth = p.P_smooth;
  j.status = p.status;
  j.items = p.items;
  return j;
}

inline Job job_of(const kf_batch& b) {
  Job j{};
  j.nx = b.nx;
  j.ny = b.ny;
  j.precision = b.precision;
  j.scan = b.scan;
  j.nseq = b.nseq;
  j.T = b.nseq > 0 ? (b.total_steps + b.nseq - 1) / b.nseq : 1;
  if (j.T < 1) j.T = 1;
  j.batch = true;
  j.nmodels = b.nmodels;
  j.total_steps = b.total_steps;
  j.len = b.T;
  j.row = b.offset;
  j.F = b.F; j.Q = b.Q; j.H = b.H; j.R = b.R; j.m0 = b.m0; j.P0 = b.P0;
  j.y = b.y;
  j.m_filt = b.m_filt; j.P_filt = b.P_filt; j.m_smooth = b.m_smooth; j.P_smooth = b.P_smooth;
  j.status = b.status;
  j.items = b.items;
  return j;
}

inline long tree_positions_for(int scan, long T) {
  if (scan == KF_SCAN_HILLIS_STEELE) return T;
  long p = 1;
  while (p < T) p <<= 1;
  return p;
}

inline Layout make_layout(const Job& j) {
  const size_t w = word_bytes(j.precision);
  const size_t halves = w / 4;                           // tagged words per scalar
  const long n = j.nx, m = j.ny, T = j.T, nseq = j.nseq;
  const int scan = j.scan;
  Layout L{};
  if (scan == KF_SCAN_SEQUENTIAL) {
    // the sequential recursions need only the error words of the two slots
    L.ctr[0] = 0;
    L.ctr[1] = 4 * sizeof(unsigned);
    L.ctrl_words = 8;
    L.cst = L.tree[0] = L.tree[1] = 256;
    L.tile_start[0] = L.tile_start[1] = L.tile_map[0] = L.tile_map[1] = 256;
    L.total = 256;
    return L;
  }
  if (is_wide(j.nx)) {
    // one tile size for both scans, batch or not
    for (int s = 0; s < 2; ++s) {
      L.items[s] = wide_items(j.nx);
      L.tile[s] = wide_tile(j.nx);
    }
  } else {
    // A ragged batch always takes the longest tiles, so that each sequence is
    // tiled, scanned and rounded the same whatever else is in the batch.
    const int lf = (scan == KF_SCAN_LOOKBACK_GENERIC) ? items_per_thread(j.nx) : items_ti(j.nx);
    const int lb = items_per_thread(j.nx);
    if (j.items > 0) {
      // the caller's tile size, capped at the longest each kernel is built for
      L.items[0] = j.items < lf ? j.items : lf;
      L.items[1] = j.items < lb ? j.items : lb;
    } else {
      L.items[0] = j.batch ? lf
                           : choose_items(T, nseq, lf,
                                          scan == KF_SCAN_LOOKBACK_GENERIC ? kTilesScan : kTilesTi);
      L.items[1] = j.batch ? lb : choose_items(T, nseq, lb, kTilesBack);
    }
    for (int s = 0; s < 2; ++s) L.tile[s] = (long)kBlock * L.items[s];
  }
  for (int s = 0; s < 2; ++s) {
    L.ntiles[s] = (T + L.tile[s] - 1) / L.tile[s];
    // a ragged batch: sum over sequences of ceil(T_i / tile) <= nseq + total / tile
    L.grid[s] = j.batch ? nseq + (j.total_steps + L.tile[s] - 1) / L.tile[s] : L.ntiles[s] * nseq;
  }
  // CLB<N, M, L>::SIZE: the model quantities and two sets of aggregate tables
  const size_t cst_words = 10 * n * n + 4 * n * m + m * m + 2 * n + 2 * 16 * (size_t)(n * m) +
                           3 * n * n + 2 * 16 * (size_t)(n * m);
  L.cst_stride = (long)((cst_words + 63) & ~size_t(63));
  const size_t elem_words = 3 * n * n + 2 * n;           // largest element (filtering)
  const size_t pre_words = n + n * n;
  size_t off = 0;
  for (int s = 0; s < 2; ++s) {
    L.ctr[s] = off;
    off += 4 * sizeof(unsigned);
  }
  // Every workgroup reads its slot's epoch as it takes its ticket; on the
  // tickets' cache line those reads would queue behind the ticket atomics.
  for (int s = 0; s < 2; ++s) L.epoch[s] = kEpochOffset + 64 * (size_t)s;
  off = kEpochOffset + 128;
  for (int s = 0; s < 2; ++s) {
    L.flags[s] = off;
    off += (size_t)L.grid[s] * sizeof(int);
  }
  off = (off + 7) & ~size_t(7);
  for (int s = 0; s < 2; ++s) {
    L.agg[s] = off;
    off += (size_t)L.grid[s] * elem_words * halves * 8;
    L.pre[s] = off;
    off += (size_t)L.grid[s] * pre_words * halves * 8;
  }
  L.ctrl_words = off / 4;
  off = align256(off);
  L.cst = off;
  off = align256(off + (size_t)(j.batch ? j.nmodels : 1) * (size_t)L.cst_stride * w);
  L.tile_start[0] = L.tile_start[1] = L.tile_map[0] = L.tile_map[1] = off;
  if (j.batch) {
    for (int s = 0; s < 2; ++s) {
      L.tile_start[s] = off;
      off = align256(off + (size_t)(nseq + 1) * sizeof(int64_t));
      L.tile_map[s] = off;
      off = align256(off + (size_t)L.grid[s] * sizeof(int));
    }
  }
  L.tree[0] = L.tree[1] = off;
  if (is_tree_scan(scan)) {
    L.tree_positions = tree_positions_for(scan, T);
    const size_t buf = (size_t)nseq * elem_words * (size_t)L.tree_positions * w;
    L.tree[0] = off;
    off = align256(off + buf);
    L.tree[1] = off;
    if (scan == KF_SCAN_HILLIS_STEELE || scan == KF_SCAN_SENGUPTA_A ||
        scan == KF_SCAN_SENGUPTA_B)
      off = align256(off + buf);
  }
  L.total = off;
  return L;
}

enum Op { OP_FILTER = 0, OP_RTS = 1, OP_TWOFILTER = 2 };

// Which kernels of an operation to enqueue.
enum Stage { ST_PREPARE = 1, ST_FORWARD = 2, ST_BACKWARD = 4, ST_ALL = 7 };

// Implemented once per precision (kf_inst_*.hip).
kf_status run_f64(Op op, int stages, const Job& p, char* ws, const Layout& L, hipStream_t st);
kf_status run_f32(Op op, int stages, const Job& p, char* ws, const Layout& L, hipStream_t st);
kf_status run_mixed(Op op, int stages, const Job& p, char* ws, const Layout& L, hipStream_t st);
bool shape_built(int nx, int ny);
bool wide_shape_built(int nx, int ny);
// A whole call on kf_problem (kf_api.hip): argument checks, then every stage
// of `op` on `ws`; *ws_needed (if given) receives the workspace size the
// problem needs, and KF_ERR_WORKSPACE is returned when ws_bytes is smaller.
kf_status run_problem(Op op, const kf_problem* p, void* ws, size_t ws_bytes, void* stream,
                      size_t* ws_needed);

}  // namespace kfs

// kf_scan.hpp -- wavefront/block scan building blocks and the device-wide
// single-pass look-back, generic over the element type and operator.
//
// All operators are associative but not commutative.  Every routine takes a
// scan-order operator  op(p, q)  where p precedes q in scan order; a forward
// (time-order) scan passes p (x) q, a reverse scan passes q (x) p, so the
// left operand of the paper's operator always stays the earlier time step
// (the reversed all-prefix-sums of Sec. II-B).
#pragma once
#include "kf_ops.hpp"

namespace kfs {

constexpr int WAVE = 64;

template <class E> KF_DEV E shfl_up(E x, int d) {
  each(x, [&](auto& v, int) { v = __shfl_up(v, d, WAVE); });
  return x;
}
template <class E> KF_DEV E shfl_down(E x, int d) {
  each(x, [&](auto& v, int) { v = __shfl_down(v, d, WAVE); });
  return x;
}

template <class E> KF_DEV E bcast_lane0(E x) {
  each(x, [&](auto& v, int) { v = __shfl(v, 0, WAVE); });
  return x;
}

// Inclusive scan across the 64 lanes of a wavefront (Hillis-Steele over lanes,
// Algorithm 1 at wavefront scale): after it, lane l holds x_0 .. x_l.
template <class E, class Op> KF_DEV void wave_inclusive_scan(E& x, int lane, Op op) {
#pragma unroll 1
  for (int s = 1; s < WAVE; s <<= 1) {
    E u = shfl_up(x, s);
    if (lane >= s) x = op(u, x);
  }
}

// ---------------------------------------------------------------------------
// Publication of tile results between workgroups.
//
// On gfx950 every agent-scope acquire or release costs a whole-L2 operation
// (buffer_inv sc1 / buffer_wbl2 sc1 on the XCD's cache), which a spinning
// look-back would issue on every poll.  Instead every published word carries
// the pass's tag and is written and read with relaxed agent-scope atomics
// (plain sc1 accesses, coherent across XCDs, no cache maintenance):
//   status word  (tag << 2) | status            32 bit
//   payload      (tag << 32) | 32 value bits    64 bit, one per 32-bit half
// A reader accepts a word only when its tag matches, so no ordering between
// payload and status stores is needed: a status seen early only means the
// payload words are still on their way, and the reader polls them too.
// The tag of a pass is one more than the epoch word left by the previous
// pass (zero after the preparation kernel clears the control region).
// ---------------------------------------------------------------------------
using u64 = unsigned long long;

template <class R> constexpr int kWords = (int)(sizeof(R) / 4);  // 32-bit halves per scalar

KF_DEV u64 ld_relaxed(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
KF_DEV void st_relaxed(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
KF_DEV unsigned ld_relaxed(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
KF_DEV void st_relaxed(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

KF_DEV unsigned half_bits(float v, int) { return __float_as_uint(v); }
KF_DEV unsigned half_bits(double v, int h) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return h ? (unsigned)(b >> 32) : (unsigned)b;
}

// The lanes of a wavefront publish x together: lane l writes words l, l+64, ...
// (word w holds half w % kWords of scalar w / kWords, in storage order).
template <class R, class E> KF_DEV void tag_publish(u64* __restrict__ p, E& x, unsigned tag,
                                                    int lane) {
  constexpr int NW = E::SIZE * kWords<R>;
#pragma unroll
  for (int w0 = 0; w0 < NW; w0 += WAVE) {
    const int w = w0 + lane;
    if (w < NW) {
      const int si = w / kWords<R>, h = w % kWords<R>;
      R val = R(0);
      each(x, [&](R& v, int k) { val = (k == si) ? v : val; });
      st_relaxed(p + w, ((u64)tag << 32) | (u64)half_bits(val, h));
    }
  }
}

// One attempt to read a whole published element into this lane; false if any
// word does not carry the tag yet.
template <class R, class E> KF_DEV bool tag_try_load(E& x, const u64* __restrict__ p,
                                                     unsigned tag) {
  bool ok = true;
  each(x, [&](R& v, int k) {
    if constexpr (sizeof(R) == 4) {
      const u64 w = ld_relaxed(p + k);
      ok = ok & ((unsigned)(w >> 32) == tag);
      v = __uint_as_float((unsigned)w);
    } else {
      const u64 lo = ld_relaxed(p + 2 * k), hi = ld_relaxed(p + 2 * k + 1);
      ok = ok & ((unsigned)(lo >> 32) == tag) & ((unsigned)(hi >> 32) == tag);
      v = __longlong_as_double((long long)(((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull)));
    }
  });
  return ok;
}

// Look-back status values.
constexpr int LB_EMPTY = 0;
constexpr int LB_AGG = 1;     // the tile's own aggregate is published
constexpr int LB_PREFIX = 2;  // the tile's inclusive (anchored) prefix is published

// Bounded waits.  A legitimate wait lasts as long as one tile's fold
// (microseconds); the bound (~2^24 polls, about a second) only guarantees
// that every wave exits even if a predecessor never publishes.  On expiry the
// wait gives up, the caller continues with whatever it read, and the sticky
// error word *err is raised so the host can tell the result is invalid.
constexpr unsigned LB_SPIN_LIMIT = 1u << 24;

KF_DEV void lb_publish_flag(int* f, unsigned tag, int status) {
  __hip_atomic_store(f, (int)((tag << 2) | (unsigned)status), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
KF_DEV int lb_wait_flag(const int* f, unsigned tag, unsigned* err) {
  const unsigned want = tag & 0x3fffffffu;
  unsigned spins = 0;
  while (true) {
    const unsigned v =
        (unsigned)__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((v >> 2) == want && (v & 3u) != 0u) return (int)(v & 3u);
    if (++spins >= LB_SPIN_LIMIT) {
      atomicOr(err, 1u);
      return LB_PREFIX;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}
template <class R, class E> KF_DEV void tag_load(E& x, const u64* __restrict__ p, unsigned tag,
                                                 unsigned* err) {
  unsigned spins = 0;
  while (!tag_try_load<R>(x, p, tag)) {
    if (++spins >= LB_SPIN_LIMIT) {
      atomicOr(err, 1u);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Windowed look-back executed by the whole workgroup (BLOCK threads).
//
// Tile `t` (scan order) needs the combination of all tiles before it.  A
// window covers BLOCK*G tiles: thread i takes the G consecutive tiles
// j-iG-G+1 .. j-iG (j = t-1 for the first window) and waits for their status
// words nearest first; the nearest tile in the window whose anchored prefix is
// published ends the search.  Each thread folds its tiles in scan order (the
// published prefix, expanded with `expand`, then the later aggregates), each
// wavefront reduces its lanes with a tree in scan order (higher lane =
// earlier), skipping levels no lane needs, the wavefront partials are folded
// through LDS (higher wavefront = earlier), and windows are folded right to
// left.  Every thread polls and loads its own tiles at once, so a window costs
// one round of memory latency.  Tile t-1 is looked at first on its own: if its
// anchored prefix is already published, that is the answer.  Block-uniform control flow: every thread of
// the workgroup must call it.  Returns, in every thread, the exclusive prefix
// of tile t as an element.
//   load_agg(idx, E&)    : element published with LB_AGG by tile idx
//   expand(idx, E&)      : element form of tile idx's anchored prefix
//   s_part, s_lp         : LDS scratch, BLOCK/64 entries each
template <int BLOCK, class E, class Op, class LoadAgg, class Expand, class TryExpand>
KF_DEV E lookback(const int* __restrict__ flags, unsigned* err, unsigned tag, long t, int G, Op op,
                  LoadAgg load_agg, Expand expand, TryExpand try_expand, E* s_part, int* s_lp) {
  constexpr int NW = BLOCK / WAVE;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  // Fast path: the nearest predecessor publishes its anchored prefix.  Every
  // payload word carries the pass tag, so a payload read whole with the tag
  // is that prefix: one thread polls the payload and the status word
  // together (one round of memory latency per poll) and hands the prefix to
  // the workgroup through LDS; a status of LB_AGG without the prefix sends
  // the workgroup to the windowed look-back.
  if (tid == 0) {
    const unsigned want = tag & 0x3fffffffu;
    unsigned spins = 0;
    int st = LB_EMPTY;
    while (true) {
      E v;
      if (try_expand(t - 1, v)) {
        s_part[0] = v;
        st = LB_PREFIX;
        break;
      }
      const unsigned fv = (unsigned)__hip_atomic_load(flags + (t - 1), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      if ((fv >> 2) == want && (fv & 3u) == (unsigned)LB_AGG) {
        st = LB_AGG;
        break;
      }
      if (++spins >= LB_SPIN_LIMIT) {  // give up: the result is flagged invalid
        atomicOr(err, 1u);
        s_part[0] = v;
        st = LB_PREFIX;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    s_lp[0] = st;
  }
  __syncthreads();
  const int f1 = s_lp[0];
  if (f1 == LB_PREFIX) {
    const E v = s_part[0];
    __syncthreads();  // s_part is scratch of the caller's later steps
    return v;
  }
  __syncthreads();
  E acc;
  bool have = false;
  long j = t - 1;
#pragma unroll 1
  while (true) {
    const long hi = j - (long)tid * G;  // this thread's latest tile
    int gp = G;                          // offset of its nearest published prefix
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
      const long idx = hi - g;
      if (idx < 0) break;
      if (lb_wait_flag(flags + idx, tag, err) == LB_PREFIX) {
        gp = g;
        break;
      }
    }
    const unsigned long long pm = __ballot(gp < G);
    if (lane == 0) s_lp[wid] = pm ? (__ffsll((long long)pm) - 1) : WAVE;
    __syncthreads();
    int first = BLOCK;  // first thread (nearest tiles first) holding a published prefix
#pragma unroll
    for (int w = NW - 1; w >= 0; --w)
      if (s_lp[w] < WAVE) first = w * WAVE + s_lp[w];
    const bool found = first < BLOCK;
    const int last = found ? first : BLOCK - 1;  // last thread taking part
    E v;
    set_identity(v);
    if (tid <= last) {
      const bool anchored = (tid == first);
      int g = anchored ? gp - 1 : G - 1;
      if (anchored) expand(hi - gp, v); else load_agg(hi - g--, v);
#pragma unroll 1
      for (; g >= 0; --g) {
        E u;
        load_agg(hi - g, u);
        v = op(v, u);
      }
    }
    // wavefront tree: at level s, lane l (multiple of 2s) folds in lane l+s (earlier)
    const int lw = last - wid * WAVE;  // last lane of this wavefront taking part
#pragma unroll 1
    for (int s = 1; s <= lw && s < WAVE; s <<= 1) {
      E u = shfl_down(v, s);
      if ((lane & (2 * s - 1)) == 0 && lane + s <= lw) v = op(u, v);
    }
    if (lane == 0 && lw >= 0) s_part[wid] = v;
    __syncthreads();
    const int nw = last / WAVE + 1;  // wavefronts taking part
    E w = s_part[nw - 1];
#pragma unroll 1
    for (int q = nw - 2; q >= 0; --q) w = op(w, s_part[q]);
    acc = have ? op(w, acc) : w;
    have = true;
    __syncthreads();  // s_part and s_lp are reused by the next window
    if (found) break;
    j -= (long)BLOCK * G;
  }
  return acc;
}

}  // namespace kfs

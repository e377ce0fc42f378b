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

// Flat global-memory access to an element (SIZE scalars, storage order).
template <class E, class R> KF_DEV void gload(E& x, const R* __restrict__ p) {
  each(x, [&](R& v, int k) { v = p[k]; });
}
template <class E, class R> KF_DEV void gstore(R* __restrict__ p, E& x) {
  each(x, [&](R& v, int k) { p[k] = v; });
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

// Look-back status words.
constexpr int LB_EMPTY = 0;
constexpr int LB_AGG = 1;     // the tile's own aggregate is published
constexpr int LB_PREFIX = 2;  // the tile's inclusive (anchored) prefix is published

KF_DEV int lb_load_flag(const int* f) {
  return __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
KF_DEV void lb_store_flag(int* f, int v) {
  __hip_atomic_store(f, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Bounded wait for a predecessor's status word.  A legitimate wait lasts as
// long as one tile's fold (microseconds); the bound (~2^24 polls, about a
// second) only guarantees that every wave exits even if a predecessor never
// publishes.  On expiry the wait reports LB_PREFIX, the caller continues with
// whatever payload is there, and the sticky error word *err is raised so the
// host can tell the result is invalid.
constexpr unsigned LB_SPIN_LIMIT = 1u << 24;
KF_DEV int lb_wait_flag(const int* f, unsigned* err) {
  int v = lb_load_flag(f);
  unsigned spins = 0;
  while (v == LB_EMPTY) {
    __builtin_amdgcn_s_sleep(1);
    v = lb_load_flag(f);
    if (++spins >= LB_SPIN_LIMIT) {
      atomicOr(err, 1u);
      return LB_PREFIX;
    }
  }
  return v;
}

// Windowed look-back executed by one full wavefront.
//
// Tile `t` (scan order) needs the combination of all tiles before it.  Lane l
// inspects tile t-1-l-64w of window w; the nearest tile whose anchored prefix
// is published ends the search.  The window's elements are reduced with a
// lane tree in scan order (higher lane = earlier), skipping levels that no
// lane needs, and windows are folded right to left.  Returns, in every lane,
// the exclusive prefix of tile t as an element (the anchored prefix is
// expanded with `expand`).
//   load_agg(idx, E&)    : element published with LB_AGG by tile idx
//   expand(idx, E&)      : element form of tile idx's anchored prefix
template <class E, class Op, class LoadAgg, class Expand>
KF_DEV E lookback(const int* __restrict__ flags, unsigned* err, long t, int lane, Op op,
                  LoadAgg load_agg, Expand expand) {
  E acc;
  bool have = false;
  long j = t - 1;
#pragma unroll 1
  while (true) {
    const long idx = j - lane;
    int f = LB_PREFIX;  // lanes before tile 0 behave as "past the anchor"
    if (idx >= 0) f = lb_wait_flag(flags + idx, err);
    const unsigned long long pm = __ballot(f == LB_PREFIX && idx >= 0);
    const int lp = pm ? (__ffsll((long long)pm) - 1) : WAVE - 1;  // last lane taking part
    E v;
    if (lane < lp) {
      load_agg(idx, v);
    } else if (lane == lp) {
      if (pm) expand(idx, v); else load_agg(idx, v);
    } else {
      set_identity(v);
    }
    // lane tree: at level s, lane l (multiple of 2s) folds in lane l+s (earlier)
#pragma unroll 1
    for (int s = 1; s <= lp; s <<= 1) {
      E u = shfl_down(v, s);
      if ((lane & (2 * s - 1)) == 0 && lane + s <= lp) v = op(u, v);
    }
    E w = bcast_lane0(v);
    acc = have ? op(w, acc) : w;
    have = true;
    if (pm) break;
    j -= WAVE;
  }
  return acc;
}

}  // namespace kfs

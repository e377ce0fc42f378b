// kf_tree.hpp -- device-wide scans with one kernel launch per tree level,
// over elements kept in global memory: Hillis-Steele (Algorithm 1), Blelloch
// (Algorithm 2), the in-place Ladner-Fischer circuit (Algorithm 3) and the
// hybrid of Sengupta et al. (Algorithm 4, threshold N).  This is the structure
// the paper runs on its GPUs; it is offered beside the single-pass look-back
// scans for comparison (KF_SCAN_HILLIS_STEELE, _BLELLOCH, _LADNER_FISCHER,
// _SENGUPTA_A, _SENGUPTA_B).
//
// Sequence s of a level of n positions occupies SIZE * n scalars from
// (s * SIZE * n).  Inside, the in-place scans (Blelloch, Ladner-Fischer) store
// each element whole; Hillis-Steele and Sengupta, whose levels are read at
// consecutive positions, store a structure of arrays (elem_load).  Scan order is time order for the filter and
// descending time for the two reverse scans (position p is row T-1-p), whose
// operator takes its operands swapped (reading of the reversed all-prefix-sums
// of Sec. II-B), as in the look-back kernels.  Positions p >= T hold the
// two-sided identity (padding to a power of two).  Hillis-Steele ping-pongs
// between two buffers, so every level reads only the previous level's values;
// Blelloch works in place and rebuilds each element from the inputs in its
// final pass (exclusive -> inclusive); Ladner-Fischer works in place and is
// inclusive; Sengupta keeps one array per reduction level in the second
// buffer, scans the top level (N positions) with Hillis-Steele, and sweeps
// back down.  Every launch is described by one host-side plan (tree_plan),
// which also gives the exact number of operator applications of each scan.
#pragma once
#include <vector>

#include "../../include/kfscan.h"
#include "kf_kernels.hpp"

namespace kfs {

template <class R> struct TreeIO {
  const R* cst;
  const R* y;
  const R* m_in;   // filter moments (reverse scans)
  const R* P_in;
  R* m_out;
  R* P_out;
  long T;          // steps per sequence
  long Tp;         // scan positions per sequence (T, or T padded to a power of two)
  TvModel<R> tv;   // per-step model of a time-varying problem (else unused)
};

// Element p of a level of n positions, in one of two layouts.  AOS: the
// element's SIZE scalars are contiguous, so a lane moves whole 16-byte pieces
// of one element and every cache line it fetches is used whole, also when the
// lanes of a wave touch elements 2s apart (the upper levels of the in-place
// up- and down-sweeps).  Structure of arrays: scalar f of all positions is
// contiguous, so a wave reading consecutive positions issues one line-sized
// request per scalar -- fewer requests than AOS when the positions are
// consecutive (Hillis-Steele levels, Sengupta's reduce and down-sweep), but
// one line per scalar and lane once the stride passes a line.
template <bool AOS, class E, class R>
KF_DEV void elem_load(E& x, const R* __restrict__ X, long n, long p) {
  if constexpr (AOS) {
    const R* __restrict__ e = X + p * (long)E::SIZE;
    each(x, [&](R& v, int f) { v = e[f]; });
  } else {
    each(x, [&](R& v, int f) { v = X[(long)f * n + p]; });
  }
}
template <bool AOS, class E, class R>
KF_DEV void elem_store(R* __restrict__ X, long n, long p, E& x) {
  if constexpr (AOS) {
    R* __restrict__ e = X + p * (long)E::SIZE;
    each(x, [&](R& v, int f) { e[f] = v; });
  } else {
    each(x, [&](R& v, int f) { X[(long)f * n + p] = v; });
  }
}

template <int N, class R> KF_DEV void store_sym(R* __restrict__ Po, long k, const R (&C)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) Po[k * N * N + r * N + c] = (c >= r) ? C[r][c] : C[c][r];
}

// Forward filter (Algorithm 5): position p = row p; inclusive prefix (b, C) =
// (x_{k|k}, P_{k|k}).
template <int N, int M, class P, bool TV = false> struct TreeFilter {
  using R = typename P::R;
  using E = FElem<N, R>;
  const R* cst;
  const R* y;
  R* mo;
  R* Po;
  long T;
  TvModel<R> tv;
  KF_DEV TreeFilter(const TreeIO<R>& io, long seq)
      : cst(io.cst), y(io.y + seq * io.T * M), mo(io.m_out + seq * io.T * N),
        Po(io.P_out + seq * io.T * N * N), T(io.T), tv(io.tv) {}
  KF_DEV static E op(const E& a, const E& b) { return fcombine<N, P>(a, b); }
  KF_DEV E element(long p) const {
    E e;
    if (p >= T) {
      set_identity(e);
      return e;
    }
    R yk[M];
#pragma unroll
    for (int c = 0; c < M; ++c) yk[c] = y[p * M + c];
    if constexpr (TV) return filter_element_tv<N, M, P>(tv, p, yk);
    else return filter_element<N, M, R>(cst, p, yk);
  }
  KF_DEV void extract(long p, const E& s) const {
#pragma unroll
    for (int r = 0; r < N; ++r) mo[p * N + r] = s.b[r];
    store_sym<N, R>(Po, p, s.C);
  }
};

// RTS smoother (Algorithm 6): position p = row T-1-p; inclusive suffix (g, L)
// = (x_{k|T}, P_{k|T}).
template <int N, int M, class P, bool TV = false> struct TreeRts {
  using R = typename P::R;
  using E = SElem<N, R>;
  const R* cst;
  const R* mf;
  const R* Pf;
  R* mo;
  R* Po;
  long T;
  TvModel<R> tv;
  KF_DEV TreeRts(const TreeIO<R>& io, long seq)
      : cst(io.cst), mf(io.m_in + seq * io.T * N), Pf(io.P_in + seq * io.T * N * N),
        mo(io.m_out + seq * io.T * N), Po(io.P_out + seq * io.T * N * N), T(io.T),
        tv(io.tv) {}
  KF_DEV static E op(const E& a, const E& b) { return scombine<N, P>(b, a); }
  KF_DEV E element(long p) const {
    E e;
    if (p >= T) {
      set_identity(e);
      return e;
    }
    const long k = T - 1 - p;
    R x[N], Pk[N][N];
    load_state<N, R>(mf, Pf, k, x, Pk);
    if constexpr (TV) return rts_element_tv<N, P>(tv, T, k, x, Pk);
    else return rts_element<N, M, P>(cst, T, k, x, Pk);
  }
  KF_DEV void extract(long p, const E& s) const {
    const long k = T - 1 - p;
#pragma unroll
    for (int r = 0; r < N; ++r) mo[k * N + r] = s.g[r];
    store_sym<N, R>(Po, k, s.L);
  }
};

// Two-filter smoother (Algorithm 7): position p = row T-1-p over
// (a_2, ..., a_T, e); the inclusive suffix's (eta, J) is combined with the
// filter moments of that row.
template <int N, int M, class P, bool TV = false> struct TreeTwoFilter {
  using R = typename P::R;
  using E = FElem<N, R>;
  const R* cst;
  const R* y;
  const R* mf;
  const R* Pf;
  R* mo;
  R* Po;
  long T;
  TvModel<R> tv;
  KF_DEV TreeTwoFilter(const TreeIO<R>& io, long seq)
      : cst(io.cst), y(io.y + seq * io.T * M), mf(io.m_in + seq * io.T * N),
        Pf(io.P_in + seq * io.T * N * N), mo(io.m_out + seq * io.T * N),
        Po(io.P_out + seq * io.T * N * N), T(io.T), tv(io.tv) {}
  KF_DEV static E op(const E& a, const E& b) { return fcombine<N, P>(b, a); }
  KF_DEV E element(long p) const {
    E e;
    if (p >= T) {
      set_identity(e);
      return e;
    }
    const long k = T - 1 - p;
    R yk[M];
#pragma unroll
    for (int c = 0; c < M; ++c) yk[c] = (k + 1 < T) ? y[(k + 1) * M + c] : R(0);
    if constexpr (TV) {
      if (k == T - 1) set_identity(e);
      else e = filter_element_tv<N, M, P>(tv, k + 1, yk);
      return e;
    } else {
      return tf_element<N, M, R>(cst, T, k, yk);
    }
  }
  KF_DEV void extract(long p, const E& s) const {
    const long k = T - 1 - p;
    R xf[N], Pk[N][N], xs[N], Ps[N][N];
    load_state<N, R>(mf, Pf, k, xf, Pk);
    tf_combine<N, P>(xf, Pk, s.e, s.J, xs, Ps);
#pragma unroll
    for (int r = 0; r < N; ++r) mo[k * N + r] = xs[r];
    store_sym<N, R>(Po, k, Ps);
  }
};

constexpr int kTreeBlock = 256;

// Positions p of sequence blockIdx.y: build the elements.
template <class Pipe, bool AOS>
__global__ __launch_bounds__(kTreeBlock) void k_tree_build(TreeIO<typename Pipe::R> io,
                                                          typename Pipe::R* X) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= io.Tp) return;
  Pipe pp(io, seq);
  E e = pp.element(p);
  elem_store<AOS>(X + seq * E::SIZE * io.Tp, io.Tp, p, e);
}

// Algorithm 1, one level with offset s over a level of n positions:
// Xout[p] = Xin[p - s] (x) Xin[p] for p >= s, Xout[p] = Xin[p] below.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_hs_level(const typename Pipe::R* Xin,
                                                        typename Pipe::R* Xout, long n, long s) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= n) return;
  const long off = seq * E::SIZE * n;
  E b;
  elem_load<false>(b, Xin + off, n, p);
  if (p >= s) {
    E a;
    elem_load<false>(a, Xin + off, n, p - s);
    b = Pipe::op(a, b);
  }
  elem_store<false>(Xout + off, n, p, b);
}

// Up-sweep level with offset s, shared by Algorithms 2 and 3: the i-th active
// position is k = (i+1)*2s - 1 (0-based; the paper's k = i + 2^(d+1) with
// i = 0, 2^(d+1), ...), X[k] = X[k - s] (x) X[k].
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_bl_up(TreeIO<typename Pipe::R> io,
                                                     typename Pipe::R* X, long s) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long i = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  const long k = (i + 1) * 2 * s - 1;
  if (k >= io.Tp) return;
  typename Pipe::R* x = X + seq * E::SIZE * io.Tp;
  E a, b;
  elem_load<true>(a, x, io.Tp, k - s);
  elem_load<true>(b, x, io.Tp, k);
  b = Pipe::op(a, b);
  elem_store<true>(x, io.Tp, k, b);
}

// Algorithm 2: the root takes the neutral element.
template <class Pipe>
__global__ void k_bl_root(TreeIO<typename Pipe::R> io, typename Pipe::R* X) {
  using E = typename Pipe::E;
  if (threadIdx.x != 0) return;
  E e;
  set_identity(e);
  elem_store<true>(X + (long)blockIdx.y * E::SIZE * io.Tp, io.Tp, io.Tp - 1, e);
}

// Algorithm 2, down-sweep level with offset s: t = X[k - s]; X[k - s] = X[k];
// X[k] = X[k] (x) t.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_bl_down(TreeIO<typename Pipe::R> io,
                                                       typename Pipe::R* X, long s) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long i = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  const long k = (i + 1) * 2 * s - 1;
  if (k >= io.Tp) return;
  typename Pipe::R* x = X + seq * E::SIZE * io.Tp;
  E l, r;
  elem_load<true>(l, x, io.Tp, k - s);
  elem_load<true>(r, x, io.Tp, k);
  elem_store<true>(x, io.Tp, k - s, r);
  r = Pipe::op(r, l);
  elem_store<true>(x, io.Tp, k, r);
}

// Algorithm 3, down-sweep level with offset s: for m = 1, 2, ... the paper's
// a_{i + s} <- a_i (x) a_{i + s} with i = 2sm, i.e. 0-based
// X[2sm + s - 1] = X[2sm - 1] (x) X[2sm + s - 1].  The positions written in a
// level are never read in it.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_lf_down(TreeIO<typename Pipe::R> io,
                                                       typename Pipe::R* X, long s) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long m = (long)blockIdx.x * kTreeBlock + threadIdx.x + 1;
  const long i = 2 * s * m - 1;
  const long j = i + s;
  if (j >= io.Tp) return;
  typename Pipe::R* x = X + seq * E::SIZE * io.Tp;
  E a, b;
  elem_load<true>(a, x, io.Tp, i);
  elem_load<true>(b, x, io.Tp, j);
  b = Pipe::op(a, b);
  elem_store<true>(x, io.Tp, j, b);
}

// Algorithm 4, reduce pass: hi[i] = lo[2i] (x) lo[2i+1] (0-based; the paper's
// a^(d)_i = a^(d-1)_{2i-1} (x) a^(d-1)_{2i}), levels of nlo and nhi positions.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_sg_reduce(const typename Pipe::R* lo, long nlo,
                                                         typename Pipe::R* hi, long nhi) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long i = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (i >= nhi) return;
  const typename Pipe::R* l = lo + seq * E::SIZE * nlo;
  E a, b;
  elem_load<false>(a, l, nlo, 2 * i);
  elem_load<false>(b, l, nlo, 2 * i + 1);
  a = Pipe::op(a, b);
  elem_store<false>(hi + seq * E::SIZE * nhi, nhi, i, a);
}

// Algorithm 4, down-sweep into a level of nlo positions from the scanned level
// above it (nhi = nlo / 2 positions).  0-based position i >= 1: odd i (the
// paper's even 1-based index) takes hi[(i-1)/2] whole; even i takes
// hi[i/2 - 1] (x) lo[i]; position 0 keeps its value.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_sg_down(const typename Pipe::R* hi, long nhi,
                                                       typename Pipe::R* lo, long nlo) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long i = (long)blockIdx.x * kTreeBlock + threadIdx.x + 1;
  if (i >= nlo) return;
  const typename Pipe::R* h = hi + seq * E::SIZE * nhi;
  typename Pipe::R* l = lo + seq * E::SIZE * nlo;
  E a;
  if (i & 1) {
    elem_load<false>(a, h, nhi, (i - 1) / 2);
  } else {
    E b;
    elem_load<false>(a, h, nhi, i / 2 - 1);
    elem_load<false>(b, l, nlo, i);
    a = Pipe::op(a, b);
  }
  elem_store<false>(l, nlo, i, a);
}

// Outputs of positions p < T from the scan result (a level of n positions):
// inclusive as it stands, or exclusive (Blelloch) combined with the element
// rebuilt from the inputs.
template <class Pipe, bool EXCLUSIVE, bool AOS>
__global__ __launch_bounds__(kTreeBlock) void k_tree_extract(TreeIO<typename Pipe::R> io,
                                                            const typename Pipe::R* X, long n) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= io.T) return;
  Pipe pp(io, seq);
  E s;
  elem_load<AOS>(s, X + seq * E::SIZE * n, n, p);
  if (EXCLUSIVE) s = Pipe::op(s, pp.element(p));
  pp.extract(p, s);
}

inline long pow2_at_least(long T) {
  long p = 1;
  while (p < T) p <<= 1;
  return p;
}

// Threshold of KF_SCAN_SENGUPTA_B: the top level that Hillis-Steele scans has
// this many positions (the paper's tuned N of 14750..20000, as the power of two
// that its length rounds to).
constexpr long kSenguptaBN = 16384;

enum TreeKind {
  TK_BUILD, TK_HS, TK_BL_UP, TK_BL_ROOT, TK_BL_DOWN, TK_LF_DOWN, TK_SG_REDUCE, TK_SG_DOWN,
  TK_EXTRACT, TK_EXTRACT_EXCL
};

// A level array: buffer 0 or 1, its first position inside the buffer (in units
// of nseq * SIZE scalars) and its positions per sequence.
struct TreeArray {
  int buf;
  long pos, n;
};

struct TreeStep {
  TreeKind kind;
  long s;            // offset of an HS / up-sweep / down-sweep level
  TreeArray in, out;
  long threads;      // threads per sequence
  long combines;     // operator applications per sequence
};

// Every launch of one scan over T steps.  Positions: HS T, the others T padded
// to a power of two P.  Buffer 0 holds P (HS: T) positions; buffer 1 the HS
// ping-pong copy, or Sengupta's levels 1..d* and its top-level ping buffer
// (P - N' + N' = P positions).
inline std::vector<TreeStep> tree_plan(int scan, long T) {
  std::vector<TreeStep> v;
  auto add = [&](TreeKind k, long s, TreeArray in, TreeArray out, long threads, long comb) {
    v.push_back(TreeStep{k, s, in, out, threads, comb});
  };
  const bool hs = scan == KF_SCAN_HILLIS_STEELE;
  const long P = hs ? T : pow2_at_least(T);
  const TreeArray base{0, 0, P};
  add(TK_BUILD, 0, base, base, P, 0);
  if (hs) {
    TreeArray a = base, b{1, 0, P};
    for (long s = 1; s < P; s <<= 1) {
      add(TK_HS, s, a, b, P, P - s);
      const TreeArray t = a;
      a = b;
      b = t;
    }
    add(TK_EXTRACT, 0, a, a, T, 0);
  } else if (scan == KF_SCAN_BLELLOCH) {
    for (long s = 1; s < P; s <<= 1) add(TK_BL_UP, s, base, base, P / (2 * s), P / (2 * s));
    add(TK_BL_ROOT, 0, base, base, 1, 0);
    for (long s = P / 2; s >= 1; s >>= 1) add(TK_BL_DOWN, s, base, base, P / (2 * s), P / (2 * s));
    add(TK_EXTRACT_EXCL, 0, base, base, T, T);
  } else if (scan == KF_SCAN_LADNER_FISCHER) {
    for (long s = 1; s < P; s <<= 1) add(TK_BL_UP, s, base, base, P / (2 * s), P / (2 * s));
    // the first down-sweep level (s = P/2) has no active position
    for (long s = P / 4; s >= 1; s >>= 1)
      add(TK_LF_DOWN, s, base, base, P / (2 * s) - 1, P / (2 * s) - 1);
    add(TK_EXTRACT, 0, base, base, T, 0);
  } else {  // Sengupta, threshold 1 (A) or kSenguptaBN (B)
    long Nt = pow2_at_least(scan == KF_SCAN_SENGUPTA_B ? kSenguptaBN : 1);
    if (Nt > P) Nt = P;
    std::vector<TreeArray> lvl{base};
    for (long n = P / 2, pos = 0; n >= Nt; pos += n, n /= 2) {
      lvl.push_back(TreeArray{1, pos, n});
      add(TK_SG_REDUCE, 0, lvl[lvl.size() - 2], lvl.back(), n, n);
    }
    // Hillis-Steele on the top level, ping-ponging with the space after it
    TreeArray a = lvl.back(), b{1, P - Nt, Nt};
    for (long s = 1; s < Nt; s <<= 1) {
      add(TK_HS, s, a, b, Nt, Nt - s);
      const TreeArray t = a;
      a = b;
      b = t;
    }
    lvl.back() = a;
    for (long d = (long)lvl.size() - 2; d >= 0; --d)
      add(TK_SG_DOWN, 0, lvl[d + 1], lvl[d], lvl[d].n - 1, lvl[d].n / 2 - 1);
    add(TK_EXTRACT, 0, lvl[0], lvl[0], T, 0);
  }
  return v;
}

// Enqueue one whole tree scan of pipeline Pipe over nseq sequences.  X0 and X1
// hold nseq * E::SIZE * P scalars each (X1 only for Hillis-Steele and
// Sengupta).
template <class Pipe>
void tree_scan(TreeIO<typename Pipe::R> io, int scan, long nseq, typename Pipe::R* X0,
               typename Pipe::R* X1, hipStream_t st) {
  using R = typename Pipe::R;
  using E = typename Pipe::E;
  auto grid = [&](long n) {
    return dim3((unsigned)((n + kTreeBlock - 1) / kTreeBlock), (unsigned)nseq);
  };
  auto ptr = [&](const TreeArray& a) {
    return (a.buf ? X1 : X0) + a.pos * nseq * (long)E::SIZE;
  };
  const bool aos = scan == KF_SCAN_BLELLOCH || scan == KF_SCAN_LADNER_FISCHER;
  for (const TreeStep& t : tree_plan(scan, io.T)) {
    if (t.threads <= 0) continue;
    const dim3 g = grid(t.threads), b(kTreeBlock);
    switch (t.kind) {
      case TK_BUILD:
        if (aos) hipLaunchKernelGGL((k_tree_build<Pipe, true>), g, b, 0, st, io, ptr(t.out));
        else hipLaunchKernelGGL((k_tree_build<Pipe, false>), g, b, 0, st, io, ptr(t.out));
        break;
      case TK_HS:
        hipLaunchKernelGGL((k_hs_level<Pipe>), g, b, 0, st, (const R*)ptr(t.in), ptr(t.out),
                           t.in.n, t.s);
        break;
      case TK_BL_UP:
        hipLaunchKernelGGL((k_bl_up<Pipe>), g, b, 0, st, io, ptr(t.out), t.s);
        break;
      case TK_BL_ROOT:
        hipLaunchKernelGGL((k_bl_root<Pipe>), dim3(1, (unsigned)nseq), dim3(64), 0, st, io,
                           ptr(t.out));
        break;
      case TK_BL_DOWN:
        hipLaunchKernelGGL((k_bl_down<Pipe>), g, b, 0, st, io, ptr(t.out), t.s);
        break;
      case TK_LF_DOWN:
        hipLaunchKernelGGL((k_lf_down<Pipe>), g, b, 0, st, io, ptr(t.out), t.s);
        break;
      case TK_SG_REDUCE:
        hipLaunchKernelGGL((k_sg_reduce<Pipe>), g, b, 0, st, (const R*)ptr(t.in), t.in.n,
                           ptr(t.out), t.out.n);
        break;
      case TK_SG_DOWN:
        hipLaunchKernelGGL((k_sg_down<Pipe>), g, b, 0, st, (const R*)ptr(t.in), t.in.n,
                           ptr(t.out), t.out.n);
        break;
      case TK_EXTRACT:
        if (aos)
          hipLaunchKernelGGL((k_tree_extract<Pipe, false, true>), g, b, 0, st, io,
                             (const R*)ptr(t.in), t.in.n);
        else
          hipLaunchKernelGGL((k_tree_extract<Pipe, false, false>), g, b, 0, st, io,
                             (const R*)ptr(t.in), t.in.n);
        break;
      case TK_EXTRACT_EXCL:  // Blelloch only
        hipLaunchKernelGGL((k_tree_extract<Pipe, true, true>), g, b, 0, st, io,
                           (const R*)ptr(t.in), t.in.n);
        break;
    }
  }
}

}  // namespace kfs

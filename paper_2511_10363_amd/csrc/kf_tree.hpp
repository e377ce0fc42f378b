// kf_tree.hpp -- device-wide Hillis-Steele (Algorithm 1) and Blelloch
// (Algorithm 2) scans, one kernel launch per tree level, over elements kept in
// global memory.  This is the structure the paper runs on its GPUs; it is
// offered beside the single-pass look-back scans for comparison
// (KF_SCAN_HILLIS_STEELE, KF_SCAN_BLELLOCH).
//
// Elements are stored as a structure of arrays per sequence: scalar f of scan
// position p of sequence s sits at X[(s * SIZE + f) * Tp + p], so the threads
// of a level read and write consecutive addresses.  Scan order is time order
// for the filter and descending time for the two reverse scans (position p is
// row T-1-p), whose operator takes its operands swapped (reading of the
// reversed all-prefix-sums of Sec. II-B), as in the look-back kernels.
// Positions p >= T hold the two-sided identity (padding to a power of two for
// Blelloch).  Hillis-Steele ping-pongs between two buffers, so every level
// reads only the previous level's values; Blelloch works in place and rebuilds
// each element from the inputs in its final pass (exclusive -> inclusive).
#pragma once
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
};

template <class E, class R> KF_DEV void soa_load(E& x, const R* __restrict__ X, long Tp, long p) {
  each(x, [&](R& v, int f) { v = X[(long)f * Tp + p]; });
}
template <class E, class R> KF_DEV void soa_store(R* __restrict__ X, long Tp, long p, E& x) {
  each(x, [&](R& v, int f) { X[(long)f * Tp + p] = v; });
}

template <int N, class R> KF_DEV void store_sym(R* __restrict__ Po, long k, const R (&C)[N][N]) {
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) Po[k * N * N + r * N + c] = (c >= r) ? C[r][c] : C[c][r];
}

// Forward filter (Algorithm 5): position p = row p; inclusive prefix (b, C) =
// (x_{k|k}, P_{k|k}).
template <int N, int M, class P> struct TreeFilter {
  using R = typename P::R;
  using E = FElem<N, R>;
  const R* cst;
  const R* y;
  R* mo;
  R* Po;
  long T;
  KF_DEV TreeFilter(const TreeIO<R>& io, long seq)
      : cst(io.cst), y(io.y + seq * io.T * M), mo(io.m_out + seq * io.T * N),
        Po(io.P_out + seq * io.T * N * N), T(io.T) {}
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
    return filter_element<N, M, R>(cst, p, yk);
  }
  KF_DEV void extract(long p, const E& s) const {
#pragma unroll
    for (int r = 0; r < N; ++r) mo[p * N + r] = s.b[r];
    store_sym<N, R>(Po, p, s.C);
  }
};

// RTS smoother (Algorithm 6): position p = row T-1-p; inclusive suffix (g, L)
// = (x_{k|T}, P_{k|T}).
template <int N, int M, class P> struct TreeRts {
  using R = typename P::R;
  using E = SElem<N, R>;
  const R* cst;
  const R* mf;
  const R* Pf;
  R* mo;
  R* Po;
  long T;
  KF_DEV TreeRts(const TreeIO<R>& io, long seq)
      : cst(io.cst), mf(io.m_in + seq * io.T * N), Pf(io.P_in + seq * io.T * N * N),
        mo(io.m_out + seq * io.T * N), Po(io.P_out + seq * io.T * N * N), T(io.T) {}
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
    return rts_element<N, M, P>(cst, T, k, x, Pk);
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
template <int N, int M, class P> struct TreeTwoFilter {
  using R = typename P::R;
  using E = FElem<N, R>;
  const R* cst;
  const R* y;
  const R* mf;
  const R* Pf;
  R* mo;
  R* Po;
  long T;
  KF_DEV TreeTwoFilter(const TreeIO<R>& io, long seq)
      : cst(io.cst), y(io.y + seq * io.T * M), mf(io.m_in + seq * io.T * N),
        Pf(io.P_in + seq * io.T * N * N), mo(io.m_out + seq * io.T * N),
        Po(io.P_out + seq * io.T * N * N), T(io.T) {}
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
    return tf_element<N, M, R>(cst, T, k, yk);
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
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_tree_build(TreeIO<typename Pipe::R> io,
                                                          typename Pipe::R* X) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= io.Tp) return;
  Pipe pp(io, seq);
  E e = pp.element(p);
  soa_store(X + seq * E::SIZE * io.Tp, io.Tp, p, e);
}

// Algorithm 1, one level with offset s: Xout[p] = Xin[p - s] (x) Xin[p] for p >= s.
template <class Pipe>
__global__ __launch_bounds__(kTreeBlock) void k_hs_level(TreeIO<typename Pipe::R> io,
                                                        const typename Pipe::R* Xin,
                                                        typename Pipe::R* Xout, long s) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= io.Tp) return;
  const long off = seq * E::SIZE * io.Tp;
  E b;
  soa_load(b, Xin + off, io.Tp, p);
  if (p >= s) {
    E a;
    soa_load(a, Xin + off, io.Tp, p - s);
    b = Pipe::op(a, b);
  }
  soa_store(Xout + off, io.Tp, p, b);
}

// Algorithm 2, up-sweep level with offset s: the i-th active position is
// k = (i+1)*2s - 1, X[k] = X[k - s] (x) X[k].
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
  soa_load(a, x, io.Tp, k - s);
  soa_load(b, x, io.Tp, k);
  b = Pipe::op(a, b);
  soa_store(x, io.Tp, k, b);
}

// Algorithm 2: the root takes the neutral element.
template <class Pipe>
__global__ void k_bl_root(TreeIO<typename Pipe::R> io, typename Pipe::R* X) {
  using E = typename Pipe::E;
  if (threadIdx.x != 0) return;
  E e;
  set_identity(e);
  soa_store(X + (long)blockIdx.y * E::SIZE * io.Tp, io.Tp, io.Tp - 1, e);
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
  soa_load(l, x, io.Tp, k - s);
  soa_load(r, x, io.Tp, k);
  soa_store(x, io.Tp, k - s, r);
  r = Pipe::op(r, l);
  soa_store(x, io.Tp, k, r);
}

// Outputs of positions p < T from the scan result: inclusive as it stands, or
// exclusive (Blelloch) combined with the element rebuilt from the inputs.
template <class Pipe, bool EXCLUSIVE>
__global__ __launch_bounds__(kTreeBlock) void k_tree_extract(TreeIO<typename Pipe::R> io,
                                                            const typename Pipe::R* X) {
  using E = typename Pipe::E;
  const long seq = blockIdx.y;
  const long p = (long)blockIdx.x * kTreeBlock + threadIdx.x;
  if (p >= io.T) return;
  Pipe pp(io, seq);
  E s;
  soa_load(s, X + seq * E::SIZE * io.Tp, io.Tp, p);
  if (EXCLUSIVE) s = Pipe::op(s, pp.element(p));
  pp.extract(p, s);
}

inline long pow2_at_least(long T) {
  long p = 1;
  while (p < T) p <<= 1;
  return p;
}

// Enqueue one whole tree scan of pipeline Pipe over nseq sequences.  X0 (and
// X1 for Hillis-Steele) hold nseq * E::SIZE * Tp scalars each.
template <class Pipe>
void tree_scan(TreeIO<typename Pipe::R> io, bool hillis_steele, long nseq, typename Pipe::R* X0,
               typename Pipe::R* X1, hipStream_t st) {
  using R = typename Pipe::R;
  auto grid = [&](long n) { return dim3((unsigned)((n + kTreeBlock - 1) / kTreeBlock), (unsigned)nseq); };
  hipLaunchKernelGGL((k_tree_build<Pipe>), grid(io.Tp), dim3(kTreeBlock), 0, st, io, X0);
  if (hillis_steele) {
    R* a = X0;
    R* b = X1;
    for (long s = 1; s < io.Tp; s <<= 1) {
      hipLaunchKernelGGL((k_hs_level<Pipe>), grid(io.Tp), dim3(kTreeBlock), 0, st, io,
                         (const R*)a, b, s);
      R* t = a;
      a = b;
      b = t;
    }
    hipLaunchKernelGGL((k_tree_extract<Pipe, false>), grid(io.T), dim3(kTreeBlock), 0, st, io,
                       (const R*)a);
  } else {
    for (long s = 1; s < io.Tp; s <<= 1)
      hipLaunchKernelGGL((k_bl_up<Pipe>), grid(io.Tp / (2 * s)), dim3(kTreeBlock), 0, st, io, X0,
                         s);
    hipLaunchKernelGGL((k_bl_root<Pipe>), dim3(1, (unsigned)nseq), dim3(64), 0, st, io, X0);
    for (long s = io.Tp / 2; s >= 1; s >>= 1)
      hipLaunchKernelGGL((k_bl_down<Pipe>), grid(io.Tp / (2 * s)), dim3(kTreeBlock), 0, st, io,
                         X0, s);
    hipLaunchKernelGGL((k_tree_extract<Pipe, true>), grid(io.T), dim3(kTreeBlock), 0, st, io,
                       (const R*)X0);
  }
}

}  // namespace kfs

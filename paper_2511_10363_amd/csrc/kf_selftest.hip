// kf_selftest.hip -- the look-back tile driver (scan_tile: fold, wavefront
// scan, windowed decoupled look-back with anchors, step walk) run with an
// operator whose results are exact, so that the device scan can be checked
// bit for bit against a host scan.
//
// Both tile drivers are covered: the thread driver of the register-resident
// scans (scan_tile) and the group driver of the wide-state scans
// (gscan_tile).
//
// The element is an affine map on pairs (v, M), v in Z_p^2, M in Z_p^{2x2}:
//   x -> A x + b  and  M -> A M + C  (A in Z_p^{2x2}, all arithmetic mod p).
// Composition is associative and not commutative, like the paper's
// operators (Sec. II-B asks only for associativity).  In scan order (p
// before q) the combined map is "p, then q":
//   op(p, q) = (A_q A_p, A_q b_p + b_q, A_q C_p + C_q).
// A map with A = 0 is constant, so whatever precedes it drops out: it plays
// the part of the paper's first filtering element (A_1 = 0) and last
// smoothing element (E_T = 0), and the anchored state of a prefix is its
// (b, C).  The forward scan gives the all-prefix-sums of Sec. II-B
// (s_k = a_1 ... a_k in composition order), the reverse scan the reversed
// all-prefix-sums (s_k = a_k ... a_T), with the same tile and thread order
// as the RTS and two-filter passes.
//
// Every value is an integer below p, p = 33554393 in FP64 and 2039 in FP32,
// so every sum of two products and a term, 2 (p-1)^2 + (p-1), stays below
// 2^52 (FP64) or 2^23 (FP32): exactly representable; the reduction mod p is
// done in integer arithmetic.
#include <cstdint>

#include "kf_inst.hpp"

namespace kfs {

template <class R> struct AffElem {
  R A[2][2];
  R b[2];
  R C[2][2];
  static constexpr int SIZE = 10;
};

template <class R, class F> KF_DEV void each(AffElem<R>& x, F f) {
  f(x.A[0][0], 0);
  f(x.A[0][1], 1);
  f(x.A[1][0], 2);
  f(x.A[1][1], 3);
  f(x.b[0], 4);
  f(x.b[1], 5);
  f(x.C[0][0], 6);
  f(x.C[0][1], 7);
  f(x.C[1][0], 8);
  f(x.C[1][1], 9);
}

template <class R> KF_DEV void set_identity(AffElem<R>& x) {
  each(x, [](R& v, int) { v = R(0); });
  x.A[0][0] = x.A[1][1] = R(1);
}

template <class R> KF_DEV bool decay_is_zero(const AffElem<R>& x) {
  return x.A[0][0] == R(0) && x.A[0][1] == R(0) && x.A[1][0] == R(0) && x.A[1][1] == R(0);
}

template <class R> constexpr long affine_modulus() { return sizeof(R) == 8 ? 33554393L : 2039L; }

template <class R> KF_DEV R modp(R x) {
  return R((long long)x % affine_modulus<R>());
}

// out = A x + y (2-vectors), exact then reduced
template <class R> KF_DEV void aff_mv(const R (&A)[2][2], const R (&x)[2], const R (&y)[2],
                                      R (&o)[2]) {
  const R o0 = modp(A[0][0] * x[0] + A[0][1] * x[1] + y[0]);
  const R o1 = modp(A[1][0] * x[0] + A[1][1] * x[1] + y[1]);
  o[0] = o0;
  o[1] = o1;
}
// O = A X + Y (2x2)
template <class R> KF_DEV void aff_mm(const R (&A)[2][2], const R (&X)[2][2], const R (&Y)[2][2],
                                      R (&O)[2][2]) {
  R t[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) t[i][j] = modp(A[i][0] * X[0][j] + A[i][1] * X[1][j] + Y[i][j]);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) O[i][j] = t[i][j];
}

template <class R, int L, bool REV> struct AffPipe {
  using E = AffElem<R>;
  const ScanArgs<R>& a;
  const R* __restrict__ in;   // [nseq][T][10]
  R* __restrict__ out;        // [nseq][T][6]
  long T, k0;
  KF_DEV AffPipe(const ScanArgs<R>& a_, const R* in_, R* out_) : a(a_), in(in_), out(out_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int tid) {
    T = s.T;
    if (REV) {
      const long tt = s.ntiles - 1 - t;
      k0 = tt * (long)(L * blockDim.x) + (long)(blockDim.x - 1 - tid) * L;
    } else {
      k0 = t * (long)(L * blockDim.x) + (long)tid * L;
    }
    in += s.row0 * E::SIZE;
    out += s.row0 * 6;
  }
  KF_DEV E load(long k) const {
    E e;
    each(e, [&](R& v, int i) { v = in[k * E::SIZE + i]; });
    return e;
  }
  // p precedes q in scan order: the map p, then q
  KF_DEV E op(const E& p, const E& q) const {
    E o;
    R zero2[2][2] = {{R(0), R(0)}, {R(0), R(0)}};
    aff_mm(q.A, p.A, zero2, o.A);
    aff_mv(q.A, p.b, q.b, o.b);
    aff_mm(q.A, p.C, q.C, o.C);
    return o;
  }
  KF_DEV E fold() const {
    E agg;
    set_identity(agg);
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
      const long k = REV ? k0 + L - 1 - j : k0 + j;
      if (k < T) agg = op(agg, load(k));
    }
    return agg;
  }
  KF_DEV void apply(St<2, R>& st, const E& e) const {
    aff_mv(e.A, st.v, e.b, st.v);
    aff_mm(e.A, st.m, e.C, st.m);
  }
  KF_DEV void initial(St<2, R>& st) const { st_zero(st); }
  KF_DEV void anchor(const E& e, St<2, R>& st) const {
    st.v[0] = e.b[0];
    st.v[1] = e.b[1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) st.m[i][j] = e.C[i][j];
  }
  KF_DEV void expand(const St<2, R>& st, E& e) const {
    set_identity(e);
    e.A[0][0] = e.A[1][1] = R(0);
    e.b[0] = st.v[0];
    e.b[1] = st.v[1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) e.C[i][j] = st.m[i][j];
  }
  KF_DEV void steps(St<2, R>& st, bool) const {
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
      const long k = REV ? k0 + L - 1 - j : k0 + j;
      if (k >= T) continue;
      apply(st, load(k));
      out[k * 6 + 0] = st.v[0];
      out[k * 6 + 1] = st.v[1];
      out[k * 6 + 2] = st.m[0][0];
      out[k * 6 + 3] = st.m[0][1];
      out[k * 6 + 4] = st.m[1][0];
      out[k * 6 + 5] = st.m[1][1];
    }
  }
};

template <class R, int BLOCK, int L, bool REV>
__global__ __launch_bounds__(BLOCK) void k_selftest_scan(ScanArgs<R> a, const R* __restrict__ in,
                                                         R* __restrict__ out) {
  AffPipe<R, L, REV> pp(a, in, out);
  scan_tile<AffPipe<R, L, REV>, 2, R, BLOCK, L>(pp, a);
}

// The same maps through the group tile driver of the wide-state scans
// (gscan_tile, glookback): every lane of a group of G holds the whole
// element (row r of a replicated element is the element), so the groups
// stand where the rows of a wide element would, and the driver's tiling,
// group scan, tagged per-row publication and windowed look-back over groups
// are checked bit for bit.  The state row packs (b, C): v = b0, m[0] = b1,
// m[1..4] = C.
template <class R> KF_DEV void set_identity_row(AffElem<R>& x, int) { set_identity(x); }

template <class R, int G, int BLOCK, int L, bool REV> struct AffGroupPipe {
  using E = AffElem<R>;
  static constexpr int NG = BLOCK / G;
  static_assert(G >= 5, "the state row holds 6 values");
  const ScanArgs<R>& a;
  const R* __restrict__ in;
  R* __restrict__ out;
  long T, k0;
  int r;
  KF_DEV AffGroupPipe(const ScanArgs<R>& a_, const R* in_, R* out_) : a(a_), in(in_), out(out_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int grp, int r_, GScr<G, R>*) {
    T = s.T;
    r = r_;
    if (REV) k0 = (s.ntiles - 1 - t) * (long)(L * NG) + (long)(NG - 1 - grp) * L;
    else k0 = t * (long)(L * NG) + (long)grp * L;
    in += s.row0 * E::SIZE;
    out += s.row0 * 6;
  }
  KF_DEV E load(long k) const {
    E e;
    each(e, [&](R& v, int i) { v = in[k * E::SIZE + i]; });
    return e;
  }
  KF_DEV E op(const E& p, const E& q) const {
    E o;
    R zero2[2][2] = {{R(0), R(0)}, {R(0), R(0)}};
    aff_mm(q.A, p.A, zero2, o.A);
    aff_mv(q.A, p.b, q.b, o.b);
    aff_mm(q.A, p.C, q.C, o.C);
    return o;
  }
  KF_DEV E fold() const {
    E agg;
    set_identity(agg);
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
      const long k = REV ? k0 + L - 1 - j : k0 + j;
      if (k < T) agg = op(agg, load(k));
    }
    return agg;
  }
  static KF_DEV void unpack(const WSt<G, R>& st, R (&v)[2], R (&m)[2][2]) {
    v[0] = st.v;
    v[1] = st.m[0];
    m[0][0] = st.m[1];
    m[0][1] = st.m[2];
    m[1][0] = st.m[3];
    m[1][1] = st.m[4];
  }
  static KF_DEV void pack(const R (&v)[2], const R (&m)[2][2], WSt<G, R>& st) {
    st_zero_row(st);
    st.v = v[0];
    st.m[0] = v[1];
    st.m[1] = m[0][0];
    st.m[2] = m[0][1];
    st.m[3] = m[1][0];
    st.m[4] = m[1][1];
  }
  KF_DEV void apply(WSt<G, R>& st, const E& e) const {
    R v[2], m[2][2];
    unpack(st, v, m);
    aff_mv(e.A, v, e.b, v);
    aff_mm(e.A, m, e.C, m);
    pack(v, m, st);
  }
  KF_DEV void initial(WSt<G, R>& st) const { st_zero_row(st); }
  KF_DEV void anchor(const E& e, WSt<G, R>& st) const { pack(e.b, e.C, st); }
  KF_DEV void expand(const WSt<G, R>& st, E& e) const {
    set_identity(e);
    e.A[0][0] = e.A[1][1] = R(0);
    unpack(st, e.b, e.C);
  }
  KF_DEV void steps(WSt<G, R>& st) const {
#pragma unroll 1
    for (int j = 0; j < L; ++j) {
      const long k = REV ? k0 + L - 1 - j : k0 + j;
      if (k >= T) continue;
      apply(st, load(k));
      if (r == 0) {
        R v[2], m[2][2];
        unpack(st, v, m);
        out[k * 6 + 0] = v[0];
        out[k * 6 + 1] = v[1];
        out[k * 6 + 2] = m[0][0];
        out[k * 6 + 3] = m[0][1];
        out[k * 6 + 4] = m[1][0];
        out[k * 6 + 5] = m[1][1];
      }
    }
  }
};

template <class R, int G, int BLOCK, int L, bool REV>
__global__ __launch_bounds__(BLOCK) void k_selftest_gscan(ScanArgs<R> a, const R* __restrict__ in,
                                                          R* __restrict__ out) {
  AffGroupPipe<R, G, BLOCK, L, REV> pp(a, in, out);
  gscan_tile<AffGroupPipe<R, G, BLOCK, L, REV>, G, R, R, BLOCK, L>(pp, a);
}

// Workspace of one scan slot: counters, status words, tagged aggregates and
// tagged anchored states, all zeroed before the scan.  The counters of a
// second slot are kept (zero), so that kf_workspace_status reads this
// workspace as it reads the others.
struct SelftestLayout {
  size_t flags, agg, pre, words, total;
  long ntiles;
};

// Steps per tile: 256 threads x items for the thread driver, and
// (wide_block(G) / G) groups x items for the group driver (G = 8 or 16).
static long selftest_tile(int group, int items) {
  return group == 1 ? (long)kBlock * items : (long)(wide_block(group) / group) * items;
}

static SelftestLayout selftest_layout(int precision, int group, int items, long T, long nseq) {
  SelftestLayout L{};
  const size_t halves = precision == KF_PREC_F64 ? 2 : 1;
  const long tile = selftest_tile(group, items);
  L.ntiles = (T + tile - 1) / tile;
  const long grid = L.ntiles * nseq;
  // a tile publishes one element (10 values) and one state (6) per thread
  // driver; one row per lane of a group in the group driver
  const size_t ew = group == 1 ? 10 : (size_t)group * 10;
  const size_t pw = group == 1 ? 6 : (size_t)group * (group + 1);
  size_t off = kEpochOffset + 128;  // the counters of two slots, then their epochs
  L.flags = off;
  off += (size_t)grid * sizeof(int);
  off = (off + 7) & ~size_t(7);
  L.agg = off;
  off += (size_t)grid * ew * halves * 8;
  L.pre = off;
  off += (size_t)grid * pw * halves * 8;
  L.words = off / 4;
  L.total = align256(off);
  return L;
}

static kf_status selftest_check(int precision, int group, int reverse, int items, long T,
                                long nseq) {
  if (precision != KF_PREC_F64 && precision != KF_PREC_F32) return KF_ERR_INVALID_ARG;
  if (group != 1 && group != 8 && group != 16) return KF_ERR_INVALID_ARG;
  if (reverse != 0 && reverse != 1) return KF_ERR_INVALID_ARG;
  if (items != 2 && items != 4 && items != 8 && items != 16) return KF_ERR_INVALID_ARG;
  if (T < 1 || nseq < 1 || T > (1L << 36) || nseq > (1L << 20)) return KF_ERR_INVALID_ARG;
  const long tile = selftest_tile(group, items);
  if ((T + tile - 1) / tile * nseq > 2147483647L) return KF_ERR_INVALID_ARG;
  return KF_OK;
}

template <class R>
static kf_status selftest_run(int group, int reverse, int items, long T, long nseq,
                              const void* elems, void* states, char* ws, const SelftestLayout& L,
                              hipStream_t st) {
  constexpr int B = kBlock;
  hipLaunchKernelGGL((k_clear<256>), dim3((unsigned)((L.words + 255) / 256 < 1024
                                                         ? (L.words + 255) / 256 : 1024)),
                     dim3(256), 0, st, reinterpret_cast<unsigned*>(ws), L.words);
  ScanArgs<R> a{};
  a.flags = reinterpret_cast<int*>(ws + L.flags);
  a.agg = reinterpret_cast<u64*>(ws + L.agg);
  a.pre = reinterpret_cast<u64*>(ws + L.pre);
  a.ctr = reinterpret_cast<unsigned*>(ws);
  a.epoch = reinterpret_cast<unsigned*>(ws + kEpochOffset);
  a.T = T;
  a.ntiles = L.ntiles;
  a.nseq = nseq;
  const dim3 grid((unsigned)(L.ntiles * nseq));
  const R* in = static_cast<const R*>(elems);
  R* out = static_cast<R*>(states);
  with_items<16>(items, [&](auto c) {
    constexpr int IL = decltype(c)::value;
    constexpr int B8 = wide_block(8), B16 = wide_block(16);
    if (group == 8) {
      if (reverse)
        hipLaunchKernelGGL((k_selftest_gscan<R, 8, B8, IL, true>), grid, dim3(B8), 0, st, a, in,
                           out);
      else
        hipLaunchKernelGGL((k_selftest_gscan<R, 8, B8, IL, false>), grid, dim3(B8), 0, st, a, in,
                           out);
    } else if (group == 16) {
      if (reverse)
        hipLaunchKernelGGL((k_selftest_gscan<R, 16, B16, IL, true>), grid, dim3(B16), 0, st, a,
                           in, out);
      else
        hipLaunchKernelGGL((k_selftest_gscan<R, 16, B16, IL, false>), grid, dim3(B16), 0, st, a,
                           in, out);
    } else if (reverse) {
      hipLaunchKernelGGL((k_selftest_scan<R, B, IL, true>), grid, dim3(B), 0, st, a, in, out);
    } else {
      hipLaunchKernelGGL((k_selftest_scan<R, B, IL, false>), grid, dim3(B), 0, st, a, in, out);
    }
  });
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

}  // namespace kfs

extern "C" {

kf_status kf_selftest_scan_workspace(int32_t precision, int32_t group, int32_t items, int64_t T,
                                     int64_t nseq, size_t* bytes) {
  if (!bytes) return KF_ERR_INVALID_ARG;
  const kf_status s = kfs::selftest_check(precision, group, 0, items, T, nseq);
  if (s != KF_OK) return s;
  *bytes = kfs::selftest_layout(precision, group, items, T, nseq).total;
  return KF_OK;
}

kf_status kf_selftest_scan(int32_t precision, int32_t group, int32_t reverse, int32_t items,
                           int64_t T, int64_t nseq, const void* elems, void* states,
                           void* workspace, size_t workspace_bytes, void* stream) {
  const kf_status s = kfs::selftest_check(precision, group, reverse, items, T, nseq);
  if (s != KF_OK) return s;
  if (!elems || !states) return KF_ERR_INVALID_ARG;
  const kfs::SelftestLayout L = kfs::selftest_layout(precision, group, items, T, nseq);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0 ||
      workspace_bytes < L.total)
    return KF_ERR_WORKSPACE;
  char* ws = static_cast<char*>(workspace);
  hipStream_t st = static_cast<hipStream_t>(stream);
  return precision == KF_PREC_F64
             ? kfs::selftest_run<double>(group, reverse, items, T, nseq, elems, states, ws, L, st)
             : kfs::selftest_run<float>(group, reverse, items, T, nseq, elems, states, ws, L, st);
}

}  // extern "C"

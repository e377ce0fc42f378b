// kf_inst.hpp -- kernel launches for one (N, M, precision); included by the
// per-precision translation units, which list the shapes that are built.
#pragma once
#include "kf_kernels.hpp"
#include "kf_wide.hpp"
#include "kf_seq.hpp"
#include "kf_tree.hpp"
#include "kf_plan.hpp"

#include <type_traits>

namespace kfs {

template <class T> struct TypeTag {
  using type = T;
};

// Calls fn(std::integral_constant<int, L>{}) for the runtime L in {2, 4, 8,
// 16}, instantiating only the values up to LMAX.
template <int LMAX, class Fn> void with_items(int L, Fn&& fn) {
  if constexpr (LMAX >= 16) {
    if (L == 16) return fn(std::integral_constant<int, 16>{});
  }
  if constexpr (LMAX >= 8) {
    if (L == 8) return fn(std::integral_constant<int, 8>{});
  }
  if constexpr (LMAX >= 4) {
    if (L == 4) return fn(std::integral_constant<int, 4>{});
  }
  fn(std::integral_constant<int, 2>{});
}

// KF_SCAN_SEQUENTIAL: one lane per sequence, 64-lane blocks.  The prepare
// stage only clears the error words.
template <int N, int M, class P>
kf_status run_sequential(Op op, int stages, const Job& p, char* ws, const Layout& L,
                         hipStream_t st) {
  using R = typename P::R;
  constexpr int B = 64;
  if (stages & ST_PREPARE)
    hipLaunchKernelGGL((k_clear<256>), dim3(1), dim3(256), 0, st, reinterpret_cast<unsigned*>(ws),
                       L.ctrl_words);
  SeqArgs<R> a{};
  a.F = static_cast<const R*>(p.F);
  a.Q = static_cast<const R*>(p.Q);
  a.H = static_cast<const R*>(p.H);
  a.Rm = static_cast<const R*>(p.R);
  a.u = p.tv ? static_cast<const R*>(p.u) : nullptr;
  a.d = p.tv ? static_cast<const R*>(p.d) : nullptr;
  a.m0 = static_cast<const R*>(p.m0);
  a.P0 = static_cast<const R*>(p.P0);
  a.T = p.T;
  a.nseq = p.nseq;
  if (p.batch) {
    a.len = p.len;
    a.row = p.row;
    a.total_steps = p.total_steps;
    a.model_stride = p.nmodels > 1 ? 1 : 0;
  }
  const dim3 grid((unsigned)((p.nseq + B - 1) / B));
  const R* y = static_cast<const R*>(p.y);
  R* mf = static_cast<R*>(p.m_filt);
  R* Pf = static_cast<R*>(p.P_filt);
  R* ms = static_cast<R*>(p.m_smooth);
  R* Ps = static_cast<R*>(p.P_smooth);
  if (stages & ST_FORWARD) {
    a.err = reinterpret_cast<unsigned*>(ws + L.ctr[0]) + 2;
    if (p.tv)
      hipLaunchKernelGGL((k_seq_filter<N, M, P, true>), grid, dim3(B), 0, st, a, y, mf, Pf);
    else
      hipLaunchKernelGGL((k_seq_filter<N, M, P, false>), grid, dim3(B), 0, st, a, y, mf, Pf);
  }
  if (op != OP_FILTER && (stages & ST_BACKWARD)) {
    a.err = reinterpret_cast<unsigned*>(ws + L.ctr[1]) + 2;
    if (op == OP_RTS && p.tv)
      hipLaunchKernelGGL((k_seq_rts<N, M, P, true>), grid, dim3(B), 0, st, a, (const R*)mf,
                         (const R*)Pf, ms, Ps);
    else if (op == OP_RTS)
      hipLaunchKernelGGL((k_seq_rts<N, M, P, false>), grid, dim3(B), 0, st, a, (const R*)mf,
                         (const R*)Pf, ms, Ps);
    else if (p.tv)
      hipLaunchKernelGGL((k_seq_twofilter<N, M, P, true>), grid, dim3(B), 0, st, a, y,
                         (const R*)mf, (const R*)Pf, ms, Ps);
    else
      hipLaunchKernelGGL((k_seq_twofilter<N, M, P, false>), grid, dim3(B), 0, st, a, y,
                         (const R*)mf, (const R*)Pf, ms, Ps);
  }
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

template <int N, int M, class P>
kf_status run_shape(Op op, int stages, const Job& p, char* ws, const Layout& L,
                    hipStream_t st) {
  using R = typename P::R;
  if (p.scan == KF_SCAN_SEQUENTIAL) return run_sequential<N, M, P>(op, stages, p, ws, L, st);
  constexpr int B = kBlock;
  constexpr int IT = items_per_thread(N);
  constexpr int ITI = items_ti(N);
  R* cst = reinterpret_cast<R*>(ws + L.cst);
  size_t prep_blocks = (L.ctrl_words + 255) / 256;
  if (prep_blocks > 1024) prep_blocks = 1024;
  if ((long)prep_blocks < p.nmodels) prep_blocks = (size_t)p.nmodels;
  const bool generic = (p.scan == KF_SCAN_LOOKBACK_GENERIC);
  const long cst_stride = (p.batch && p.nmodels > 1) ? L.cst_stride : 0;
  // the aggregate tables are built for the forward scan's L (unused by the
  // generic scan, whose L only sizes them)
  TvModel<R> tvm{};
  if (p.tv) {
    tvm = TvModel<R>{static_cast<const R*>(p.F), static_cast<const R*>(p.Q),
                     static_cast<const R*>(p.H), static_cast<const R*>(p.R),
                     static_cast<const R*>(p.u), static_cast<const R*>(p.d),
                     static_cast<const R*>(p.m0), static_cast<const R*>(p.P0)};
    if (stages & ST_PREPARE)
      hipLaunchKernelGGL((k_clear<256>), dim3((unsigned)prep_blocks), dim3(256), 0, st,
                         reinterpret_cast<unsigned*>(ws), L.ctrl_words);
  } else if (stages & ST_PREPARE) {
    with_items<ITI>(L.items[0], [&](auto cf) {
      with_items<IT>(L.items[1], [&](auto cb) {
        hipLaunchKernelGGL((k_prepare<N, M, R, decltype(cf)::value, decltype(cb)::value>),
                           dim3((unsigned)prep_blocks), dim3(256), 0, st,
                           static_cast<const R*>(p.F), static_cast<const R*>(p.Q),
                           static_cast<const R*>(p.H), static_cast<const R*>(p.R),
                           static_cast<const R*>(p.m0), static_cast<const R*>(p.P0), cst,
                           reinterpret_cast<unsigned*>(ws), L.ctrl_words, p.nmodels,
                           L.cst_stride);
      });
    });
    if (p.batch)
      hipLaunchKernelGGL((k_batch_tiles<1024>), dim3(1), dim3(1024), 0, st, p.len, p.row, p.nseq,
                         p.total_steps, L.tile[0], L.tile[1],
                         reinterpret_cast<int64_t*>(ws + L.tile_start[0]),
                         reinterpret_cast<int64_t*>(ws + L.tile_start[1]),
                         reinterpret_cast<int*>(ws + L.tile_map[0]),
                         reinterpret_cast<int*>(ws + L.tile_map[1]), L.grid[0], L.grid[1],
                         reinterpret_cast<unsigned*>(ws + L.ctr[0]) + 2,
                         reinterpret_cast<unsigned*>(ws + L.ctr[1]) + 2);
  }
  const R* y = static_cast<const R*>(p.y);
  R* mf = static_cast<R*>(p.m_filt);
  R* Pf = static_cast<R*>(p.P_filt);
  R* ms = static_cast<R*>(p.m_smooth);
  R* Ps = static_cast<R*>(p.P_smooth);
  if (is_tree_scan(p.scan)) {
    R* X0 = reinterpret_cast<R*>(ws + L.tree[0]);
    R* X1 = reinterpret_cast<R*>(ws + L.tree[1]);
    TreeIO<R> io{cst, y, mf, Pf, mf, Pf, p.T, L.tree_positions, tvm};
    auto scan = [&](auto tag) {
      tree_scan<typename decltype(tag)::type>(io, p.scan, p.nseq, X0, X1, st);
    };
    if (stages & ST_FORWARD) {
      if (p.tv) scan(TypeTag<TreeFilter<N, M, P, true>>{});
      else scan(TypeTag<TreeFilter<N, M, P>>{});
    }
    if (op != OP_FILTER && (stages & ST_BACKWARD)) {
      io.m_out = ms;
      io.P_out = Ps;
      if (op == OP_RTS) {
        if (p.tv) scan(TypeTag<TreeRts<N, M, P, true>>{});
        else scan(TypeTag<TreeRts<N, M, P>>{});
      } else {
        if (p.tv) scan(TypeTag<TreeTwoFilter<N, M, P, true>>{});
        else scan(TypeTag<TreeTwoFilter<N, M, P>>{});
      }
    }
    return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
  }
  auto args = [&](int slot) {
    ScanArgs<R> a{};
    a.flags = reinterpret_cast<int*>(ws + L.flags[slot]);
    a.agg = reinterpret_cast<u64*>(ws + L.agg[slot]);
    a.pre = reinterpret_cast<u64*>(ws + L.pre[slot]);
    a.ctr = reinterpret_cast<unsigned*>(ws + L.ctr[slot]);
    a.epoch = reinterpret_cast<unsigned*>(ws + L.epoch[slot]);
    a.T = p.T;
    a.ntiles = L.ntiles[slot];
    a.nseq = p.nseq;
    if (p.batch) {
      a.tile_seq = reinterpret_cast<const int*>(ws + L.tile_map[slot]);
      a.tile_start = reinterpret_cast<const int64_t*>(ws + L.tile_start[slot]);
      a.seq_len = p.len;
      a.seq_row = p.row;
      a.cst_stride = cst_stride;
    }
    return a;
  };
  auto grid = [&](int slot) { return dim3((unsigned)L.grid[slot]); };
  if (stages & ST_FORWARD) {
    ScanArgs<R> fa = args(0);
    if (p.tv)
      with_items<IT>(L.items[0], [&](auto c) {
        hipLaunchKernelGGL((k_filter<N, M, P, B, decltype(c)::value, true>), grid(0), dim3(B), 0,
                           st, fa, tvm, cst, y, (const R*)nullptr, (const R*)nullptr, mf, Pf);
      });
    else if (generic)
      with_items<IT>(L.items[0], [&](auto c) {
        hipLaunchKernelGGL((k_filter<N, M, P, B, decltype(c)::value>), grid(0), dim3(B), 0, st,
                           fa, tvm, cst, y, (const R*)nullptr, (const R*)nullptr, mf, Pf);
      });
    else
      with_items<ITI>(L.items[0], [&](auto c) {
        hipLaunchKernelGGL((k_filter_ti<N, M, P, B, decltype(c)::value>), grid(0), dim3(B), 0,
                           st, fa, cst, y, (const R*)nullptr, (const R*)nullptr, mf, Pf);
      });
  }
  if (op != OP_FILTER && (stages & ST_BACKWARD)) {
    ScanArgs<R> ba = args(1);
    with_items<IT>(L.items[1], [&](auto c) {
      constexpr int IL = decltype(c)::value;
      if (op == OP_RTS && p.tv)
        hipLaunchKernelGGL((k_rts<N, M, P, B, IL, true>), grid(1), dim3(B), 0, st, ba, tvm, cst, y,
                           (const R*)mf, (const R*)Pf, ms, Ps);
      else if (op == OP_RTS)
        hipLaunchKernelGGL((k_rts<N, M, P, B, IL>), grid(1), dim3(B), 0, st, ba, tvm, cst, y,
                           (const R*)mf, (const R*)Pf, ms, Ps);
      else if (p.tv)
        hipLaunchKernelGGL((k_twofilter<N, M, P, B, IL, false, true>), grid(1), dim3(B), 0, st, ba,
                           tvm, cst, y, (const R*)mf, (const R*)Pf, ms, Ps);
      else if (generic)
        hipLaunchKernelGGL((k_twofilter<N, M, P, B, IL, false>), grid(1), dim3(B), 0, st, ba, tvm,
                           cst, y, (const R*)mf, (const R*)Pf, ms, Ps);
      else
        hipLaunchKernelGGL((k_twofilter<N, M, P, B, IL, true>), grid(1), dim3(B), 0, st, ba, tvm,
                           cst, y, (const R*)mf, (const R*)Pf, ms, Ps);
    });
  }
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

// States wider than nx = 4 (kf_wide.hpp): the look-back scans over
// row-distributed elements, for equal-length sequences and ragged batches.
template <int N, int M, class P>
kf_status run_wide(Op op, int stages, const Job& p, char* ws, const Layout& L, hipStream_t st) {
  using R = typename P::R;
  constexpr int B = wide_block(N);
  constexpr int IL = wide_items(N);
  R* cst = reinterpret_cast<R*>(ws + L.cst);
  size_t prep_blocks = (L.ctrl_words + 255) / 256;
  if (prep_blocks > 1024) prep_blocks = 1024;
  if ((long)prep_blocks < p.nmodels) prep_blocks = (size_t)p.nmodels;
  const long cst_stride = (p.batch && p.nmodels > 1) ? L.cst_stride : 0;
  if (stages & ST_PREPARE) {
    hipLaunchKernelGGL((k_wprepare<N, M, R>), dim3((unsigned)prep_blocks), dim3(256), 0, st,
                       static_cast<const R*>(p.F), static_cast<const R*>(p.Q),
                       static_cast<const R*>(p.H), static_cast<const R*>(p.R),
                       static_cast<const R*>(p.m0), static_cast<const R*>(p.P0), cst,
                       reinterpret_cast<unsigned*>(ws), L.ctrl_words, p.nmodels, L.cst_stride);
    if (p.batch)
      hipLaunchKernelGGL((k_batch_tiles<1024>), dim3(1), dim3(1024), 0, st, p.len, p.row, p.nseq,
                         p.total_steps, L.tile[0], L.tile[1],
                         reinterpret_cast<int64_t*>(ws + L.tile_start[0]),
                         reinterpret_cast<int64_t*>(ws + L.tile_start[1]),
                         reinterpret_cast<int*>(ws + L.tile_map[0]),
                         reinterpret_cast<int*>(ws + L.tile_map[1]), L.grid[0], L.grid[1],
                         reinterpret_cast<unsigned*>(ws + L.ctr[0]) + 2,
                         reinterpret_cast<unsigned*>(ws + L.ctr[1]) + 2);
  }
  const R* y = static_cast<const R*>(p.y);
  R* mf = static_cast<R*>(p.m_filt);
  R* Pf = static_cast<R*>(p.P_filt);
  R* ms = static_cast<R*>(p.m_smooth);
  R* Ps = static_cast<R*>(p.P_smooth);
  auto args = [&](int slot) {
    ScanArgs<R> a{};
    a.flags = reinterpret_cast<int*>(ws + L.flags[slot]);
    a.agg = reinterpret_cast<u64*>(ws + L.agg[slot]);
    a.pre = reinterpret_cast<u64*>(ws + L.pre[slot]);
    a.ctr = reinterpret_cast<unsigned*>(ws + L.ctr[slot]);
    a.epoch = reinterpret_cast<unsigned*>(ws + L.epoch[slot]);
    a.T = p.T;
    a.ntiles = L.ntiles[slot];
    a.nseq = p.nseq;
    if (p.batch) {
      a.tile_seq = reinterpret_cast<const int*>(ws + L.tile_map[slot]);
      a.tile_start = reinterpret_cast<const int64_t*>(ws + L.tile_start[slot]);
      a.seq_len = p.len;
      a.seq_row = p.row;
      a.cst_stride = cst_stride;
    }
    return a;
  };
  if (stages & ST_FORWARD)
    hipLaunchKernelGGL((k_wfilter<N, M, P, B, IL>), dim3((unsigned)L.grid[0]), dim3(B), 0, st,
                       args(0), cst, y, (const R*)nullptr, (const R*)nullptr, mf, Pf);
  if (op != OP_FILTER && (stages & ST_BACKWARD)) {
    if (op == OP_RTS)
      hipLaunchKernelGGL((k_wrts<N, M, P, B, IL>), dim3((unsigned)L.grid[1]), dim3(B), 0, st,
                         args(1), cst, y, (const R*)mf, (const R*)Pf, ms, Ps);
    else
      hipLaunchKernelGGL((k_wtwofilter<N, M, P, B, IL>), dim3((unsigned)L.grid[1]), dim3(B), 0,
                         st, args(1), cst, y, (const R*)mf, (const R*)Pf, ms, Ps);
  }
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

// Wide shapes compiled into the library (each in a translation unit of its
// own, kf_wide_<precision>_<nx>.hip).
#define KFS_WIDE_SHAPES(X) \
  X(8, 4)                  \
  X(16, 8)

#define KFS_WIDE_EXTERN(n, m)                                                              \
  extern template kf_status run_wide<n, m, PrecF64>(Op, int, const Job&, char*,           \
                                                    const Layout&, hipStream_t);          \
  extern template kf_status run_wide<n, m, PrecF32>(Op, int, const Job&, char*,           \
                                                    const Layout&, hipStream_t);          \
  extern template kf_status run_wide<n, m, PrecMixed>(Op, int, const Job&, char*,         \
                                                      const Layout&, hipStream_t);
KFS_WIDE_SHAPES(KFS_WIDE_EXTERN)
#undef KFS_WIDE_EXTERN

#define KFS_WIDE_INSTANTIATE(n, m, P)                                                      \
  template kf_status run_wide<n, m, P>(Op, int, const Job&, char*, const Layout&, hipStream_t);

// Shapes compiled into the library.
#define KFS_SHAPES(X) \
  X(1, 1)             \
  X(2, 1)             \
  X(2, 2)             \
  X(3, 1)             \
  X(3, 2)             \
  X(4, 1)             \
  X(4, 2)             \
  X(4, 4)

// Each shape's launches are instantiated in a translation unit of their own
// (kf_inst_<precision>_<group>.hip), so the library compiles in parallel.
#define KFS_EXTERN(n, m)                                                                   \
  extern template kf_status run_shape<n, m, PrecF64>(Op, int, const Job&, char*,    \
                                                     const Layout&, hipStream_t);          \
  extern template kf_status run_shape<n, m, PrecF32>(Op, int, const Job&, char*,    \
                                                     const Layout&, hipStream_t);          \
  extern template kf_status run_shape<n, m, PrecMixed>(Op, int, const Job&, char*,  \
                                                       const Layout&, hipStream_t);
KFS_SHAPES(KFS_EXTERN)
#undef KFS_EXTERN

#define KFS_INSTANTIATE(n, m, P)                                                           \
  template kf_status run_shape<n, m, P>(Op, int, const Job&, char*, const Layout&,  \
                                        hipStream_t);

template <class P>
kf_status run_prec(Op op, int stages, const Job& p, char* ws, const Layout& L,
                   hipStream_t st) {
#define KFS_CASE(n, m) \
  if (p.nx == n && p.ny == m) return run_shape<n, m, P>(op, stages, p, ws, L, st);
  KFS_SHAPES(KFS_CASE)
#undef KFS_CASE
#define KFS_WCASE(n, m) \
  if (p.nx == n && p.ny == m) return run_wide<n, m, P>(op, stages, p, ws, L, st);
  KFS_WIDE_SHAPES(KFS_WCASE)
#undef KFS_WCASE
  return KF_ERR_UNSUPPORTED;
}

}  // namespace kfs

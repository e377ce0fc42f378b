// kf_kernels.hpp -- single-pass look-back scan kernels for the parallel
// Kalman filter (Algorithm 5), the RTS smoother's reverse scan (Algorithm 6)
// and the two-filter smoother's backward scan fused with the combination
// (Algorithm 7), plus the per-model preparation kernel.
//
// Tiling: one workgroup of BLOCK threads per tile of BLOCK*L time steps; a
// thread owns L consecutive steps.  Per tile:
//   1. load inputs, build the elements, fold each thread's L elements (serial);
//   2. scan the thread aggregates across the workgroup (wavefront Hillis-Steele
//      over lanes, then the per-wave totals through LDS);
//   3. publish the tile aggregate, look back over earlier tiles (windowed,
//      one wavefront), publish the tile's anchored inclusive prefix;
//   4. each thread applies its exclusive prefix to its own steps in order and
//      writes the outputs.
// Tiles are taken in scan order from an atomic counter, so every tile a block
// waits on belongs to a block that is already running.  The status words and
// counters are zeroed by the preparation kernel that precedes the scans.
#pragma once
#include "kf_scan.hpp"

namespace kfs {

// Derived model quantities, FP64-computed once per call (eqs. pkf_init1..3):
//   generic element (k >= 2): S = H Q H^T + R, K = Q H^T S^{-1},
//     A = (I - K H) F, C = (I - K H) Q, W = F^T H^T S^{-1}, J = W H F,
//     b_k = K y_k, eta_k = W y_k;
//   first element (k = 1): x = F m0, P = F P0 F^T + Q, S1 = H P H^T + R,
//     K1 = P H^T S1^{-1}, A_1 = 0, b_1 = c1 + K1 y_1 with c1 = x - K1 H x,
//     C_1 = P - K1 S1 K1^T, eta_1 = W y_1, J_1 = J (reading C4).
// F and Q are copied for the smoothing elements.  Layout (type R):
template <int N, int M> struct CL {
  static constexpr int A = 0, C = A + N * N, J = C + N * N, K = J + N * N, W = K + N * M,
                       K1 = W + N * M, c1 = K1 + N * M, C1 = c1 + N, F = C1 + N * N,
                       Q = F + N * N, SIZE = Q + N * N;
};

// The same launch zeroes the workspace's control words (tile tickets,
// timeout flags, look-back status words) with a grid-stride loop.
template <int N, int M, class R>
__global__ __launch_bounds__(256) void k_prepare(const R* __restrict__ F_, const R* __restrict__ Q_,
                                                 const R* __restrict__ H_, const R* __restrict__ R_,
                                                 const R* __restrict__ m0_,
                                                 const R* __restrict__ P0_, R* __restrict__ cst,
                                                 unsigned* __restrict__ ctrl, size_t ctrl_words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ctrl_words;
       i += (size_t)gridDim.x * blockDim.x)
    ctrl[i] = 0u;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  using D = double;
  using L = CL<N, M>;
  D F[N][N], Q[N][N], H[M][N], Rm[M][M], m0[N], P0[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    m0[i] = D(m0_[i]);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      F[i][j] = D(F_[i * N + j]);
      Q[i][j] = D(Q_[i * N + j]);
      P0[i][j] = D(P0_[i * N + j]);
    }
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) H[i][j] = D(H_[i * N + j]);
#pragma unroll
    for (int j = 0; j < M; ++j) Rm[i][j] = D(R_[i * M + j]);
  }
  // generic element
  D HQ[M][N], S[M][M], sd[M];
  mm<M, N, N, D>(H, Q, HQ);
  sym_xyt_plus<M, N, D>(HQ, H, Rm, S);
  chol_factor<M, D>(S, sd);
  D Kt[M][N];  // K^T = S^{-1} H Q
  copy_mat<M, N, D>(HQ, Kt);
  chol_solve<M, N, D>(S, sd, Kt);
  D IKH[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      D s = (i == j) ? D(1) : D(0);
#pragma unroll
      for (int t = 0; t < M; ++t) s -= Kt[t][i] * H[t][j];
      IKH[i][j] = s;
    }
  D A[N][N], C[N][N];
  mm<N, N, N, D>(IKH, F, A);
  mm<N, N, N, D>(IKH, Q, C);
  D HF[M][N], Wt[M][N];  // W^T = S^{-1} H F
  mm<M, N, N, D>(H, F, HF);
  copy_mat<M, N, D>(HF, Wt);
  chol_solve<M, N, D>(S, sd, Wt);
  D Jm[N][N];
  D Z[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Z[i][j] = D(0);
  sym_xty_plus<N, M, D>(Wt, HF, Z, Jm);  // J = (S^{-1} H F)^T (H F)
  // first element
  D x[N], FP[N][N], P[N][N];
  mv<N, N, D>(F, m0, x);
  mm<N, N, N, D>(F, P0, FP);
  sym_xyt_plus<N, N, D>(FP, F, Q, P);
  D HP[M][N], S1[M][M], s1d[M];
  mm<M, N, N, D>(H, P, HP);
  sym_xyt_plus<M, N, D>(HP, H, Rm, S1);
  chol_factor<M, D>(S1, s1d);
  D K1t[M][N];
  copy_mat<M, N, D>(HP, K1t);
  chol_solve<M, N, D>(S1, s1d, K1t);
  D Hx[M], c1[N], C1[N][N];
  mv<M, N, D>(H, x, Hx);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    D s = x[i];
#pragma unroll
    for (int t = 0; t < M; ++t) s -= K1t[t][i] * Hx[t];
    c1[i] = s;
  }
  // C_1 = P - K1 S1 K1^T = P - (H P)^T S1^{-1} (H P)
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      D s = P[i][j];
#pragma unroll
      for (int t = 0; t < M; ++t) s -= HP[t][i] * K1t[t][j];
      C1[i][j] = s;
      C1[j][i] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cst[L::c1 + i] = R(c1[i]);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cst[L::A + i * N + j] = R(A[i][j]);
      cst[L::C + i * N + j] = R(0.5 * (C[i][j] + C[j][i]));
      cst[L::J + i * N + j] = R(Jm[i][j]);
      cst[L::C1 + i * N + j] = R(C1[i][j]);
      cst[L::F + i * N + j] = R(F[i][j]);
      cst[L::Q + i * N + j] = R(0.5 * (Q[i][j] + Q[j][i]));
    }
#pragma unroll
    for (int t = 0; t < M; ++t) {
      cst[L::K + i * M + t] = R(Kt[t][i]);
      cst[L::W + i * M + t] = R(Wt[t][i]);
      cst[L::K1 + i * M + t] = R(K1t[t][i]);
    }
  }
}

// Kernel arguments shared by the three scans.
template <class R> struct ScanArgs {
  const R* cst;   // CL layout
  const R* y;     // [nseq][T][M]
  const R* m_in;  // filter means     (RTS, two-filter)
  const R* P_in;  // filter covariances
  R* m_out;
  R* P_out;
  int* flags;      // [nseq * ntiles]
  R* agg;          // [nseq * ntiles][elem size]
  R* pre;          // [nseq * ntiles][anchored prefix size]
  unsigned* ctr;   // [0] tile ticket, [1] finished blocks, [2] look-back timeout flag
  long T;
  long ntiles;     // tiles per sequence
  long nseq;
};

// Element of step k (0-based row k, i.e. time step k+1) from its measurement.
template <int N, int M, class R>
KF_DEV FElem<N, R> filter_element(const R* __restrict__ cst, long k, const R (&y)[M]) {
  using L = CL<N, M>;
  FElem<N, R> a;
  const bool first = (k == 0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R b = first ? cst[L::c1 + i] : R(0);
    R e = R(0);
#pragma unroll
    for (int t = 0; t < M; ++t) {
      b += (first ? cst[L::K1 + i * M + t] : cst[L::K + i * M + t]) * y[t];
      e += cst[L::W + i * M + t] * y[t];
    }
    a.b[i] = b;
    a.e[i] = e;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      a.A[i][j] = first ? R(0) : cst[L::A + i * N + j];
      a.C[i][j] = first ? cst[L::C1 + i * N + j] : cst[L::C + i * N + j];
      a.J[i][j] = cst[L::J + i * N + j];
    }
  }
  return a;
}

template <int N, class R> struct State {
  R x[N];
  R P[N][N];
};

// After the last block of a scan has finished, clear that scan's status
// words and tile ticket, so the pass can be enqueued again without another
// preparation launch.  The timeout flag (ctr[2]) is left for diagnosis.
template <int BLOCK>
KF_DEV void finish_grid(int* __restrict__ flags, unsigned* __restrict__ ctr, long nflags,
                        int* s_last) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(ctr + 1, 1u);
    *s_last = (done == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (*s_last) {
    __threadfence();
    for (long i = threadIdx.x; i < nflags; i += BLOCK) flags[i] = LB_EMPTY;
    if (threadIdx.x == 0) {
      ctr[0] = 0u;
      ctr[1] = 0u;
    }
  }
}

// ===========================================================================
// Forward filter (Algorithm 5)
// ===========================================================================
template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_filter(ScanArgs<typename P::R> a) {
  using R = typename P::R;
  using E = FElem<N, R>;
  constexpr int NW = BLOCK / WAVE;
  constexpr int TILE = BLOCK * L;
  constexpr int PS = N + N * N;  // anchored prefix payload: (b, C)
  __shared__ E s_wt[NW];
  __shared__ R s_pre[PS];
  __shared__ long s_tile;
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  if (tid == 0) s_tile = (long)atomicAdd(a.ctr, 1u);
  __syncthreads();
  const long gt = s_tile;
  const long seq = gt / a.ntiles, t = gt - seq * a.ntiles;
  const long k0 = t * TILE + (long)tid * L;
  const R* __restrict__ y = a.y + seq * a.T * M;
  const R* __restrict__ cst = a.cst;
  auto op = [](const E& p, const E& q) { return fcombine<N, P>(p, q); };

  // 1. thread fold
  R yv[L][M];
#pragma unroll
  for (int i = 0; i < L; ++i)
#pragma unroll
    for (int c = 0; c < M; ++c) yv[i][c] = (k0 + i < a.T) ? y[(k0 + i) * M + c] : R(0);
  E agg;
  if (k0 < a.T) {
    agg = filter_element<N, M, R>(cst, k0, yv[0]);
  } else {
    set_identity(agg);
  }
#pragma unroll
  for (int i = 1; i < L; ++i) {
    if (k0 + i < a.T) agg = op(agg, filter_element<N, M, R>(cst, k0 + i, yv[i]));
  }

  // 2. workgroup scan
  E x = agg;
  wave_inclusive_scan(x, lane, op);
  if (lane == WAVE - 1) s_wt[wid] = x;
  E lex = shfl_up(x, 1);
  __syncthreads();
  E tex;  // exclusive prefix of this thread within the tile (valid if tid > 0)
  if (wid > 0) {
    E wex = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < wid; ++w) wex = op(wex, s_wt[w]);
    tex = (lane > 0) ? op(wex, lex) : wex;
  } else {
    tex = lex;
  }

  // 3. publish + look-back (wave 0)
  const long base = seq * a.ntiles;
  if (wid == 0) {
    E tot = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < NW; ++w) tot = op(tot, s_wt[w]);
    if (t == 0) {
      // tile 0 holds step 1 (A_1 = 0): its aggregate is the anchored prefix
      if (lane == 0) {
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = tot.b[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = tot.C[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    } else {
      if (lane == 0) {
        gstore(a.agg + (base + t) * E::SIZE, tot);
        lb_store_flag(a.flags + base + t, LB_AGG);
      }
      auto load_agg = [&](long idx, E& v) { gload(v, a.agg + (base + idx) * E::SIZE); };
      auto expand = [&](long idx, E& v) {
        const R* p = a.pre + (base + idx) * PS;
        set_identity(v);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          v.A[i][i] = R(0);
          v.b[i] = p[i];
#pragma unroll
          for (int j = 0; j < N; ++j) v.C[i][j] = p[N + i * N + j];
        }
      };
      E ex = lookback<E>(a.flags + base, a.ctr + 2, t, lane, op, load_agg, expand);
      if (lane == 0) {
        State<N, R> st;
        copy_vec<N, R>(ex.b, st.x);
        copy_mat<N, N, R>(ex.C, st.P);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          s_pre[i] = st.x[i];
#pragma unroll
          for (int j = 0; j < N; ++j) s_pre[N + i * N + j] = st.P[i][j];
        }
        fapply<N, P>(st.x, st.P, tot);
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = st.x[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = st.P[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    }
  }
  __syncthreads();

  // 4. apply prefixes and write x_{k|k}, P_{k|k}
  State<N, R> st;
  bool have;
  if (t > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      st.x[i] = s_pre[i];
#pragma unroll
      for (int j = 0; j < N; ++j) st.P[i][j] = s_pre[N + i * N + j];
    }
    if (tid > 0) fapply<N, P>(st.x, st.P, tex);
    have = true;
  } else {
    // tile 0: a thread's in-tile exclusive prefix contains step 1 (A = 0)
    copy_vec<N, R>(tex.b, st.x);
    copy_mat<N, N, R>(tex.C, st.P);
    have = tid > 0;
  }
  R* __restrict__ mo = a.m_out + seq * a.T * N;
  R* __restrict__ Po = a.P_out + seq * a.T * N * N;
#pragma unroll 1
  for (int i = 0; i < L; ++i) {
    const long k = k0 + i;
    if (k >= a.T) break;
    E el = filter_element<N, M, R>(cst, k, yv[i]);
    if (have) {
      fapply<N, P>(st.x, st.P, el);
    } else {
      copy_vec<N, R>(el.b, st.x);
      copy_mat<N, N, R>(el.C, st.P);
      have = true;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      mo[k * N + r] = st.x[r];
#pragma unroll
      for (int c = 0; c < N; ++c) Po[k * N * N + r * N + c] = st.P[r][c];
    }
  }
  finish_grid<BLOCK>(a.flags, a.ctr, a.nseq * a.ntiles, &s_last);
}

// ===========================================================================
// RTS smoother reverse scan (Algorithm 6).  Scan order is descending time:
// tile t (scan order) covers time tile ntiles-1-t, thread tid covers time
// chunk BLOCK-1-tid of it and walks its steps from last to first.
// ===========================================================================
template <int N, class R> KF_DEV void load_state(const R* __restrict__ m, const R* __restrict__ Pm,
                                                  long k, R (&x)[N], R (&P)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    x[i] = m[k * N + i];
#pragma unroll
    for (int j = 0; j < N; ++j) P[i][j] = Pm[k * N * N + i * N + j];
  }
}

template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_rts(ScanArgs<typename P::R> a) {
  using R = typename P::R;
  using E = SElem<N, R>;
  using LY = CL<N, M>;
  constexpr int NW = BLOCK / WAVE;
  constexpr int TILE = BLOCK * L;
  constexpr int PS = N + N * N;  // anchored suffix payload: (g, L)
  __shared__ E s_wt[NW];
  __shared__ R s_pre[PS];
  __shared__ long s_tile;
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  if (tid == 0) s_tile = (long)atomicAdd(a.ctr, 1u);
  __syncthreads();
  const long gt = s_tile;
  const long seq = gt / a.ntiles, t = gt - seq * a.ntiles;  // t: scan order
  const long tt = a.ntiles - 1 - t;                           // time tile
  const long k0 = tt * TILE + (long)(BLOCK - 1 - tid) * L;    // first step (time order)
  const R* __restrict__ mf = a.m_in + seq * a.T * N;
  const R* __restrict__ Pf = a.P_in + seq * a.T * N * N;
  R Fm[N][N], Qm[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      Fm[i][j] = a.cst[LY::F + i * N + j];
      Qm[i][j] = a.cst[LY::Q + i * N + j];
    }
  // scan-order operator: p precedes q in scan order, so p is later in time
  auto op = [](const E& p, const E& q) { return scombine<N, P>(q, p); };
  auto element = [&](long k) {
    R x[N], Pk[N][N];
    load_state<N, R>(mf, Pf, k, x, Pk);
    E e;
    if (k == a.T - 1) {  // eq. prts_init2
      set_identity(e);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        e.E[i][i] = R(0);
        e.g[i] = x[i];
#pragma unroll
        for (int j = 0; j < N; ++j) e.L[i][j] = Pk[i][j];
      }
    } else {
      e = smooth_element<N, P>(x, Pk, Fm, Qm);
    }
    return e;
  };

  // 1. thread fold over the chunk, last step first
  E agg;
  bool any = false;
#pragma unroll 1
  for (int i = L - 1; i >= 0; --i) {
    const long k = k0 + i;
    if (k >= a.T) continue;
    E el = element(k);
    agg = any ? scombine<N, P>(el, agg) : el;
    any = true;
  }
  if (!any) set_identity(agg);

  // 2. workgroup scan (scan order = thread order)
  E x = agg;
  wave_inclusive_scan(x, lane, op);
  if (lane == WAVE - 1) s_wt[wid] = x;
  E lex = shfl_up(x, 1);
  __syncthreads();
  E tex;
  if (wid > 0) {
    E wex = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < wid; ++w) wex = op(wex, s_wt[w]);
    tex = (lane > 0) ? op(wex, lex) : wex;
  } else {
    tex = lex;
  }

  // 3. publish + look-back
  const long base = seq * a.ntiles;
  if (wid == 0) {
    E tot = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < NW; ++w) tot = op(tot, s_wt[w]);
    if (t == 0) {
      // the time-last tile holds step T (E_T = 0): its aggregate is anchored
      if (lane == 0) {
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = tot.g[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = tot.L[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    } else {
      if (lane == 0) {
        gstore(a.agg + (base + t) * E::SIZE, tot);
        lb_store_flag(a.flags + base + t, LB_AGG);
      }
      auto load_agg = [&](long idx, E& v) { gload(v, a.agg + (base + idx) * E::SIZE); };
      auto expand = [&](long idx, E& v) {
        const R* p = a.pre + (base + idx) * PS;
        set_identity(v);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          v.E[i][i] = R(0);
          v.g[i] = p[i];
#pragma unroll
          for (int j = 0; j < N; ++j) v.L[i][j] = p[N + i * N + j];
        }
      };
      E ex = lookback<E>(a.flags + base, a.ctr + 2, t, lane, op, load_agg, expand);
      if (lane == 0) {
        State<N, R> st;
        copy_vec<N, R>(ex.g, st.x);
        copy_mat<N, N, R>(ex.L, st.P);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          s_pre[i] = st.x[i];
#pragma unroll
          for (int j = 0; j < N; ++j) s_pre[N + i * N + j] = st.P[i][j];
        }
        sapply<N, P>(tot, st.x, st.P);
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = st.x[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = st.P[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    }
  }
  __syncthreads();

  // 4. apply suffixes, last step first, and write x_{k|T}, P_{k|T}
  State<N, R> st;
  bool have;
  if (t > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      st.x[i] = s_pre[i];
#pragma unroll
      for (int j = 0; j < N; ++j) st.P[i][j] = s_pre[N + i * N + j];
    }
    if (tid > 0) sapply<N, P>(tex, st.x, st.P);
    have = true;
  } else {
    copy_vec<N, R>(tex.g, st.x);
    copy_mat<N, N, R>(tex.L, st.P);
    have = tid > 0;
  }
  R* __restrict__ mo = a.m_out + seq * a.T * N;
  R* __restrict__ Po = a.P_out + seq * a.T * N * N;
#pragma unroll 1
  for (int i = L - 1; i >= 0; --i) {
    const long k = k0 + i;
    if (k >= a.T) continue;
    if (have) {
      E el = element(k);
      sapply<N, P>(el, st.x, st.P);
    } else {
      load_state<N, R>(mf, Pf, k, st.x, st.P);  // step T: x_{T|T}, P_{T|T}
      have = true;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      mo[k * N + r] = st.x[r];
#pragma unroll
      for (int c = 0; c < N; ++c) Po[k * N * N + r * N + c] = st.P[r][c];
    }
  }
  finish_grid<BLOCK>(a.flags, a.ctr, a.nseq * a.ntiles, &s_last);
}

// ===========================================================================
// Two-filter smoother backward pass (Algorithm 7): reverse scan over
// (a_2, ..., a_T, e) with the filtering operator; position k (0-based row)
// holds a_{k+2} for k < T-1 and the identity e at k = T-1, so the suffix at
// row k is a_{k+2} (x) ... (x) a_T (x) e, whose (eta, J) is eta_{k+1|k+2:T},
// J_{k+1|k+2:T}.  The combination with the filter result (m_in, P_in) is
// fused into the apply phase.
// ===========================================================================
template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_twofilter(ScanArgs<typename P::R> a) {
  using R = typename P::R;
  using E = FElem<N, R>;
  constexpr int NW = BLOCK / WAVE;
  constexpr int TILE = BLOCK * L;
  constexpr int PS = N + N * N;  // anchored suffix payload: (eta, J)
  __shared__ E s_wt[NW];
  __shared__ R s_pre[PS];
  __shared__ long s_tile;
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  if (tid == 0) s_tile = (long)atomicAdd(a.ctr, 1u);
  __syncthreads();
  const long gt = s_tile;
  const long seq = gt / a.ntiles, t = gt - seq * a.ntiles;
  const long tt = a.ntiles - 1 - t;
  const long k0 = tt * TILE + (long)(BLOCK - 1 - tid) * L;
  const R* __restrict__ y = a.y + seq * a.T * M;
  const R* __restrict__ cst = a.cst;
  auto op = [](const E& p, const E& q) { return fcombine<N, P>(q, p); };
  // measurement of the element at row k: y_{k+2} (row k+1); none at k = T-1
  R yv[L][M];
#pragma unroll
  for (int i = 0; i < L; ++i)
#pragma unroll
    for (int c = 0; c < M; ++c) yv[i][c] = (k0 + i + 1 < a.T) ? y[(k0 + i + 1) * M + c] : R(0);
  auto element = [&](long k, const R (&yk)[M]) {
    E e;
    if (k == a.T - 1) set_identity(e);
    else e = filter_element<N, M, R>(cst, k + 1, yk);
    return e;
  };

  // 1. thread fold, last step first
  E agg;
  bool any = false;
#pragma unroll
  for (int i = L - 1; i >= 0; --i) {
    const long k = k0 + i;
    if (k >= a.T) continue;
    E el = element(k, yv[i]);
    agg = any ? fcombine<N, P>(el, agg) : el;
    any = true;
  }
  if (!any) set_identity(agg);

  // 2. workgroup scan
  E x = agg;
  wave_inclusive_scan(x, lane, op);
  if (lane == WAVE - 1) s_wt[wid] = x;
  E lex = shfl_up(x, 1);
  __syncthreads();
  E tex;
  if (wid > 0) {
    E wex = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < wid; ++w) wex = op(wex, s_wt[w]);
    tex = (lane > 0) ? op(wex, lex) : wex;
  } else {
    tex = lex;
  }

  // 3. publish + look-back
  const long base = seq * a.ntiles;
  if (wid == 0) {
    E tot = s_wt[0];
#pragma unroll 1
    for (int w = 1; w < NW; ++w) tot = op(tot, s_wt[w]);
    if (t == 0) {
      if (lane == 0) {
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = tot.e[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = tot.J[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    } else {
      if (lane == 0) {
        gstore(a.agg + (base + t) * E::SIZE, tot);
        lb_store_flag(a.flags + base + t, LB_AGG);
      }
      auto load_agg = [&](long idx, E& v) { gload(v, a.agg + (base + idx) * E::SIZE); };
      auto expand = [&](long idx, E& v) {
        // only (eta, J) of an anchored suffix is ever read: it is the right
        // operand of every combine it takes part in
        const R* p = a.pre + (base + idx) * PS;
        set_identity(v);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          v.e[i] = p[i];
#pragma unroll
          for (int j = 0; j < N; ++j) v.J[i][j] = p[N + i * N + j];
        }
      };
      E ex = lookback<E>(a.flags + base, a.ctr + 2, t, lane, op, load_agg, expand);
      if (lane == 0) {
        R eta[N], J[N][N];
        copy_vec<N, R>(ex.e, eta);
        copy_mat<N, N, R>(ex.J, J);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          s_pre[i] = eta[i];
#pragma unroll
          for (int j = 0; j < N; ++j) s_pre[N + i * N + j] = J[i][j];
        }
        fapply_back<N, P>(tot, eta, J);
        R* p = a.pre + (base + t) * PS;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          p[i] = eta[i];
#pragma unroll
          for (int j = 0; j < N; ++j) p[N + i * N + j] = J[i][j];
        }
        lb_store_flag(a.flags + base + t, LB_PREFIX);
      }
    }
  }
  __syncthreads();

  // 4. apply suffixes, combine with the filter result, write x_{k|T}, P_{k|T}
  R eta[N], J[N][N];
  bool have;
  if (t > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      eta[i] = s_pre[i];
#pragma unroll
      for (int j = 0; j < N; ++j) J[i][j] = s_pre[N + i * N + j];
    }
    if (tid > 0) fapply_back<N, P>(tex, eta, J);
    have = true;
  } else {
    copy_vec<N, R>(tex.e, eta);
    copy_mat<N, N, R>(tex.J, J);
    have = tid > 0;
  }
  const R* __restrict__ mf = a.m_in + seq * a.T * N;
  const R* __restrict__ Pf = a.P_in + seq * a.T * N * N;
  R* __restrict__ mo = a.m_out + seq * a.T * N;
  R* __restrict__ Po = a.P_out + seq * a.T * N * N;
#pragma unroll 1
  for (int i = L - 1; i >= 0; --i) {
    const long k = k0 + i;
    if (k >= a.T) continue;
    if (have) {
      E el = element(k, yv[i]);
      fapply_back<N, P>(el, eta, J);
    } else {
      // suffix of the last row is e alone: eta = 0, J = 0
#pragma unroll
      for (int r = 0; r < N; ++r) {
        eta[r] = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) J[r][c] = R(0);
      }
      have = true;
    }
    R xf[N], Pk[N][N], xs[N], Ps[N][N];
    load_state<N, R>(mf, Pf, k, xf, Pk);
    tf_combine<N, P>(xf, Pk, eta, J, xs, Ps);
#pragma unroll
    for (int r = 0; r < N; ++r) {
      mo[k * N + r] = xs[r];
#pragma unroll
      for (int c = 0; c < N; ++c) Po[k * N * N + r * N + c] = Ps[r][c];
    }
  }
  finish_grid<BLOCK>(a.flags, a.ctr, a.nseq * a.ntiles, &s_last);
}

}  // namespace kfs

// kf_seq.hpp -- the sequential recursions of Sec. III, one lane per sequence.
//
// The classical Kalman filter (Sec. III-A), the RTS smoother and the
// backward information filter with the two-filter combination (Sec. III-B)
// run step by step: a lane carries one sequence from its first step to its
// last, so a single sequence is the work of one GPU lane -- the sequential
// baseline of the speedup experiment (Sec. VI, GPU speedup analysis) -- and a
// batch fills the lanes of as many waves as it has sequences.  The inputs of
// a step (its measurement, its model if time-varying, the filtered moments
// in the backward passes) are loaded a few steps ahead into a ring of
// register sets, so a lane's time per step is its dependency chain, not a
// memory round trip.  Products are formed in P::R, the factorisations and
// solves in P::S, as in the scan kernels.
#pragma once
#include <type_traits>

#include "kf_kernels.hpp"

namespace kfs {

template <class R> struct SeqArgs {
  // time-invariant: one model, or one per sequence of a batch (model_stride
  // 1); time-varying: per-step arrays indexed by the step's row within its
  // sequence, shared by all sequences (u and d may be null = zero)
  const R* F;
  const R* Q;
  const R* H;
  const R* Rm;
  const R* u;
  const R* d;
  const R* m0;
  const R* P0;
  long T;               // steps per sequence (plain and time-varying problems)
  long nseq;
  const int64_t* len;   // ragged batch: steps of sequence i (null otherwise)
  const int64_t* row;   // ragged batch: first row of sequence i
  long total_steps;     // ragged batch: rows of y and of the outputs
  long model_stride;    // 1 if each sequence of a batch has its own model
  unsigned* err;        // error word; bit 1: a batch entry was skipped
};

// Steps and first row of sequence s; false (and bit 1 raised) for a batch
// entry with no steps or rows outside [0, total_steps).
template <class R>
KF_DEV bool seq_bounds(const SeqArgs<R>& a, long s, long& T, long& row0) {
  if (!a.len) {
    T = a.T;
    row0 = s * a.T;
    return true;
  }
  const long t = a.len[s], r = a.row[s];
  if (t < 1 || r < 0 || r > a.total_steps - t) {
    atomicOr(a.err, 2u);
    return false;
  }
  T = t;
  row0 = r;
  return true;
}

template <int N, int M, class R> struct StepModel {
  R F[N][N], Q[N][N], H[M][N], Rm[M][M], u[N], d[M];
};

// Calls f(integral_constant<int, j>) for j = 0 .. D-1 (register-ring slots
// must be compile-time indices).
template <int D, int J = 0, class Fn> KF_DEV void static_for(Fn& f) {
  if constexpr (J < D) {
    f(std::integral_constant<int, J>{});
    static_for<D, J + 1>(f);
  }
}

// Runs body(k, slot) for k = 0 .. n-1 in order, with fetch(k', slot) of
// iteration k' = k + D issued right after body(k) into the slot body(k) has
// just consumed (a ring of D register sets).  Fetches past the end are
// clamped to n - 1 and stay in bounds.  The main loop holds no branch other
// than its back edge, so outstanding loads are counted exactly and only the
// set about to be used is waited for; the last n mod D iterations run
// unrolled under a guard.
template <int D, class Fetch, class Body>
KF_DEV void pipelined(long n, Fetch&& fetch, Body&& body) {
  auto first = [&](auto j) { fetch(j < n ? (long)j : n - 1, j); };
  static_for<D>(first);
  // Drain the prologue's loads (and the caller's) once: with nothing pending
  // on entry, the counts the compiler derives at the loop header are those of
  // the steady state, not the worst case of the two incoming paths.
  __builtin_amdgcn_s_waitcnt(0);
  long k0 = 0;
  auto step = [&](auto j) {
    body(k0 + j, j);
    const long kn = k0 + j + D;
    fetch(kn < n ? kn : n - 1, j);
    // keep the fetch where it is: sunk towards its use, it would be waited for
    // a step or more too early
    __builtin_amdgcn_sched_barrier(0);
  };
  for (; k0 + D <= n; k0 += D) static_for<D>(step);
  auto tail = [&](auto j) {
    if (k0 + j < n) body(k0 + j, j);
  };
  static_for<D>(tail);
}

// Steps fetched ahead: four cover a memory round trip with the work of the
// steps between; two when four sets of W scalars would not leave the step's
// own arithmetic enough of the 256 architectural VGPRs (FP64 arithmetic
// needs twice the registers, so its sets get a smaller share).
template <class R, int W> constexpr int seq_depth() {
  return 4 * W * (int)(sizeof(R) / 4) <= (sizeof(R) == 4 ? 232 : 128) ? 4 : 2;
}

// Loads of the per-step model with branch-free inputs: an absent u or d reads
// the first elements of P0 with stride 0, and its consumer replaces the value
// by zero (in the step's arithmetic, not at the load, which would wait for
// the load right there).
template <class R> struct InputView {
  const R* u;
  const R* d;
  long su, sd;
  bool hu, hd;
};

template <int N, int M, class R> KF_DEV InputView<R> input_view(const SeqArgs<R>& a) {
  InputView<R> v;
  v.hu = a.u != nullptr;
  v.hd = a.d != nullptr;
  v.u = v.hu ? a.u : a.P0;
  v.d = v.hd ? a.d : a.P0;
  v.su = v.hu ? N : 0;
  v.sd = v.hd ? M : 0;
  return v;
}

template <int N, class R> KF_DEV void load_transition(const SeqArgs<R>& a, const InputView<R>& iv,
                                                      long k, R (&F)[N][N], R (&Q)[N][N],
                                                      R (&u)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      F[i][j] = a.F[k * N * N + i * N + j];
      Q[i][j] = a.Q[k * N * N + i * N + j];
    }
#pragma unroll
  for (int i = 0; i < N; ++i) u[i] = iv.u[k * iv.su + i];
}

template <int N, int M, class R>
KF_DEV void load_measurement(const SeqArgs<R>& a, const InputView<R>& iv, long k, R (&H)[M][N],
                             R (&Rm)[M][M], R (&d)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) H[i][j] = a.H[k * M * N + i * N + j];
#pragma unroll
    for (int j = 0; j < M; ++j) Rm[i][j] = a.Rm[k * M * M + i * M + j];
    d[i] = iv.d[k * iv.sd + i];
  }
}

// The model of row r: of step r+1 for H, R, d (eq. y_k), of the transition
// from step r to r+1 for F, Q, u.  Time-invariant models read model `mi` and
// have no inputs.
template <int N, int M, class R, bool TV>
KF_DEV void load_step(const SeqArgs<R>& a, const InputView<R>& iv, long mi, long r,
                      StepModel<N, M, R>& s) {
  if constexpr (TV) {
    load_transition<N>(a, iv, r, s.F, s.Q, s.u);
    load_measurement<N, M>(a, iv, r, s.H, s.Rm, s.d);
  } else {
    load_mat<N, R>(a.F + mi * N * N, s.F);
    load_mat<N, R>(a.Q + mi * N * N, s.Q);
#pragma unroll
    for (int i = 0; i < M; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) s.H[i][j] = a.H[mi * M * N + i * N + j];
#pragma unroll
      for (int j = 0; j < M; ++j) s.Rm[i][j] = a.Rm[mi * M * M + i * M + j];
      s.d[i] = R(0);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) s.u[i] = R(0);
  }
}

template <int K, class R> KF_DEV void load_row(const R* __restrict__ p, long r, R (&v)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = p[r * K + i];
}

template <int N, class R> KF_DEV void load_cov(const R* __restrict__ p, long r, R (&A)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = p[r * N * N + i * N + j];
}

template <int N, class R>
KF_DEV void store_moments(R* __restrict__ mo, R* __restrict__ Po, long r, const R (&x)[N],
                          const R (&Pm)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) mo[r * N + i] = x[i];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Po[r * N * N + i * N + j] = Pm[i][j];
}

// One predict/update step of Sec. III-A with inputs: x^- = F x + u,
// P^- = F P F^T + Q, S = H P^- H^T + R (Cholesky in P::S), innovation
// v = y - H x^- - d; x = x^- + (H P^-)^T S^{-1} v,
// P = P^- - (H P^-)^T S^{-1} H P^-.
template <int N, int M, class P, bool UD>
KF_DEV void seq_kf_step(typename P::R (&x)[N], typename P::R (&Pm)[N][N],
                        const StepModel<N, M, typename P::R>& md, const typename P::R (&y)[M],
                        bool hu, bool hd) {
  using R = typename P::R;
  using S = typename P::S;
  R xp[N], FP[N][N], Pp[N][N], HP[M][N];
  mv<N, N, R>(md.F, x, xp);
  if constexpr (UD) {
#pragma unroll
    for (int i = 0; i < N; ++i) xp[i] += hu ? md.u[i] : R(0);
  }
  mm<N, N, N, R>(md.F, Pm, FP);
  sym_xyt_plus<N, N, R>(FP, md.F, md.Q, Pp);
  mm<M, N, N, R>(md.H, Pp, HP);
  S Sm[M][M], sd[M];
  sym_xyt_plus<M, N, S>(HP, md.H, md.Rm, Sm);
  chol_factor<M, S>(Sm, sd);
  S B[M][N + 1];  // [S^{-1} H P^- | S^{-1} v]
#pragma unroll
  for (int r = 0; r < M; ++r) {
    S v = S(y[r]);
    if constexpr (UD) v -= hd ? S(md.d[r]) : S(0);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      B[r][c] = S(HP[r][c]);
      v -= S(md.H[r][c]) * S(xp[c]);
    }
    B[r][N] = v;
  }
  chol_solve<M, N + 1, S>(Sm, sd, B);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S s = S(xp[i]);
#pragma unroll
    for (int t = 0; t < M; ++t) s += S(HP[t][i]) * B[t][N];
    x[i] = R(s);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      S s = S(Pp[i][j]);
#pragma unroll
      for (int t = 0; t < M; ++t) s -= S(HP[t][i]) * B[t][j];
      Pm[i][j] = R(s);
      Pm[j][i] = R(s);
    }
}

// Kalman filter over each sequence (Sec. III-A), from x_{0|0} = m0,
// P_{0|0} = P0; writes x_{k|k}, P_{k|k} at the sequence's rows.
template <int N, int M, class P, bool TV>
__global__ __launch_bounds__(64) void k_seq_filter(SeqArgs<typename P::R> a,
                                                   const typename P::R* __restrict__ y,
                                                   typename P::R* __restrict__ mo,
                                                   typename P::R* __restrict__ Po) {
  using R = typename P::R;
  constexpr int D = seq_depth<R, M + (TV ? 2 * N * N + M * N + M * M + N + M : 0)>();
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= a.nseq) return;
  long T, row0;
  if (!seq_bounds(a, s, T, row0)) return;
  const long mi = s * a.model_stride;
  const InputView<R> iv = input_view<N, M>(a);
  R x[N], Pm[N][N];
  load_row<N>(a.m0, mi, x);
  load_cov<N>(a.P0, mi, Pm);
  StepModel<N, M, R> md[TV ? D : 1];
  if constexpr (!TV) load_step<N, M, R, false>(a, iv, mi, 0, md[0]);
  R yb[D][M];
  pipelined<D>(
      T,
      [&](long k, auto j) {
        if constexpr (TV) load_step<N, M, R, true>(a, iv, mi, k, md[j]);
        load_row<M>(y, row0 + k, yb[j]);
      },
      [&](long k, auto j) {
        seq_kf_step<N, M, P, TV>(x, Pm, md[TV ? (int)j : 0], yb[j], iv.hu, iv.hd);
        store_moments<N>(mo, Po, row0 + k, x, Pm);
      });
}

// RTS smoother over each sequence (Sec. III-B), from x_{T|T}, P_{T|T}
// backwards: with x^- = F x_{k|k} + u, P^- = F P_{k|k} F^T + Q (the
// transition to step k+1), G^T = (P^-)^{-1} F P_{k|k} (Cholesky in P::S),
// x_{k|T} = x_{k|k} + G (x_{k+1|T} - x^-),
// P_{k|T} = P_{k|k} + G (P_{k+1|T} - P^-) G^T.
template <int N, int M, class P, bool TV>
__global__ __launch_bounds__(64) void k_seq_rts(SeqArgs<typename P::R> a,
                                                const typename P::R* __restrict__ mf,
                                                const typename P::R* __restrict__ Pf,
                                                typename P::R* __restrict__ ms,
                                                typename P::R* __restrict__ Ps) {
  using R = typename P::R;
  using S = typename P::S;
  constexpr int D = seq_depth<R, N + N * N + (TV ? 2 * N * N + N : 0)>();
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= a.nseq) return;
  long T, row0;
  if (!seq_bounds(a, s, T, row0)) return;
  const long mi = s * a.model_stride;
  const InputView<R> iv = input_view<N, M>(a);
  R xs[N], Pss[N][N];
  load_row<N>(mf, row0 + T - 1, xs);
  load_cov<N>(Pf, row0 + T - 1, Pss);
  store_moments<N>(ms, Ps, row0 + T - 1, xs, Pss);
  if (T < 2) return;
  // iteration k smooths row r = T - 2 - k with the transition of row r + 1
  R Ft[TV ? D : 1][N][N], Qt[TV ? D : 1][N][N], ut[TV ? D : 1][N];
  if constexpr (!TV) {
    load_mat<N, R>(a.F + mi * N * N, Ft[0]);
    load_mat<N, R>(a.Q + mi * N * N, Qt[0]);
#pragma unroll
    for (int i = 0; i < N; ++i) ut[0][i] = R(0);
  }
  R xb[D][N], Pb[D][N][N];
  pipelined<D>(
      T - 1,
      [&](long k, auto j) {
        const long r = T - 2 - k;
        if constexpr (TV) load_transition<N>(a, iv, r + 1, Ft[j], Qt[j], ut[j]);
        load_row<N>(mf, row0 + r, xb[j]);
        load_cov<N>(Pf, row0 + r, Pb[j]);
      },
      [&](long k, auto j) {
        const long r = T - 2 - k;
        constexpr int t = TV ? (int)decltype(j)::value : 0;
        const R(&F)[N][N] = Ft[t];
        const R(&xc)[N] = xb[j];
        const R(&Pc)[N][N] = Pb[j];
        R xp[N], FP[N][N];
        mv<N, N, R>(F, xc, xp);
        if constexpr (TV) {
#pragma unroll
          for (int i = 0; i < N; ++i) xp[i] += iv.hu ? ut[t][i] : R(0);
        }
        mm<N, N, N, R>(F, Pc, FP);
        S Pp[N][N], L[N][N], dl[N], B[N][N];
        sym_xyt_plus<N, N, S>(FP, F, Qt[t], Pp);
        copy_mat<N, N, S>(Pp, L);
        chol_factor<N, S>(L, dl);
        copy_mat<N, N, S>(FP, B);
        chol_solve<N, N, S>(L, dl, B);  // B = G^T
        S dv[N], Dm[N][N], DB[N][N];
#pragma unroll
        for (int i = 0; i < N; ++i) dv[i] = S(xs[i]) - S(xp[i]);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          S g = S(xc[i]);
#pragma unroll
          for (int q = 0; q < N; ++q) g += B[q][i] * dv[q];
          xs[i] = R(g);
        }
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int q = 0; q < N; ++q) Dm[i][q] = S(Pss[i][q]) - Pp[i][q];
        mm<N, N, N, S>(Dm, B, DB);
        sym_xty_plus<N, N, S>(B, DB, Pc, Pss);
        store_moments<N>(ms, Ps, row0 + r, xs, Pss);
      });
}

// H^T R^{-1} H and (R^{-1} H)^T = H^T R^{-1} of one step, in P::S.
template <int N, int M, class P>
KF_DEV void info_terms(const typename P::R (&H)[M][N], const typename P::R (&Rm)[M][M],
                       typename P::S (&HtRi)[N][M], typename P::S (&HtRiH)[N][N]) {
  using S = typename P::S;
  S Rl[M][M], rd[M], X[M][N], Z[N][N];
  copy_mat<M, M, S>(Rm, Rl);
  chol_factor<M, S>(Rl, rd);
  copy_mat<M, N, S>(H, X);
  chol_solve<M, N, S>(Rl, rd, X);  // R^{-1} H
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < M; ++q) HtRi[i][q] = X[q][i];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Z[i][j] = S(0);
  sym_xty_plus<N, M, S>(H, X, Z, HtRiH);
}

// Measurement update of the backward information filter: eta += H^T R^{-1}
// (y - d), J += H^T R^{-1} H.  The pair is carried in P::S: it is never
// stored, and J grows with R^{-1}, so an FP32 copy of it would lose what
// (I + P J)^{-1} needs in the combination.
template <int N, int M, class P>
KF_DEV void info_update(typename P::S (&eta)[N], typename P::S (&J)[N][N],
                        const typename P::S (&HtRi)[N][M], const typename P::S (&HtRiH)[N][N],
                        const typename P::R (&d)[M], const typename P::R (&y)[M]) {
  using S = typename P::S;
  S v[M];
#pragma unroll
  for (int q = 0; q < M; ++q) v[q] = S(y[q]) - S(d[q]);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < M; ++q) eta[i] += HtRi[i][q] * v[q];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      const S t = J[i][j] + HtRiH[i][j];
      J[i][j] = t;
      J[j][i] = t;
    }
}

// What one backward two-filter iteration reads (row r, transition of r + 1).
template <int N, int M, class R, bool TV> struct TfFetch {
  R x[N], Pm[N][N], y[M];
  R F[TV ? N : 1][TV ? N : 1], Q[TV ? N : 1][TV ? N : 1], u[TV ? N : 1];
  R H[TV ? M : 1][TV ? N : 1], Rm[TV ? M : 1][TV ? M : 1], d[TV ? M : 1];
};

// Two-filter smoother over each sequence (Sec. III-B): the backward
// information filter from eta_{T|T:T}, J_{T|T:T} (its prediction
// eta <- F^T (I + J Q)^{-1} (eta - J u), J <- F^T (I + J Q)^{-1} J F with
// the transition into the next step, LU in P::S), each predicted pair
// combined with the filtered moments by eqs. mean_tf_combination and
// cov_tf_combination.  The information pair stays in P::S throughout.  At
// the last step the predicted pair is zero and the smoothed moments are the
// filtered ones.
template <int N, int M, class P, bool TV>
__global__ __launch_bounds__(64) void k_seq_twofilter(SeqArgs<typename P::R> a,
                                                      const typename P::R* __restrict__ y,
                                                      const typename P::R* __restrict__ mf,
                                                      const typename P::R* __restrict__ Pf,
                                                      typename P::R* __restrict__ ms,
                                                      typename P::R* __restrict__ Ps) {
  using R = typename P::R;
  using S = typename P::S;
  constexpr int D =
      seq_depth<R, N + N * N + M + (TV ? 2 * N * N + N + M * N + M * M + M : 0)>();
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= a.nseq) return;
  long T, row0;
  if (!seq_bounds(a, s, T, row0)) return;
  const long mi = s * a.model_stride;
  const InputView<R> iv = input_view<N, M>(a);
  {
    R x[N], Pm[N][N];
    load_row<N>(mf, row0 + T - 1, x);
    load_cov<N>(Pf, row0 + T - 1, Pm);
    store_moments<N>(ms, Ps, row0 + T - 1, x, Pm);
  }
  // time-invariant models: the model and H^T R^{-1}, H^T R^{-1} H once
  StepModel<N, M, R> md;
  S HtRi[N][M], HtRiH[N][N];
  R dz[M];
#pragma unroll
  for (int q = 0; q < M; ++q) dz[q] = R(0);
  S eta[N], J[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    eta[i] = S(0);
#pragma unroll
    for (int j = 0; j < N; ++j) J[i][j] = S(0);
  }
  {
    // the measurement of row T - 1
    R H[M][N], Rm[M][M], d[M], yl[M];
    if constexpr (TV) {
      load_measurement<N, M>(a, iv, T - 1, H, Rm, d);
#pragma unroll
      for (int q = 0; q < M; ++q) d[q] = iv.hd ? d[q] : R(0);
    } else {
      load_step<N, M, R, false>(a, iv, mi, 0, md);
      copy_mat<M, N, R>(md.H, H);
      copy_mat<M, M, R>(md.Rm, Rm);
      copy_vec<M, R>(dz, d);
    }
    load_row<M>(y, row0 + T - 1, yl);
    info_terms<N, M, P>(H, Rm, HtRi, HtRiH);
    info_update<N, M, P>(eta, J, HtRi, HtRiH, d, yl);
  }
  if (T < 2) return;
  // iteration k: predict through the transition of row r + 1 (r = T - 2 - k),
  // combine at row r, then add the measurement of row r
  TfFetch<N, M, R, TV> fb[D];
  pipelined<D>(
      T - 1,
      [&](long k, auto j) {
        const long r = T - 2 - k;
        load_row<N>(mf, row0 + r, fb[j].x);
        load_cov<N>(Pf, row0 + r, fb[j].Pm);
        load_row<M>(y, row0 + r, fb[j].y);
        if constexpr (TV) {
          load_transition<N>(a, iv, r + 1, fb[j].F, fb[j].Q, fb[j].u);
          load_measurement<N, M>(a, iv, r, fb[j].H, fb[j].Rm, fb[j].d);
        }
      },
      [&](long k, auto j) {
        const long r = T - 2 - k;
        const TfFetch<N, M, R, TV>& f = fb[j];
        const R(&F)[N][N] = [&]() -> const R(&)[N][N] {
          if constexpr (TV) return f.F; else return md.F;
        }();
        const R(&Q)[N][N] = [&]() -> const R(&)[N][N] {
          if constexpr (TV) return f.Q; else return md.Q;
        }();
        S Mi[N][N];
        mm<N, N, N, S>(J, Q, Mi);
#pragma unroll
        for (int i = 0; i < N; ++i) Mi[i][i] += S(1);
        int piv[N];
        S di[N];
        lu_factor<N, S>(Mi, piv, di);
        S B[N][N + 1];  // [J F | eta - J u]
#pragma unroll
        for (int i = 0; i < N; ++i) {
          S e = eta[i];
#pragma unroll
          for (int c = 0; c < N; ++c) {
            S t = S(0);
#pragma unroll
            for (int q = 0; q < N; ++q) t += J[i][q] * S(F[q][c]);
            B[i][c] = t;
            if constexpr (TV) e -= iv.hu ? J[i][c] * S(f.u[c]) : S(0);
          }
          B[i][N] = e;
        }
        lu_solve<N, N + 1, S>(Mi, piv, di, B);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          S e = S(0);
#pragma unroll
          for (int q = 0; q < N; ++q) e += S(F[q][i]) * B[q][N];
          eta[i] = e;
        }
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int c = i; c < N; ++c) {
            S t = S(0);
#pragma unroll
            for (int q = 0; q < N; ++q) t += S(F[q][i]) * B[q][c];
            J[i][c] = t;
            J[c][i] = t;
          }
        R xo[N], Po_[N][N];
        tf_combine<N, P>(f.x, f.Pm, eta, J, xo, Po_);
        store_moments<N>(ms, Ps, row0 + r, xo, Po_);
        if constexpr (TV) {
          R d[M];
#pragma unroll
          for (int q = 0; q < M; ++q) d[q] = iv.hd ? f.d[q] : R(0);
          info_terms<N, M, P>(f.H, f.Rm, HtRi, HtRiH);
          info_update<N, M, P>(eta, J, HtRi, HtRiH, d, f.y);
        } else {
          info_update<N, M, P>(eta, J, HtRi, HtRiH, dz, f.y);
        }
      });
}

}  // namespace kfs

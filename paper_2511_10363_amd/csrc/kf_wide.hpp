// kf_wide.hpp -- the three scans for states too wide for a register-resident
// element (nx = 8 and 16: a filtering element of Sec. IV-C has 3 nx^2 + 2 nx
// scalars, 416 at nx = 8).
//
// An element is spread over a group of G = nx lanes of a wavefront, one row
// per lane: lane r holds row r of A, C, J (resp. E, L) and entry r of b, eta
// (resp. g).  The operators of Lemma 1 and Lemma 2 are computed row by row:
//   * a product X Y takes row r of X from the lane's registers and Y from a
//     per-group LDS scratch where every lane has put its row of Y (all lanes
//     of a group read the same addresses, so the reads are broadcasts);
//     transposed operands are read as columns of a staged matrix;
//   * the solves with I + C_i J_j (Lemma 1), I + P J (the two-filter
//     combination) and F P F^T + Q (eq. prts_init1) are one Gauss-Jordan
//     elimination with partial pivoting across the group's lanes: the pivot
//     row of each column is chosen from the candidates every lane posts in
//     LDS and broadcast through LDS, and each lane keeps the solution row of
//     the column it was pivot for, which the next product stages at that
//     row -- so the row interchanges cost nothing;
//   * symmetric results are formed in the upper triangle (the lane's columns
//     c >= r) and mirrored through LDS, so they are exactly symmetric.
// The groups of a workgroup take the place of the threads of the
// register-resident scans: a tile holds (BLOCK / G) * L steps, each group
// folds L of them, the groups of a wavefront scan with cross-lane shuffles
// (G lanes apart), the wavefront totals combine through LDS, and the
// decoupled look-back assigns predecessor tiles to groups.
// The precision policy is the same as elsewhere: P::R for elements and
// storage, P::S for the factorisations, solves and symmetric assemblies.
#pragma once
#include "kf_kernels.hpp"

namespace kfs {

// ---------------------------------------------------------------------------
// Rows of elements and states
// ---------------------------------------------------------------------------
template <int N, class R> struct WFE {  // row of a filtering element (A, b, C, eta, J)
  R A[N];
  R b;
  R C[N];
  R e;
  R J[N];
  static constexpr int SIZE = 3 * N + 2;
};
template <int N, class R> struct WSE {  // row of a smoothing element (E, g, L)
  R E[N];
  R g;
  R L[N];
  static constexpr int SIZE = 2 * N + 1;
};
template <int N, class R> struct WSt {  // row of an anchored state (v, m)
  R v;
  R m[N];
  static constexpr int SIZE = N + 1;
};

template <int N, class R, class F> KF_DEV void each(WFE<N, R>& x, F f) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.A[i], k++);
  f(x.b, k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.C[i], k++);
  f(x.e, k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.J[i], k++);
}
template <int N, class R, class F> KF_DEV void each(WSE<N, R>& x, F f) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.E[i], k++);
  f(x.g, k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.L[i], k++);
}
template <int N, class R, class F> KF_DEV void each(WSt<N, R>& x, F f) {
  f(x.v, 0);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.m[i], i + 1);
}

// Row r of the two-sided identities (I, 0, 0, 0, 0) and (I, 0, 0).
template <int N, class R> KF_DEV void set_identity_row(WFE<N, R>& x, int r) {
  each(x, [](R& v, int) { v = R(0); });
#pragma unroll
  for (int i = 0; i < N; ++i) x.A[i] = (i == r) ? R(1) : R(0);
}
template <int N, class R> KF_DEV void set_identity_row(WSE<N, R>& x, int r) {
  each(x, [](R& v, int) { v = R(0); });
#pragma unroll
  for (int i = 0; i < N; ++i) x.E[i] = (i == r) ? R(1) : R(0);
}
template <int N, class R> KF_DEV void st_zero_row(WSt<N, R>& s) {
  each(s, [](R& v, int) { v = R(0); });
}

// ---------------------------------------------------------------------------
// Per-group LDS scratch and the row-distributed primitives.  Every primitive
// is collective over the lanes of one group, which execute it together.
// ---------------------------------------------------------------------------
template <int N, class S> struct GScr {
  S X[N * N];        // a staged matrix, row-major
  S Y[N * N];        // a second one
  S u[N], w[N];      // staged vectors
  S pr[3 * N + 2];   // pivot row of the elimination
  S cand[N];         // pivot candidates
};

// Lane r puts its row into a staged matrix / its entry into a staged vector.
template <int N, class S, class T> KF_DEV void g_put(S* buf, int r, const T (&row)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) buf[r * N + c] = S(row[c]);
}
// o = x Y (row r of X Y), Y staged; accumulated in Acc in the order of k
template <int N, class Acc, class S, class T>
KF_DEV void g_mul(const T (&x)[N], const S* __restrict__ Y, Acc (&o)[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) o[c] = Acc(x[0]) * Acc(Y[c]);
#pragma unroll
  for (int k = 1; k < N; ++k) {
    const Acc xk = Acc(x[k]);
#pragma unroll
    for (int c = 0; c < N; ++c) o[c] += xk * Acc(Y[k * N + c]);
  }
}
// x . v, v staged
template <int N, class Acc, class S, class T>
KF_DEV Acc g_dot(const T (&x)[N], const S* __restrict__ v) {
  Acc s = Acc(x[0]) * Acc(v[0]);
#pragma unroll
  for (int k = 1; k < N; ++k) s += Acc(x[k]) * Acc(v[k]);
  return s;
}
// column r of a staged matrix
template <int N, class T, class S> KF_DEV void g_col(const S* __restrict__ X, int r, T (&o)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) o[k] = T(X[k * N + r]);
}
// Make a row-distributed matrix exactly symmetric: keep the lane's upper
// triangle (c >= r), take the lower one from the lanes that own it.
template <int N, class T, class S> KF_DEV void g_mirror(T (&o)[N], int r, S* __restrict__ buf) {
  g_put<N>(buf, r, o);
  wave_lds_sync();
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const T t = T(buf[c * N + r]);
    o[c] = (c < r) ? t : o[c];
  }
  wave_lds_sync();
}
// o = X V^T + D for a symmetric result: row r of X in registers, V staged
// (row c of V at V[c]); upper triangle in Acc, then mirrored through buf.
template <int N, class Acc, class TO, class TX, class TD, class S>
KF_DEV void g_sym_xvt(const TX (&x)[N], const S* __restrict__ V, const TD (&d)[N], int r,
                      TO (&o)[N], S* __restrict__ buf) {
#pragma unroll
  for (int c = 0; c < N; ++c) {
    Acc s = Acc(d[c]);
#pragma unroll
    for (int t = 0; t < N; ++t) s += Acc(x[t]) * Acc(V[c * N + t]);
    o[c] = TO(s);
  }
  wave_lds_sync();
  g_mirror<N>(o, r, buf);
}
// o = Z^T Y + D for a symmetric result: Z and Y staged (column r of Z, all
// of Y); upper triangle in Acc, mirrored through buf.
template <int N, class Acc, class TO, class TD, class S>
KF_DEV void g_sym_zty(const S* __restrict__ Z, const S* __restrict__ Y, const TD (&d)[N], int r,
                      TO (&o)[N], S* __restrict__ buf) {
  Acc zc[N];
  g_col<N>(Z, r, zc);
#pragma unroll
  for (int c = 0; c < N; ++c) {
    Acc s = Acc(d[c]);
#pragma unroll
    for (int t = 0; t < N; ++t) s += zc[t] * Acc(Y[t * N + c]);
    o[c] = TO(s);
  }
  wave_lds_sync();
  g_mirror<N>(o, r, buf);
}

// Gauss-Jordan elimination with partial pivoting of M X = B, with row r of M
// and of B in lane r (m, b; both destroyed).  Column p takes as pivot the
// unused row of largest |M[.][p]| (lowest row on ties); every other row
// eliminates column p with it, and the pivot row is scaled by its inverse.
// Returns the column this lane's row was pivot for: b then holds that row
// of X.  A zero pivot (singular M) or a non-finite entry makes X non-finite.
template <int N, int NR, class S>
KF_DEV int g_solve(S (&m)[N], S (&b)[NR], int r, S* __restrict__ pr, S* __restrict__ cand) {
  bool used = false;
  int mine = 0;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    cand[r] = used ? S(-1) : kabs(m[p]);
    wave_lds_sync();
    int piv = 0;
    S best = cand[0];
#pragma unroll
    for (int q = 1; q < N; ++q) {
      const S cq = cand[q];
      const bool gt = cq > best;
      best = gt ? cq : best;
      piv = gt ? q : piv;
    }
    if (r == piv) {
#pragma unroll
      for (int c = p; c < N; ++c) pr[c] = m[c];
#pragma unroll
      for (int j = 0; j < NR; ++j) pr[N + j] = b[j];
    }
    wave_lds_sync();
    const S d = krcp(pr[p]);
    if (r == piv) {
      used = true;
      mine = p;
#pragma unroll
      for (int c = p + 1; c < N; ++c) m[c] *= d;
#pragma unroll
      for (int j = 0; j < NR; ++j) b[j] *= d;
    } else {
      const S f = m[p] * d;
#pragma unroll
      for (int c = p + 1; c < N; ++c) m[c] -= f * pr[c];
#pragma unroll
      for (int j = 0; j < NR; ++j) b[j] -= f * pr[N + j];
    }
    wave_lds_sync();
  }
  return mine;
}

// ---------------------------------------------------------------------------
// Lemma 1, row-distributed.  With M = I + C_x J_y, Z = M^{-1} A_x,
// Y = M^{-1} C_x and v = M^{-1}(b_x + C_x eta_y):
//   A = A_y Z,  b = A_y v + b_y,  C = A_y Y A_y^T + C_y,
//   eta = Z^T (eta_y - J_y b_x) + eta_x,  J = Z^T (J_y A_x) + J_x.
// ---------------------------------------------------------------------------
template <int N, class P>
KF_DEV WFE<N, typename P::R> g_fcombine(const WFE<N, typename P::R>& x,
                                        const WFE<N, typename P::R>& y, int r,
                                        GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.X, r, y.J);
  g.u[r] = S(y.e);
  wave_lds_sync();
  S m[N];
  g_mul<N, S>(x.C, g.X, m);
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] += (c == r) ? S(1) : S(0);
  S b[2 * N + 1];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    b[c] = S(x.A[c]);
    b[N + c] = S(x.C[c]);
  }
  b[2 * N] = S(x.b) + g_dot<N, S>(x.C, g.u);
  wave_lds_sync();
  const int row = g_solve<N, 2 * N + 1, S>(m, b, r, g.pr, g.cand);
  // Z -> X, Y -> Y, v -> u, each row at the column it solved for
#pragma unroll
  for (int c = 0; c < N; ++c) {
    g.X[row * N + c] = S(R(b[c]));
    g.Y[row * N + c] = S(R(b[N + c]));
  }
  g.u[row] = S(R(b[2 * N]));
  g.w[r] = S(x.b);
  wave_lds_sync();
  WFE<N, R> o;
  g_mul<N, R>(y.A, g.X, o.A);
  o.b = g_dot<N, R>(y.A, g.u) + y.b;
  R AY[N];
  g_mul<N, R>(y.A, g.Y, AY);
  // w = eta_y - J_y b_x
  const R wr = y.e - g_dot<N, R>(y.J, g.w);
  wave_lds_sync();
  g_put<N>(g.Y, r, y.A);
  g.u[r] = S(wr);
  wave_lds_sync();
  g_sym_xvt<N, S>(AY, g.Y, y.C, r, o.C, g.Y);
  // eta = Z^T w + eta_x (column r of Z)
  {
    R zc[N];
    g_col<N>(g.X, r, zc);
    o.e = g_dot<N, R>(zc, g.u) + x.e;
  }
  wave_lds_sync();
  g_put<N>(g.Y, r, x.A);
  wave_lds_sync();
  R JA[N];
  g_mul<N, R>(y.J, g.Y, JA);
  wave_lds_sync();
  g_put<N>(g.Y, r, JA);
  wave_lds_sync();
  g_sym_zty<N, S>(g.X, g.Y, x.J, r, o.J, g.Y);
  return o;
}

// Lemma 1 with a left operand whose A is zero (an anchored filtering state
// (x, P), row r: st.v = x_r, st.m = row r of P): only b and C are formed,
//   b' = A_y M^{-1}(x + P eta_y) + b_y,  C' = A_y M^{-1} P A_y^T + C_y,  M = I + P J_y.
template <int N, class P>
KF_DEV void g_fapply(WSt<N, typename P::R>& st, const WFE<N, typename P::R>& y, int r,
                     GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.X, r, y.J);
  g.u[r] = S(y.e);
  wave_lds_sync();
  S m[N];
  g_mul<N, S>(st.m, g.X, m);
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] += (c == r) ? S(1) : S(0);
  S b[N + 1];
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = S(st.m[c]);
  b[N] = S(st.v) + g_dot<N, S>(st.m, g.u);
  wave_lds_sync();
  const int row = g_solve<N, N + 1, S>(m, b, r, g.pr, g.cand);
#pragma unroll
  for (int c = 0; c < N; ++c) g.Y[row * N + c] = S(R(b[c]));
  g.u[row] = S(R(b[N]));
  wave_lds_sync();
  st.v = g_dot<N, R>(y.A, g.u) + y.b;
  R AY[N];
  g_mul<N, R>(y.A, g.Y, AY);
  wave_lds_sync();
  g_put<N>(g.X, r, y.A);
  wave_lds_sync();
  g_sym_xvt<N, S>(AY, g.X, y.C, r, st.m, g.Y);
}

// Lemma 1 with a right operand of which only (eta, J) is needed (a suffix
// of the two-filter backward scan; st.v = eta_r, st.m = row r of J):
//   eta' = Z^T (eta - J b_a) + eta_a,  J' = Z^T (J A_a) + J_a,  Z = (I + C_a J)^{-1} A_a.
template <int N, class P>
KF_DEV void g_fapply_back(const WFE<N, typename P::R>& a, WSt<N, typename P::R>& st, int r,
                          GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.X, r, st.m);
  g.w[r] = S(a.b);
  wave_lds_sync();
  S m[N];
  g_mul<N, S>(a.C, g.X, m);
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] += (c == r) ? S(1) : S(0);
  S b[N];
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = S(a.A[c]);
  const R wr = st.v - g_dot<N, R>(st.m, g.w);
  wave_lds_sync();
  const int row = g_solve<N, N, S>(m, b, r, g.pr, g.cand);
  // J stays staged in Y for J A_a; Z -> X
  g_put<N>(g.Y, r, a.A);
  wave_lds_sync();
  R JA[N];
  g_mul<N, R>(st.m, g.Y, JA);
  wave_lds_sync();
#pragma unroll
  for (int c = 0; c < N; ++c) g.X[row * N + c] = S(R(b[c]));
  g.u[r] = S(wr);
  g_put<N>(g.Y, r, JA);
  wave_lds_sync();
  {
    R zc[N];
    g_col<N>(g.X, r, zc);
    st.v = g_dot<N, R>(zc, g.u) + a.e;
  }
  g_sym_zty<N, S>(g.X, g.Y, a.J, r, st.m, g.Y);
}

// ---------------------------------------------------------------------------
// Lemma 2, row-distributed: E = E_x E_y, g = E_x g_y + g_x,
// L = E_x L_y E_x^T + L_x.
// ---------------------------------------------------------------------------
template <int N, class P>
KF_DEV WSE<N, typename P::R> g_scombine(const WSE<N, typename P::R>& x,
                                        const WSE<N, typename P::R>& y, int r,
                                        GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.X, r, y.E);
  g_put<N>(g.Y, r, y.L);
  g.u[r] = S(y.g);
  wave_lds_sync();
  WSE<N, R> o;
  g_mul<N, R>(x.E, g.X, o.E);
  o.g = g_dot<N, R>(x.E, g.u) + x.g;
  R EL[N];
  g_mul<N, R>(x.E, g.Y, EL);
  wave_lds_sync();
  g_put<N>(g.X, r, x.E);
  wave_lds_sync();
  g_sym_xvt<N, S>(EL, g.X, x.L, r, o.L, g.Y);
  return o;
}

// Lemma 2 with a right operand whose E is zero (an anchored smoothing state
// (g, L), row r): st := a (x) (0, g, L).
template <int N, class P>
KF_DEV void g_sapply(const WSE<N, typename P::R>& a, WSt<N, typename P::R>& st, int r,
                     GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.Y, r, st.m);
  g.u[r] = S(st.v);
  wave_lds_sync();
  st.v = g_dot<N, R>(a.E, g.u) + a.g;
  R EL[N];
  g_mul<N, R>(a.E, g.Y, EL);
  wave_lds_sync();
  g_put<N>(g.X, r, a.E);
  wave_lds_sync();
  g_sym_xvt<N, S>(EL, g.X, a.L, r, st.m, g.Y);
}

// Smoothing element of eq. prts_init1, row r, from the filter moments (x_r,
// row r of P) and rows r of F, Q:  E = P F^T (F P F^T + Q)^{-1},
// g = x - E F x,  L = P - E F P  (all in S).
template <int N, class P, class TF>
KF_DEV WSE<N, typename P::R> g_smooth_element(typename P::R xr, const typename P::R (&Pr)[N],
                                              const TF (&Fr)[N], const TF (&Qr)[N], int r,
                                              GScr<N, typename P::S>& g) {
  using R = typename P::R;
  using S = typename P::S;
  g_put<N>(g.X, r, Pr);
  g_put<N>(g.Y, r, Fr);
  g.u[r] = S(xr);
  wave_lds_sync();
  S FP[N];
  g_mul<N, S>(Fr, g.X, FP);                 // row r of F P
  const S Fx = g_dot<N, S>(Fr, g.u);        // (F x)_r
  S Sm[N];                                  // row r of F P F^T + Q, upper triangle
#pragma unroll
  for (int c = 0; c < N; ++c) {
    S s = S(Qr[c]);
#pragma unroll
    for (int t = 0; t < N; ++t) s += FP[t] * g.Y[c * N + t];
    Sm[c] = s;
  }
  wave_lds_sync();
  g_mirror<N>(Sm, r, g.X);
  S b[N];
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = FP[c];
  const int row = g_solve<N, N, S>(Sm, b, r, g.pr, g.cand);
  // E^T = (F P F^T + Q)^{-1} F P -> X (row at its column), F P -> Y, F x -> w
#pragma unroll
  for (int c = 0; c < N; ++c) g.X[row * N + c] = b[c];
  g_put<N>(g.Y, r, FP);
  g.w[r] = Fx;
  wave_lds_sync();
  WSE<N, R> o;
  S ec[N];                                  // row r of E = column r of E^T
  g_col<N>(g.X, r, ec);
#pragma unroll
  for (int c = 0; c < N; ++c) o.E[c] = R(ec[c]);
  {
    S s = S(xr);
#pragma unroll
    for (int t = 0; t < N; ++t) s -= ec[t] * g.w[t];
    o.g = R(s);
  }
#pragma unroll
  for (int c = 0; c < N; ++c) {
    S s = S(Pr[c]);
#pragma unroll
    for (int t = 0; t < N; ++t) s -= ec[t] * g.Y[t * N + c];
    o.L[c] = R(s);
  }
  wave_lds_sync();
  g_mirror<N>(o.L, r, g.Y);
  return o;
}

// Two-filter combination (eqs. mean_tf_combination, cov_tf_combination), row
// r: x_s = (I + P J)^{-1}(x + P eta), P_s = (I + P J)^{-1} P symmetrised by
// averaging with its transpose (in S).  (eta, J) is the anchored suffix
// state st.
template <int N, class P>
KF_DEV void g_tf_combine(typename P::R xr, const typename P::R (&Pr)[N],
                         const WSt<N, typename P::R>& st, int r, typename P::R& xs,
                         typename P::R (&Ps)[N], GScr<N, typename P::S>& g) {
  using S = typename P::S;
  using R = typename P::R;
  g_put<N>(g.X, r, st.m);
  g.u[r] = S(st.v);
  wave_lds_sync();
  S m[N];
  g_mul<N, S>(Pr, g.X, m);
#pragma unroll
  for (int c = 0; c < N; ++c) m[c] += (c == r) ? S(1) : S(0);
  S b[N + 1];
#pragma unroll
  for (int c = 0; c < N; ++c) b[c] = S(Pr[c]);
  b[N] = S(xr) + g_dot<N, S>(Pr, g.u);
  wave_lds_sync();
  const int row = g_solve<N, N + 1, S>(m, b, r, g.pr, g.cand);
#pragma unroll
  for (int c = 0; c < N; ++c) g.Y[row * N + c] = b[c];
  g.w[row] = b[N];
  wave_lds_sync();
  xs = R(g.w[r]);
#pragma unroll
  for (int c = 0; c < N; ++c) Ps[c] = R(S(0.5) * (g.Y[r * N + c] + g.Y[c * N + r]));
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// Per-model constants (eqs. pkf_init1..3), FP64, one workgroup per model,
// every product spread over the workgroup's threads.  Same quantities and
// layout (CL<N, M>) as k_prepare, without the aggregate tables; also zeroes
// the workspace's control region.
// ---------------------------------------------------------------------------
template <int N, int M>
struct WPrep {
  double F[N][N], Q[N][N], H[M][N], Rm[M][M], m0[N], P0[N][N];
  double HQ[M][N], HF[M][N], FP0[N][N], x[N];
  double S[M][M], P[N][N], HP[M][N], S1[M][M], Hx[M];
  double Kt[M][N], Wt[M][N], K1t[M][N];
  double IKH[N][N], A[N][N], C[N][N];
};

// Solve (L L^T) X = B for an SPD K x K matrix S (one thread), B: K x N in place.
template <int K, int N>
KF_DEV void chol_solve_shared(const double (&S)[K][K], double (&B)[K][N]) {
  double Lm[K][K], dinv[K];
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) Lm[i][j] = S[i][j];
  chol_factor<K, double>(Lm, dinv);
  for (int c = 0; c < N; ++c) {
    double v[K][1];
#pragma unroll
    for (int i = 0; i < K; ++i) v[i][0] = B[i][c];
    chol_solve<K, 1, double>(Lm, dinv, v);
#pragma unroll
    for (int i = 0; i < K; ++i) B[i][c] = v[i][0];
  }
}

template <int N, int M, class R>
__global__ __launch_bounds__(256) void k_wprepare(const R* __restrict__ F_, const R* __restrict__ Q_,
                                                  const R* __restrict__ H_, const R* __restrict__ R_,
                                                  const R* __restrict__ m0_,
                                                  const R* __restrict__ P0_, R* __restrict__ cst,
                                                  unsigned* __restrict__ ctrl, size_t ctrl_words,
                                                  long nmodels, long cst_stride) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ctrl_words;
       i += (size_t)gridDim.x * blockDim.x)
    ctrl[i] = 0u;
  const long mdl = blockIdx.x;
  if (mdl >= nmodels) return;
  F_ += mdl * N * N;
  Q_ += mdl * N * N;
  H_ += mdl * M * N;
  R_ += mdl * M * M;
  m0_ += mdl * N;
  P0_ += mdl * N * N;
  cst += mdl * cst_stride;
  using LY = CL<N, M>;
  __shared__ WPrep<N, M> s;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < N * N; i += nt) {
    (&s.F[0][0])[i] = double(F_[i]);
    (&s.Q[0][0])[i] = double(Q_[i]);
    (&s.P0[0][0])[i] = double(P0_[i]);
  }
  for (int i = tid; i < M * N; i += nt) (&s.H[0][0])[i] = double(H_[i]);
  for (int i = tid; i < M * M; i += nt) (&s.Rm[0][0])[i] = double(R_[i]);
  for (int i = tid; i < N; i += nt) s.m0[i] = double(m0_[i]);
  __syncthreads();
  // H Q, H F, F P0, F m0
  for (int i = tid; i < M * N; i += nt) {
    const int a = i / N, b = i % N;
    double q = 0, f = 0;
    for (int t = 0; t < N; ++t) {
      q += s.H[a][t] * s.Q[t][b];
      f += s.H[a][t] * s.F[t][b];
    }
    s.HQ[a][b] = q;
    s.HF[a][b] = f;
  }
  for (int i = tid; i < N * N; i += nt) {
    const int a = i / N, b = i % N;
    double v = 0;
    for (int t = 0; t < N; ++t) v += s.F[a][t] * s.P0[t][b];
    s.FP0[a][b] = v;
  }
  for (int i = tid; i < N; i += nt) {
    double v = 0;
    for (int t = 0; t < N; ++t) v += s.F[i][t] * s.m0[t];
    s.x[i] = v;
  }
  __syncthreads();
  // S = H Q H^T + R, P = F P0 F^T + Q (upper triangles mirrored)
  for (int i = tid; i < M * M; i += nt) {
    const int a = i / M, b = i % M;
    if (b < a) continue;
    double v = s.Rm[a][b];
    for (int t = 0; t < N; ++t) v += s.HQ[a][t] * s.H[b][t];
    s.S[a][b] = s.S[b][a] = v;
  }
  for (int i = tid; i < N * N; i += nt) {
    const int a = i / N, b = i % N;
    if (b < a) continue;
    double v = s.Q[a][b];
    for (int t = 0; t < N; ++t) v += s.FP0[a][t] * s.F[b][t];
    s.P[a][b] = s.P[b][a] = v;
  }
  for (int i = tid; i < M; i += nt) {
    double v = 0;
    for (int t = 0; t < N; ++t) v += s.H[i][t] * s.x[t];
    s.Hx[i] = v;
  }
  __syncthreads();
  // H P, S1 = H P H^T + R
  for (int i = tid; i < M * N; i += nt) {
    const int a = i / N, b = i % N;
    double v = 0;
    for (int t = 0; t < N; ++t) v += s.H[a][t] * s.P[t][b];
    s.HP[a][b] = v;
  }
  __syncthreads();
  for (int i = tid; i < M * M; i += nt) {
    const int a = i / M, b = i % M;
    if (b < a) continue;
    double v = s.Rm[a][b];
    for (int t = 0; t < N; ++t) v += s.HP[a][t] * s.H[b][t];
    s.S1[a][b] = s.S1[b][a] = v;
  }
  for (int i = tid; i < M * N; i += nt) {
    const int a = i / N, b = i % N;
    s.Kt[a][b] = s.HQ[a][b];
    s.Wt[a][b] = s.HF[a][b];
    s.K1t[a][b] = s.HP[a][b];
  }
  __syncthreads();
  // K^T = S^{-1} H Q, W^T = S^{-1} H F, K1^T = S1^{-1} H P (Cholesky, three threads)
  if (tid == 0) chol_solve_shared<M, N>(s.S, s.Kt);
  if (tid == 64) chol_solve_shared<M, N>(s.S, s.Wt);
  if (tid == 128) chol_solve_shared<M, N>(s.S1, s.K1t);
  __syncthreads();
  for (int i = tid; i < N * N; i += nt) {
    const int a = i / N, b = i % N;
    double v = (a == b) ? 1.0 : 0.0;
    for (int t = 0; t < M; ++t) v -= s.Kt[t][a] * s.H[t][b];
    s.IKH[a][b] = v;
  }
  __syncthreads();
  for (int i = tid; i < N * N; i += nt) {
    const int a = i / N, b = i % N;
    double va = 0, vc = 0;
    for (int t = 0; t < N; ++t) {
      va += s.IKH[a][t] * s.F[t][b];
      vc += s.IKH[a][t] * s.Q[t][b];
    }
    s.A[a][b] = va;
    s.C[a][b] = vc;
  }
  __syncthreads();
  for (int i = tid; i < N * N; i += nt) {
    const int a = i / N, b = i % N;
    cst[LY::A + i] = R(s.A[a][b]);
    cst[LY::C + i] = R(0.5 * (s.C[a][b] + s.C[b][a]));
    // J = (S^{-1} H F)^T (H F), upper triangle mirrored
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    double j = 0;
    for (int t = 0; t < M; ++t) j += s.Wt[t][lo] * s.HF[t][hi];
    cst[LY::J + i] = R(j);
    // C_1 = P - (H P)^T S1^{-1} (H P), upper triangle mirrored
    double c1 = s.P[lo][hi];
    for (int t = 0; t < M; ++t) c1 -= s.HP[t][lo] * s.K1t[t][hi];
    cst[LY::C1 + i] = R(c1);
    cst[LY::F + i] = R(s.F[a][b]);
    cst[LY::Q + i] = R(0.5 * (s.Q[a][b] + s.Q[b][a]));
    cst[LY::P0 + i] = R(0.5 * (s.P0[a][b] + s.P0[b][a]));
  }
  for (int i = tid; i < N * M; i += nt) {
    const int a = i / M, t = i % M;
    cst[LY::K + i] = R(s.Kt[t][a]);
    cst[LY::W + i] = R(s.Wt[t][a]);
    cst[LY::K1 + i] = R(s.K1t[t][a]);
  }
  for (int i = tid; i < N; i += nt) {
    double v = s.x[i];
    for (int t = 0; t < M; ++t) v -= s.K1t[t][i] * s.Hx[t];
    cst[LY::c1 + i] = R(v);
    cst[LY::m0 + i] = R(s.m0[i]);
  }
  for (int i = tid; i < M * N; i += nt) cst[LY::H + i] = R((&s.H[0][0])[i]);
  for (int i = tid; i < M * M; i += nt) {
    const int a = i / M, b = i % M;
    cst[LY::Rm + i] = R(0.5 * (s.Rm[a][b] + s.Rm[b][a]));
  }
}

// ---------------------------------------------------------------------------
// Tagged publication of rows (each lane its own row's words).
// ---------------------------------------------------------------------------
template <class R, class E> KF_DEV void tag_publish_row(u64* __restrict__ p, E& x, unsigned tag) {
  each(x, [&](R& v, int k) {
#pragma unroll
    for (int h = 0; h < kWords<R>; ++h)
      st_relaxed(p + k * kWords<R> + h, ((u64)tag << 32) | (u64)half_bits(v, h));
  });
}

// Windowed look-back over groups (the group form of lookback() in
// kf_scan.hpp): group i of the workgroup takes the Gw consecutive tiles
// j-i*Gw-Gw+1 .. j-i*Gw and waits for their status words nearest first; the
// first group (nearest tiles) that meets a published anchored prefix ends
// the search; each group folds its tiles in scan order, the groups of a
// wavefront reduce with a tree over shuffles G lanes apart (higher group =
// earlier), and group 0 folds the wavefront partials (higher wavefront =
// earlier) and the windows right to left, into s_part[NW].  Block-uniform
// control flow; the result (the exclusive prefix of tile t as an element, by
// rows) is valid in group 0.
template <int BLOCK, int G, class E, class Op, class LoadAgg, class Expand>
KF_DEV E glookback(const int* __restrict__ flags, unsigned* err, unsigned tag, long t, int Gw,
                   Op op, LoadAgg load_agg, Expand expand, E (*s_part)[G], int* s_lp, int* s_f1) {
  constexpr int NG = BLOCK / G, GPW = WAVE / G, NW = BLOCK / WAVE;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  const int grp = tid / G, r = tid % G, gw = lane / G;
  if (tid == 0) *s_f1 = lb_wait_flag(flags + (t - 1), tag, err);
  __syncthreads();
  const int f1 = *s_f1;
  __syncthreads();
  if (f1 == LB_PREFIX) {
    E v;
    expand(t - 1, v);
    return v;
  }
  // group 0 accumulates the windows in s_part[NW] (an extra row set), so no
  // accumulator stays in registers from one window to the next
  bool have = false;
  long j = t - 1;
#pragma unroll 1
  while (true) {
    const long hi = j - (long)grp * Gw;  // this group's latest tile
    int gp = Gw;                         // offset of its nearest published prefix
#pragma unroll 1
    for (int q = 0; q < Gw; ++q) {
      const long idx = hi - q;
      if (idx < 0) break;
      if (lb_wait_flag(flags + idx, tag, err) == LB_PREFIX) {
        gp = q;
        break;
      }
    }
    if (r == 0) s_lp[grp] = (gp < Gw) ? 1 : 0;
    __syncthreads();
    int first = NG;  // first group (nearest tiles first) holding a published prefix
#pragma unroll 1
    for (int q = NG - 1; q >= 0; --q)
      if (s_lp[q]) first = q;
    const bool found = first < NG;
    const int last = found ? first : NG - 1;  // last group taking part
    E v;
    set_identity_row(v, r);
    if (grp <= last) {
      const bool anchored = (grp == first);
      int q = anchored ? gp - 1 : Gw - 1;
      if (anchored) expand(hi - gp, v); else load_agg(hi - q--, v);
#pragma unroll 1
      for (; q >= 0; --q) {
        E u;
        load_agg(hi - q, u);
        v = op(v, u);
      }
    }
    const int lw = last - wid * GPW;  // last group of this wavefront taking part
#pragma unroll 1
    for (int s = 1; s <= lw && s < GPW; s <<= 1) {
      E u = shfl_down(v, s * G);
      if ((gw & (2 * s - 1)) == 0 && gw + s <= lw) v = op(u, v);
    }
    if (gw == 0 && lw >= 0) s_part[wid][r] = v;
    __syncthreads();
    if (grp == 0) {
      const int nw = last / GPW + 1;  // wavefronts taking part
      E w = s_part[nw - 1][r];
#pragma unroll 1
      for (int q = nw - 2; q >= 0; --q) w = op(w, s_part[q][r]);
      s_part[NW][r] = have ? op(w, s_part[NW][r]) : w;
    }
    have = true;
    __syncthreads();  // s_part and s_lp are reused by the next window
    if (found) break;
    j -= (long)NG * Gw;
  }
  return s_part[NW][r];
}

// ---------------------------------------------------------------------------
// Tile driver over groups (the group form of scan_tile).  A pipeline supplies
// the same members as for scan_tile, on rows: E (element row), op, fold,
// apply, initial, anchor, expand, steps; bind() also receives the group
// index, the row and the group's scratch.
// ---------------------------------------------------------------------------
template <class Pipe, int N, class R, class S, int BLOCK, int L>
KF_DEV void gscan_tile(Pipe& pp, const ScanArgs<R>& a) {
  using E = typename Pipe::E;
  using Stt = WSt<N, R>;
  constexpr int G = N, NG = BLOCK / G, GPW = WAVE / G, NW = BLOCK / WAVE;
  static_assert(WAVE % G == 0 && BLOCK % WAVE == 0, "groups must tile the wavefronts");
  constexpr int ESW = E::SIZE * kWords<R>;    // tagged words per published element row
  constexpr int PSW = Stt::SIZE * kWords<R>;  // tagged words per published state row
  __shared__ GScr<N, S> s_g[NG];
  __shared__ E s_x[BLOCK];      // each group's inclusive prefix in its wavefront, by lane
  __shared__ E s_wt[NW][N];     // inclusive totals of each wavefront, by row
  __shared__ E s_tot[N];        // the tile aggregate (group 0)
  __shared__ E s_part[NW + 1][N];  // look-back: wavefront partials of a window, accumulator
  __shared__ Stt s_pre[N];      // the tile's exclusive anchored state
  __shared__ int s_lp[NG], s_f1;
  __shared__ long s_tile, s_seq, s_t, s_base;
  __shared__ SeqInfo s_info;
  __shared__ unsigned s_tag;
  const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
  const int grp = tid / G, r = tid % G, gw = lane / G;
  if (tid == 0) {
    // read before the ticket, as in scan_tile: the epoch word changes only
    // when this pass's last workgroup finishes
    const unsigned epoch = ld_relaxed(a.epoch);
    const long g = (long)atomicAdd(a.ctr, 1u);
    s_tile = g;
    s_tag = epoch + 1u;
    SeqInfo si;
    long sq, tt, bs;
    if (a.tile_seq) {
      sq = a.tile_seq[g];
      if (sq >= 0) {
        bs = (long)a.tile_start[sq];
        tt = g - bs;
        si.ntiles = (long)a.tile_start[sq + 1] - bs;
        si.T = (long)a.seq_len[sq];
        si.row0 = (long)a.seq_row[sq];
        si.model = a.cst_stride ? sq : 0;
      } else {
        bs = tt = 0;
        si = SeqInfo{0, 0, 0, 0};
      }
    } else {
      sq = g / a.ntiles;
      tt = g - sq * a.ntiles;
      bs = sq * a.ntiles;
      si = SeqInfo{a.T, a.ntiles, sq * a.T, 0};
    }
    s_seq = sq;
    s_t = tt;
    s_base = bs;
    s_info = si;
  }
  __syncthreads();
  const unsigned tag = s_tag;
  if (s_seq < 0) {
    finish_grid(a.ctr, a.epoch, tag);
    return;
  }
  const long t = uniform(s_t);
  const long base = uniform(s_base);
  const SeqInfo si{uniform(s_info.T), uniform(s_info.ntiles), uniform(s_info.row0),
                   uniform(s_info.model)};
  pp.bind(si, t, grp, r, &s_g[grp]);
  auto op = [&](const E& p, const E& q) { return pp.op(p, q); };

  // 1. group fold; 2. inclusive scan over the groups of each wavefront,
  //    kept in LDS (nothing of it stays in registers through the look-back)
  {
    E x = pp.fold();
#pragma unroll 1
    for (int s = 1; s < GPW; s <<= 1) {
      E u = shfl_up(x, s * G);
      if (gw >= s) x = op(u, x);
    }
    s_x[tid] = x;
    if (gw == GPW - 1) s_wt[wid][r] = x;
  }
  __syncthreads();

  // 3. group 0 publishes the tile aggregate (tile 0: its anchored prefix),
  //    the workgroup looks back, group 0 publishes the anchored prefix
  if (grp == 0) {
    if (t == 0) {
      Stt st;
      pp.initial(st);
#pragma unroll 1
      for (int w = 0; w < NW; ++w) pp.apply(st, s_wt[w][r]);
      tag_publish_row<R>(a.pre + ((base + t) * N + r) * PSW, st, tag);
      if (r == 0) lb_publish_flag(a.flags + base + t, tag, LB_PREFIX);
    } else {
      E tot = s_wt[0][r];
#pragma unroll 1
      for (int w = 1; w < NW; ++w) tot = op(tot, s_wt[w][r]);
      s_tot[r] = tot;
      tag_publish_row<R>(a.agg + ((base + t) * N + r) * ESW, tot, tag);
      if (r == 0) lb_publish_flag(a.flags + base + t, tag, LB_AGG);
    }
  }
  if (t > 0) {
    auto load_agg = [&](long idx, E& v) {
      tag_load<R>(v, a.agg + ((base + idx) * N + r) * ESW, tag, a.ctr + 2);
    };
    auto expand = [&](long idx, E& v) {
      Stt sp;
      tag_load<R>(sp, a.pre + ((base + idx) * N + r) * PSW, tag, a.ctr + 2);
      pp.expand(sp, v);
    };
    // tiles per group in a look-back window: one window reaches back over a
    // sequence of up to 16 * NG tiles
    const long gq = (si.ntiles + NG - 1) / NG;
    const int Gw = (int)(gq < 1 ? 1 : (gq > 16 ? 16 : gq));
    E ex = glookback<BLOCK, G, E>(a.flags + base, a.ctr + 2, tag, t, Gw, op, load_agg, expand,
                                  s_part, s_lp, &s_f1);
    if (grp == 0) {
      Stt st;
      pp.anchor(ex, st);
      s_pre[r] = st;
      pp.apply(st, s_tot[r]);
      tag_publish_row<R>(a.pre + ((base + t) * N + r) * PSW, st, tag);
      if (r == 0) lb_publish_flag(a.flags + base + t, tag, LB_PREFIX);
    }
  }
  __syncthreads();

  // 4. this group's exclusive anchored state: the tile's, then the totals of
  //    the earlier wavefronts, then the earlier groups of this wavefront
  Stt st;
  if (t > 0) st = s_pre[r];
  else pp.initial(st);
#pragma unroll 1
  for (int w = 0; w < wid; ++w) pp.apply(st, s_wt[w][r]);
  if (gw > 0) pp.apply(st, s_x[tid - G]);
  pp.steps(st);
  finish_grid(a.ctr, a.epoch, tag);
}

// ---------------------------------------------------------------------------
// Pipelines
// ---------------------------------------------------------------------------
// Row r of the filtering element of step k (0-based row k) of a time-invariant
// model from the constants of k_wprepare (eqs. pkf_init1..3; reading C4 at k = 0).
template <int N, int M, class R>
KF_DEV WFE<N, R> w_filter_element(const R* __restrict__ cst, long k, const R* __restrict__ yk,
                                  int r) {
  using LY = CL<N, M>;
  WFE<N, R> e;
  const bool first = (k == 0);
  R b = first ? cst[LY::c1 + r] : R(0), h = R(0);
#pragma unroll
  for (int t = 0; t < M; ++t) {
    const R yt = yk[t];
    b += (first ? cst[LY::K1 + r * M + t] : cst[LY::K + r * M + t]) * yt;
    h += cst[LY::W + r * M + t] * yt;
  }
  e.b = b;
  e.e = h;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    e.A[c] = first ? R(0) : cst[LY::A + r * N + c];
    e.C[c] = first ? cst[LY::C1 + r * N + c] : cst[LY::C + r * N + c];
    e.J[c] = cst[LY::J + r * N + c];
  }
  return e;
}

template <int N, int M, class P, int BLOCK, int L> struct WFilterPipe {
  using R = typename P::R;
  using S = typename P::S;
  using E = WFE<N, R>;
  static constexpr int NG = BLOCK / N;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  int r;
  GScr<N, S>* g;
  const R* __restrict__ cst;
  const R* __restrict__ y;
  R* __restrict__ mo;
  R* __restrict__ Po;
  KF_DEV WFilterPipe(const ScanArgs<R>& a_, const IO<R>& io_) : a(a_), io(io_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int grp, int r_, GScr<N, S>* g_) {
    T = s.T;
    r = r_;
    g = g_;
    k0 = t * (long)(L * NG) + (long)grp * L;
    cst = io.cst + s.model * a.cst_stride;
    y = io.y + s.row0 * M;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  KF_DEV E element(long k) const { return w_filter_element<N, M, R>(cst, k, y + k * M, r); }
  KF_DEV E op(const E& p, const E& q) const { return g_fcombine<N, P>(p, q, r, *g); }
  KF_DEV E fold() const {
    E agg;
    set_identity_row(agg, r);
#pragma unroll 1
    for (int i = 0; i < L; ++i) {
      const long k = k0 + i;
      if (k >= T) break;
      const E el = element(k);
      agg = (i == 0) ? el : op(agg, el);
    }
    return agg;
  }
  KF_DEV void apply(WSt<N, R>& st, const E& e) const { g_fapply<N, P>(st, e, r, *g); }
  KF_DEV void initial(WSt<N, R>& st) const { st_zero_row(st); }
  KF_DEV void anchor(const E& e, WSt<N, R>& st) const {
    st.v = e.b;
#pragma unroll
    for (int c = 0; c < N; ++c) st.m[c] = e.C[c];
  }
  KF_DEV void expand(const WSt<N, R>& st, E& v) const {
    set_identity_row(v, r);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      v.A[c] = R(0);
      v.C[c] = st.m[c];
    }
    v.b = st.v;
  }
  KF_DEV void steps(WSt<N, R>& st) const {
#pragma unroll 1
    for (int i = 0; i < L; ++i) {
      const long k = k0 + i;
      if (k >= T) break;
      g_fapply<N, P>(st, element(k), r, *g);
      st_out(&mo[k * N + r], st.v);
#pragma unroll
      for (int c = 0; c < N; ++c) st_out(&Po[(k * N + r) * N + c], st.m[c]);
    }
  }
};

template <int N, int M, class P, int BLOCK, int L> struct WRtsPipe {
  using R = typename P::R;
  using S = typename P::S;
  using E = WSE<N, R>;
  using LY = CL<N, M>;
  static constexpr int NG = BLOCK / N;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  int r;
  GScr<N, S>* g;
  const R* __restrict__ cst;
  const R* __restrict__ mf;
  const R* __restrict__ Pf;
  R* __restrict__ mo;
  R* __restrict__ Po;
  KF_DEV WRtsPipe(const ScanArgs<R>& a_, const IO<R>& io_) : a(a_), io(io_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int grp, int r_, GScr<N, S>* g_) {
    T = s.T;
    r = r_;
    g = g_;
    const long tt = s.ntiles - 1 - t;
    k0 = tt * (long)(L * NG) + (long)(NG - 1 - grp) * L;
    cst = io.cst + s.model * a.cst_stride;
    mf = io.m_in + s.row0 * N;
    Pf = io.P_in + s.row0 * N * N;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  // p precedes q in scan order, so p is the later one in time
  KF_DEV E op(const E& p, const E& q) const { return g_scombine<N, P>(q, p, r, *g); }
  KF_DEV E element(long k) const {
    const R xr = mf[k * N + r];
    R Pr[N];
#pragma unroll
    for (int c = 0; c < N; ++c) Pr[c] = Pf[(k * N + r) * N + c];
    E e;
    if (k == T - 1) {  // eq. prts_init2
#pragma unroll
      for (int c = 0; c < N; ++c) {
        e.E[c] = R(0);
        e.L[c] = Pr[c];
      }
      e.g = xr;
      return e;
    }
    R Fr[N], Qr[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      Fr[c] = cst[LY::F + r * N + c];
      Qr[c] = cst[LY::Q + r * N + c];
    }
    return g_smooth_element<N, P>(xr, Pr, Fr, Qr, r, *g);
  }
  KF_DEV E fold() const {
    E agg;
    set_identity_row(agg, r);
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      if (k < T) agg = op(agg, element(k));
    }
    return agg;
  }
  KF_DEV void apply(WSt<N, R>& st, const E& e) const { g_sapply<N, P>(e, st, r, *g); }
  KF_DEV void initial(WSt<N, R>& st) const { st_zero_row(st); }
  KF_DEV void anchor(const E& e, WSt<N, R>& st) const {
    st.v = e.g;
#pragma unroll
    for (int c = 0; c < N; ++c) st.m[c] = e.L[c];
  }
  KF_DEV void expand(const WSt<N, R>& st, E& v) const {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      v.E[c] = R(0);
      v.L[c] = st.m[c];
    }
    v.g = st.v;
  }
  KF_DEV void steps(WSt<N, R>& st) const {
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      if (k >= T) continue;
      g_sapply<N, P>(element(k), st, r, *g);
      st_out(&mo[k * N + r], st.v);
#pragma unroll
      for (int c = 0; c < N; ++c) st_out(&Po[(k * N + r) * N + c], st.m[c]);
    }
  }
};

// Two-filter backward scan over (a_2, ..., a_T, e): row k holds a_{k+2} (its
// measurement is y at row k+1) and the identity at k = T-1; the anchored
// state is the suffix's (eta, J); the combination with the filter result is
// fused into the steps.
template <int N, int M, class P, int BLOCK, int L> struct WTwoFilterPipe {
  using R = typename P::R;
  using S = typename P::S;
  using E = WFE<N, R>;
  static constexpr int NG = BLOCK / N;
  const ScanArgs<R>& a;
  const IO<R>& io;
  long T, k0;
  int r;
  GScr<N, S>* g;
  const R* __restrict__ cst;
  const R* __restrict__ y;
  const R* __restrict__ mf;
  const R* __restrict__ Pf;
  R* __restrict__ mo;
  R* __restrict__ Po;
  KF_DEV WTwoFilterPipe(const ScanArgs<R>& a_, const IO<R>& io_) : a(a_), io(io_) {}
  KF_DEV void bind(const SeqInfo& s, long t, int grp, int r_, GScr<N, S>* g_) {
    T = s.T;
    r = r_;
    g = g_;
    const long tt = s.ntiles - 1 - t;
    k0 = tt * (long)(L * NG) + (long)(NG - 1 - grp) * L;
    cst = io.cst + s.model * a.cst_stride;
    y = io.y + s.row0 * M;
    mf = io.m_in + s.row0 * N;
    Pf = io.P_in + s.row0 * N * N;
    mo = io.m_out + s.row0 * N;
    Po = io.P_out + s.row0 * N * N;
  }
  KF_DEV E op(const E& p, const E& q) const { return g_fcombine<N, P>(q, p, r, *g); }
  KF_DEV E element(long k) const {
    E e;
    if (k == T - 1) set_identity_row(e, r);
    else e = w_filter_element<N, M, R>(cst, k + 1, y + (k + 1) * M, r);
    return e;
  }
  KF_DEV E fold() const {
    E agg;
    set_identity_row(agg, r);
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      if (k < T) agg = op(agg, element(k));
    }
    return agg;
  }
  KF_DEV void apply(WSt<N, R>& st, const E& e) const { g_fapply_back<N, P>(e, st, r, *g); }
  KF_DEV void initial(WSt<N, R>& st) const { st_zero_row(st); }
  KF_DEV void anchor(const E& e, WSt<N, R>& st) const {
    st.v = e.e;
#pragma unroll
    for (int c = 0; c < N; ++c) st.m[c] = e.J[c];
  }
  // only (eta, J) of an anchored suffix is ever read: it is the right operand
  // of every combine it takes part in
  KF_DEV void expand(const WSt<N, R>& st, E& v) const {
    set_identity_row(v, r);
    v.e = st.v;
#pragma unroll
    for (int c = 0; c < N; ++c) v.J[c] = st.m[c];
  }
  KF_DEV void steps(WSt<N, R>& st) const {
#pragma unroll 1
    for (int i = L - 1; i >= 0; --i) {
      const long k = k0 + i;
      if (k >= T) continue;
      g_fapply_back<N, P>(element(k), st, r, *g);
      const R xr = mf[k * N + r];
      R Pr[N];
#pragma unroll
      for (int c = 0; c < N; ++c) Pr[c] = Pf[(k * N + r) * N + c];
      R xs, Ps[N];
      g_tf_combine<N, P>(xr, Pr, st, r, xs, Ps, *g);
      st_out(&mo[k * N + r], xs);
#pragma unroll
      for (int c = 0; c < N; ++c) st_out(&Po[(k * N + r) * N + c], Ps[c]);
    }
  }
};

template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_wfilter(ScanArgs<typename P::R> a,
                                                   KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  WFilterPipe<N, M, P, BLOCK, L> pp(a, io);
  gscan_tile<WFilterPipe<N, M, P, BLOCK, L>, N, typename P::R, typename P::S, BLOCK, L>(pp, a);
}

template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_wrts(ScanArgs<typename P::R> a,
                                                KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  WRtsPipe<N, M, P, BLOCK, L> pp(a, io);
  gscan_tile<WRtsPipe<N, M, P, BLOCK, L>, N, typename P::R, typename P::S, BLOCK, L>(pp, a);
}

template <int N, int M, class P, int BLOCK, int L>
__global__ __launch_bounds__(BLOCK) void k_wtwofilter(ScanArgs<typename P::R> a,
                                                      KFS_IO_PARAMS(typename P::R)) {
  KFS_IO_MAKE(typename P::R);
  WTwoFilterPipe<N, M, P, BLOCK, L> pp(a, io);
  gscan_tile<WTwoFilterPipe<N, M, P, BLOCK, L>, N, typename P::R, typename P::S, BLOCK, L>(pp,
                                                                                           a);
}

}  // namespace kfs

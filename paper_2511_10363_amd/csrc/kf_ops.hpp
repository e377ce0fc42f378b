// kf_ops.hpp -- the paper's associative elements and operators on gfx950.
//
// Filtering element a = (A, b, C, eta, J)  (Sec. IV-C, eqs. pkf_init1..3)
// Filtering operator                        (Lemma 1)
// Smoothing element a = (E, g, L)           (Sec. IV-D, eqs. prts_init1..2)
// Smoothing operator                        (Lemma 2)
//
// Precision policy P: P::R is the element/storage type, P::S the type of the
// (I + C_i J_j) factorisation, its solves and the assembly of symmetric
// covariance blocks.  For KF_PREC_F32_F64SOLVE, R = float and S = double.
#pragma once
#include "kf_math.hpp"

namespace kfs {

template <class R_, class S_> struct Prec {
  using R = R_;
  using S = S_;
};
using PrecF64 = Prec<double, double>;
using PrecF32 = Prec<float, float>;
using PrecMixed = Prec<float, double>;

template <int N, class R> struct FElem {
  R A[N][N];
  R b[N];
  R C[N][N];
  R e[N];  // eta
  R J[N][N];
  static constexpr int SIZE = 3 * N * N + 2 * N;
};

template <int N, class R> struct SElem {
  R E[N][N];
  R g[N];
  R L[N][N];
  static constexpr int SIZE = 2 * N * N + N;
};

// Visit every scalar of an element in its flat (storage) order.
template <int N, class R, class F> KF_DEV void each(FElem<N, R>& x, F f) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.A[i][j], k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.b[i], k++);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.C[i][j], k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.e[i], k++);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.J[i][j], k++);
}

template <int N, class R, class F> KF_DEV void each(SElem<N, R>& x, F f) {
  int k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.E[i][j], k++);
#pragma unroll
  for (int i = 0; i < N; ++i) f(x.g[i], k++);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) f(x.L[i][j], k++);
}

// An element whose decay matrix (A of a filtering element, E of a smoothing
// element) is exactly zero is an anchor: by Lemma 1 (resp. Lemma 2), whatever
// is combined before it in scan order enters the anchored part of the result
// -- (b, C), (g, L), or (eta, J) in the reversed two-filter scan -- only
// through products with that zero matrix, so those parts equal the
// element's own.  The first filtering element (A_1 = 0, eq. pkf_init2) and the
// last smoothing element (E_T = 0, eq. prts_init2) are anchors by
// construction; long aggregates of a stable model become anchors once their
// decay matrix underflows to zero.
template <int N, class R> KF_DEV bool decay_is_zero(const FElem<N, R>& x) {
  bool z = true;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) z = z & (x.A[i][j] == R(0));
  return z;
}
template <int N, class R> KF_DEV bool decay_is_zero(const SElem<N, R>& x) {
  bool z = true;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) z = z & (x.E[i][j] == R(0));
  return z;
}

// Two-sided identities (I, 0, 0, 0, 0) and (I, 0, 0).
template <int N, class R> KF_DEV void set_identity(FElem<N, R>& x) {
  each(x, [](R& v, int) { v = R(0); });
#pragma unroll
  for (int i = 0; i < N; ++i) x.A[i][i] = R(1);
}
template <int N, class R> KF_DEV void set_identity(SElem<N, R>& x) {
  each(x, [](R& v, int) { v = R(0); });
#pragma unroll
  for (int i = 0; i < N; ++i) x.E[i][i] = R(1);
}

// ---------------------------------------------------------------------------
// Lemma 1.  With M = I + C_i J_j, the transposed factor (I + J_j C_i)^{-1}
// equals M^{-T}, so A_i^T (I + J_j C_i)^{-1} = Z^T with Z = M^{-1} A_i and
// one factorisation with 2N+1 right-hand sides serves all five outputs:
//   A_ij = A_j Z                       b_ij = A_j M^{-1}(b_i + C_i eta_j) + b_j
//   C_ij = A_j (M^{-1} C_i) A_j^T + C_j  eta_ij = Z^T (eta_j - J_j b_i) + eta_i
//   J_ij = Z^T (J_j A_i) + J_i
// ---------------------------------------------------------------------------
template <int N, class P>
KF_DEV FElem<N, typename P::R> fcombine(const FElem<N, typename P::R>& x,
                                        const FElem<N, typename P::R>& y) {
  using R = typename P::R;
  using S = typename P::S;
  S M[N][N];
  mm<N, N, N, S>(x.C, y.J, M);
#pragma unroll
  for (int i = 0; i < N; ++i) M[i][i] += S(1);
  int piv[N];
  S dinv[N];
  lu_factor<N, S>(M, piv, dinv);
  S B[N][2 * N + 1];
#pragma unroll
  for (int r = 0; r < N; ++r) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      B[r][c] = S(x.A[r][c]);
      B[r][N + c] = S(x.C[r][c]);
    }
    S s = S(x.b[r]);
#pragma unroll
    for (int t = 0; t < N; ++t) s += S(x.C[r][t]) * S(y.e[t]);
    B[r][2 * N] = s;
  }
  lu_solve<N, 2 * N + 1, S>(M, piv, dinv, B);
  R Z[N][N], Y[N][N], v[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      Z[r][c] = R(B[r][c]);
      Y[r][c] = R(B[r][N + c]);
    }
    v[r] = R(B[r][2 * N]);
  }
  FElem<N, R> o;
  mm<N, N, N, R>(y.A, Z, o.A);
  R Av[N];
  mv<N, N, R>(y.A, v, Av);
#pragma unroll
  for (int i = 0; i < N; ++i) o.b[i] = Av[i] + y.b[i];
  R AY[N][N];
  mm<N, N, N, R>(y.A, Y, AY);
  sym_xyt_plus<N, N, S>(AY, y.A, y.C, o.C);
  R Jb[N], w[N], Ztw[N];
  mv<N, N, R>(y.J, x.b, Jb);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = y.e[i] - Jb[i];
  mtv<N, N, R>(Z, w, Ztw);
#pragma unroll
  for (int i = 0; i < N; ++i) o.e[i] = Ztw[i] + x.e[i];
  R JA[N][N];
  mm<N, N, N, R>(y.J, x.A, JA);
  sym_xty_plus<N, N, S>(Z, JA, x.J, o.J);
  return o;
}

// Lemma 1 with a left operand whose A is zero (any prefix that starts at
// step 1, since A_1 = 0): only b and C of the result are formed,
//   b' = A_j M^{-1}(x + P eta_j) + b_j,   C' = A_j M^{-1} P A_j^T + C_j,
// M = I + P J_j.  (x, P) is the filtering mean/covariance so far.
template <int N, class P>
KF_DEV void fapply(typename P::R (&x)[N], typename P::R (&Pm)[N][N],
                   const FElem<N, typename P::R>& y) {
  using R = typename P::R;
  using S = typename P::S;
  S M[N][N];
  mm<N, N, N, S>(Pm, y.J, M);
#pragma unroll
  for (int i = 0; i < N; ++i) M[i][i] += S(1);
  int piv[N];
  S dinv[N];
  lu_factor<N, S>(M, piv, dinv);
  S B[N][N + 1];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    S s = S(x[r]);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      B[r][c] = S(Pm[r][c]);
      s += S(Pm[r][c]) * S(y.e[c]);
    }
    B[r][N] = s;
  }
  lu_solve<N, N + 1, S>(M, piv, dinv, B);
  R Y[N][N], v[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
#pragma unroll
    for (int c = 0; c < N; ++c) Y[r][c] = R(B[r][c]);
    v[r] = R(B[r][N]);
  }
  R Av[N];
  mv<N, N, R>(y.A, v, Av);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = Av[i] + y.b[i];
  R AY[N][N];
  mm<N, N, N, R>(y.A, Y, AY);
  sym_xyt_plus<N, N, S>(AY, y.A, y.C, Pm);
}

// Lemma 1 with a right operand that is a suffix of the backward pass, of
// which only (eta_j, J_j) is needed: returns the (eta, J) part of a_i (x) s,
//   eta' = Z^T (eta_j - J_j b_i) + eta_i,   J' = Z^T (J_j A_i) + J_i,
// Z = (I + C_i J_j)^{-1} A_i.  This is the backward information-filter step
// (eqs. tf_vector_pred..tf_matrix_upd) written in element form.
template <int N, class P>
KF_DEV void fapply_back(const FElem<N, typename P::R>& a, typename P::R (&eta)[N],
                        typename P::R (&J)[N][N]) {
  using R = typename P::R;
  using S = typename P::S;
  S M[N][N];
  mm<N, N, N, S>(a.C, J, M);
#pragma unroll
  for (int i = 0; i < N; ++i) M[i][i] += S(1);
  int piv[N];
  S dinv[N];
  lu_factor<N, S>(M, piv, dinv);
  S B[N][N];
  copy_mat<N, N, S>(a.A, B);
  lu_solve<N, N, S>(M, piv, dinv, B);
  R Z[N][N];
  copy_mat<N, N, R>(B, Z);
  R Jb[N], w[N], Ztw[N];
  mv<N, N, R>(J, a.b, Jb);
#pragma unroll
  for (int i = 0; i < N; ++i) w[i] = eta[i] - Jb[i];
  mtv<N, N, R>(Z, w, Ztw);
  R JA[N][N];
  mm<N, N, N, R>(J, a.A, JA);
#pragma unroll
  for (int i = 0; i < N; ++i) eta[i] = Ztw[i] + a.e[i];
  sym_xty_plus<N, N, S>(Z, JA, a.J, J);
}

// ---------------------------------------------------------------------------
// Lemma 2: E_ij = E_i E_j, g_ij = E_i g_j + g_i, L_ij = E_i L_j E_i^T + L_i.
// ---------------------------------------------------------------------------
template <int N, class P>
KF_DEV SElem<N, typename P::R> scombine(const SElem<N, typename P::R>& x,
                                        const SElem<N, typename P::R>& y) {
  using R = typename P::R;
  using S = typename P::S;
  SElem<N, R> o;
  mm<N, N, N, R>(x.E, y.E, o.E);
  R Eg[N];
  mv<N, N, R>(x.E, y.g, Eg);
#pragma unroll
  for (int i = 0; i < N; ++i) o.g[i] = Eg[i] + x.g[i];
  R EL[N][N];
  mm<N, N, N, R>(x.E, y.L, EL);
  sym_xyt_plus<N, N, S>(EL, x.E, x.L, o.L);
  return o;
}

// Lemma 2 with a right operand whose E is zero (any suffix that ends at T,
// since E_T = 0): only (g, L) is formed.  (g, L) is the smoothed
// mean/covariance of the suffix; on return it holds a (x) (0, g, L).
template <int N, class P>
KF_DEV void sapply(const SElem<N, typename P::R>& a, typename P::R (&g)[N],
                   typename P::R (&L)[N][N]) {
  using R = typename P::R;
  using S = typename P::S;
  R Eg[N];
  mv<N, N, R>(a.E, g, Eg);
  R EL[N][N];
  mm<N, N, N, R>(a.E, L, EL);
#pragma unroll
  for (int i = 0; i < N; ++i) g[i] = Eg[i] + a.g[i];
  sym_xyt_plus<N, N, S>(EL, a.E, a.L, L);
}

// Smoothing element of eq. prts_init1 from the filter result (x, P) at step
// k < T:  E = P F^T (F P F^T + Q)^{-1}, g = x - E F x, L = P - E F P.
template <int N, class P, class TF>
KF_DEV SElem<N, typename P::R> smooth_element(const typename P::R (&x)[N],
                                              const typename P::R (&Pm)[N][N],
                                              const TF (&F)[N][N], const TF (&Q)[N][N]) {
  using R = typename P::R;
  using S = typename P::S;
  S FP[N][N];
  mm<N, N, N, S>(F, Pm, FP);
  S Sm[N][N];
  sym_xyt_plus<N, N, S>(FP, F, Q, Sm);  // F P F^T + Q
  S dinv[N];
  chol_factor<N, S>(Sm, dinv);
  S Et[N][N];  // E^T = S^{-1} F P
  copy_mat<N, N, S>(FP, Et);
  chol_solve<N, N, S>(Sm, dinv, Et);
  SElem<N, R> o;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) o.E[i][j] = R(Et[j][i]);
  S Fx[N];
  mv<N, N, S>(F, x, Fx);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S s = S(x[i]);
#pragma unroll
    for (int t = 0; t < N; ++t) s -= Et[t][i] * Fx[t];
    o.g[i] = R(s);
  }
  // L = P - E (F P): symmetric, upper triangle mirrored
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      S s = S(Pm[i][j]);
#pragma unroll
      for (int t = 0; t < N; ++t) s -= Et[t][i] * FP[t][j];
      o.L[i][j] = R(s);
      o.L[j][i] = R(s);
    }
  return o;
}

// Two-filter combination (eqs. mean_tf_combination, cov_tf_combination):
// x_s = (I + P J)^{-1}(x + P eta), P_s = (I + P J)^{-1} P, symmetrised by
// averaging with its transpose.
template <int N, class P, class TE>
KF_DEV void tf_combine(const typename P::R (&x)[N], const typename P::R (&Pm)[N][N],
                       const TE (&eta)[N], const TE (&J)[N][N],
                       typename P::R (&xs)[N], typename P::R (&Ps)[N][N]) {
  using R = typename P::R;
  using S = typename P::S;
  S M[N][N];
  mm<N, N, N, S>(Pm, J, M);
#pragma unroll
  for (int i = 0; i < N; ++i) M[i][i] += S(1);
  int piv[N];
  S dinv[N];
  lu_factor<N, S>(M, piv, dinv);
  S B[N][N + 1];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    S s = S(x[r]);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      B[r][c] = S(Pm[r][c]);
      s += S(Pm[r][c]) * S(eta[c]);
    }
    B[r][N] = s;
  }
  lu_solve<N, N + 1, S>(M, piv, dinv, B);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    xs[r] = R(B[r][N]);
#pragma unroll
    for (int c = r; c < N; ++c) {
      S s = S(0.5) * (B[r][c] + B[c][r]);
      Ps[r][c] = R(s);
      Ps[c][r] = R(s);
    }
  }
}

}  // namespace kfs

namespace kfs {

// ---------------------------------------------------------------------------
// Matrix part (A, C, J) of a filtering element.  Lemma 1 closes over it:
// A_ij, C_ij, J_ij depend only on the matrix parts of the operands, so for a
// time-invariant model the matrix part of an aggregate of j consecutive
// generic elements depends on j alone.
// ---------------------------------------------------------------------------
template <int N, class T> struct MPart {
  T A[N][N];
  T C[N][N];
  T J[N][N];
};

// Orders the LDS accesses of the lanes of one wavefront around this point.
KF_DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Determinant of a K x K matrix (K <= 3) by cofactor expansion.
template <int K, class T> KF_DEV T det_small(const T (&a)[3][3]) {
  if constexpr (K == 0) return T(1);
  else if constexpr (K == 1) return a[0][0];
  else if constexpr (K == 2) return a[0][0] * a[1][1] - a[0][1] * a[1][0];
  else
    return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
           a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
           a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
}

// Cofactor (r, c) of the N x N matrix M (N <= 4): the signed determinant of
// M without row r and column c (rows and columns picked by index, from LDS).
template <int N, class T> KF_DEV T cofactor(const T (&M)[N][N], int r, int c) {
  T a[3][3];
#pragma unroll
  for (int i = 0; i < N - 1; ++i)
#pragma unroll
    for (int j = 0; j < N - 1; ++j) a[i][j] = M[i + (i >= r)][j + (j >= c)];
  const T d = det_small<N - 1, T>(a);
  return ((r + c) & 1) ? -d : d;
}

// Coefficients of the vector part of Lemma 1 for left x (matrix part Sx) and
// right y (matrix part Sy): with M = I + C_x J_y and Z = M^{-1} A_x,
//   b = P1 b_x + P2 eta_y + b_y,   eta = P3 eta_y - P4 b_x + eta_x,
//   P1 = A_y M^{-1}, P2 = P1 C_x, P3 = Z^T, P4 = Z^T J_y.
// The combine also gives the matrix part of x (x) y.
// It is spread over the first N*N lanes of a wavefront, lane
// l = r*N + c owning entry (r, c) of every result; every lane of the
// wavefront must call it (it synchronises the wavefront between phases).
// x, y, o, the coefficients Pc = {P1, P2, P3, P4} and the scratch W live in
// LDS; o must not alias x or y.  M^{-1} is formed from cofactors: lane
// (r, c) forms the cofactor of entry (r, c), every lane the determinant from
// the cofactors of row 0, so the inverse takes a few dependent operations
// per lane instead of a whole pivoted factorisation.  (M has eigenvalues
// >= 1, since C_x and J_y are positive semi-definite, so its determinant is
// >= 1.)  The products then take one dot product per lane.  Symmetric results
// are formed from the upper triangle in both lanes (r, c) and (c, r), so they
// are exactly symmetric.
template <int N, class T>
KF_DEV void mpart_combine_lanes(const MPart<N, T>& x, const MPart<N, T>& y, MPart<N, T>& o,
                                T (&Pc)[4][N][N], T (&W)[4][N][N], int lane) {
  static_assert(N <= 4, "cofactor inverse of at most 4 x 4");
  const bool on = lane < N * N;
  const int r = on ? lane / N : 0, c = on ? lane % N : 0;
  const int i = r < c ? r : c, j = r < c ? c : r;
  if (on) {
    T m = (r == c) ? T(1) : T(0);
#pragma unroll
    for (int t = 0; t < N; ++t) m += x.C[r][t] * y.J[t][c];
    W[0][r][c] = m;
  }
  wave_lds_sync();
  if (on) W[3][r][c] = cofactor<N, T>(W[0], r, c);
  wave_lds_sync();
  if (on) {
    // det(M) by the first row, then with M^{-1} = adj(M) / det(M) and
    // adj(M)[a][b] = cofactor (b, a):  Z = M^{-1} A_x, Y = M^{-1} C_x,
    // P1 = A_y M^{-1}
    T det = T(0);
#pragma unroll
    for (int t = 0; t < N; ++t) det += W[0][0][t] * W[3][0][t];
    const T idet = krcp(det);
    T zr = T(0), yr = T(0), pr = T(0);
#pragma unroll
    for (int t = 0; t < N; ++t) {
      zr += W[3][t][r] * x.A[t][c];
      yr += W[3][t][r] * x.C[t][c];
      pr += y.A[r][t] * W[3][c][t];
    }
    W[1][r][c] = zr * idet;  // Z
    W[2][r][c] = yr * idet;  // Y
    Pc[0][r][c] = pr * idet;
  }
  wave_lds_sync();
  if (on) {
    T p2 = T(0), p4 = T(0), oa = T(0), ay = T(0), ja = T(0);
#pragma unroll
    for (int t = 0; t < N; ++t) {
      p2 += Pc[0][r][t] * x.C[t][c];
      p4 += W[1][t][r] * y.J[t][c];
      oa += y.A[r][t] * W[1][t][c];
      ay += y.A[r][t] * W[2][t][c];
      ja += y.J[r][t] * x.A[t][c];
    }
    Pc[1][r][c] = p2;
    Pc[2][r][c] = W[1][c][r];
    Pc[3][r][c] = p4;
    o.A[r][c] = oa;
    W[0][r][c] = ay;  // A_y Y
    W[3][r][c] = ja;  // J_y A_x
  }
  wave_lds_sync();
  if (on) {
    T oc = y.C[i][j], oj = x.J[i][j];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      oc += W[0][i][t] * y.A[j][t];
      oj += W[1][t][i] * W[3][t][j];
    }
    o.C[r][c] = oc;
    o.J[r][c] = oj;
  }
  wave_lds_sync();
}

// One Kalman predict/update step (Sec. III-A) applied to an anchored state
// (x, P).  By Lemma 1 with a left operand whose A is zero, (0, x, P) (x) a_k for
// the generic element a_k of eq. pkf_init1 is exactly this step, so the
// per-step apply uses it.  S = H P^- H^T + R is factorised (Cholesky) in
// precision P::S; P = P^- - (H P^-)^T S^{-1} (H P^-) is formed symmetric.
template <int N, int M, class P, class TF>
KF_DEV void kf_step(typename P::R (&x)[N], typename P::R (&Pm)[N][N], const TF (&F)[N][N],
                    const TF (&Q)[N][N], const TF (&H)[M][N], const TF (&Rm)[M][M],
                    const typename P::R (&y)[M]) {
  using R = typename P::R;
  using S = typename P::S;
  R xp[N], FP[N][N], Pp[N][N];
  mv<N, N, R>(F, x, xp);
  mm<N, N, N, R>(F, Pm, FP);
  sym_xyt_plus<N, N, R>(FP, F, Q, Pp);
  R HP[M][N];
  mm<M, N, N, R>(H, Pp, HP);
  S Sm[M][M], sd[M];
  sym_xyt_plus<M, N, S>(HP, H, Rm, Sm);
  chol_factor<M, S>(Sm, sd);
  S Kt[M][N + 1];  // [S^{-1} H P^- | S^{-1} (y - H x^-)]
#pragma unroll
  for (int r = 0; r < M; ++r) {
    S s = S(y[r]);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      Kt[r][c] = S(HP[r][c]);
      s -= S(H[r][c]) * S(xp[c]);
    }
    Kt[r][N] = s;
  }
  chol_solve<M, N + 1, S>(Sm, sd, Kt);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S s = S(xp[i]);
#pragma unroll
    for (int t = 0; t < M; ++t) s += S(HP[t][i]) * Kt[t][N];
    x[i] = R(s);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      S s = S(Pp[i][j]);
#pragma unroll
      for (int t = 0; t < M; ++t) s -= S(HP[t][i]) * Kt[t][j];
      Pm[i][j] = R(s);
      Pm[j][i] = R(s);
    }
}

}  // namespace kfs

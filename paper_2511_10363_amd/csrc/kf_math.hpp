// kf_math.hpp -- register-resident small dense linear algebra for gfx950.
//
// Every routine takes compile-time sizes, so fully unrolled loops keep all
// operands in VGPRs.  Row pivots are chosen with compares and selects
// (v_cndmask), never with dynamically indexed registers.
#pragma once
#include <hip/hip_runtime.h>

#define KF_DEV __device__ __forceinline__

namespace kfs {

template <class T> KF_DEV T kabs(T x) { return x < T(0) ? -x : x; }

// Reciprocal and square root used by the factorisations.  FP32: the
// hardware v_rcp_f32 / v_sqrt_f32 (about 1 ulp), FP64: v_rcp_f64 refined by
// two Newton steps (below 1 ulp for normal inputs) and the library sqrt.
KF_DEV float krcp(float x) { return __builtin_amdgcn_rcpf(x); }
KF_DEV double krcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
KF_DEV float ksqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
KF_DEV double ksqrt(double x) { return sqrt(x); }

// In-place LU with partial pivoting, P M = L U (unit-lower L below the
// diagonal, whole rows interchanged).  piv[k] is the row swapped into row k
// at step k; dinv[k] = 1 / U[k][k].
template <int N, class T>
KF_DEV void lu_factor(T (&M)[N][N], int (&piv)[N], T (&dinv)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int p = k;
    T best = kabs(M[k][k]);
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      T a = kabs(M[r][k]);
      bool g = a > best;
      best = g ? a : best;
      p = g ? r : p;
    }
    piv[k] = p;
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      bool s = (p == r);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        T a = M[k][c], b = M[r][c];
        M[k][c] = s ? b : a;
        M[r][c] = s ? a : b;
      }
    }
    T inv = krcp(M[k][k]);
    dinv[k] = inv;
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      T l = M[r][k] * inv;
      M[r][k] = l;
#pragma unroll
      for (int c = k + 1; c < N; ++c) M[r][c] -= l * M[k][c];
    }
  }
}

// Solve M X = B in place (B is N x K) from lu_factor's output.
template <int N, int K, class T>
KF_DEV void lu_solve(const T (&LU)[N][N], const int (&piv)[N], const T (&dinv)[N], T (&B)[N][K]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      bool s = (piv[k] == r);
#pragma unroll
      for (int c = 0; c < K; ++c) {
        T a = B[k][c], b = B[r][c];
        B[k][c] = s ? b : a;
        B[r][c] = s ? a : b;
      }
    }
  }
#pragma unroll
  for (int i = 1; i < N; ++i)
#pragma unroll
    for (int t = 0; t < i; ++t)
#pragma unroll
      for (int c = 0; c < K; ++c) B[i][c] -= LU[i][t] * B[t][c];
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
#pragma unroll
    for (int t = i + 1; t < N; ++t)
#pragma unroll
      for (int c = 0; c < K; ++c) B[i][c] -= LU[i][t] * B[t][c];
#pragma unroll
    for (int c = 0; c < K; ++c) B[i][c] *= dinv[i];
  }
}

// Solve M^T x = b in place from lu_factor's output (P M = L U, so
// M^T = U^T L^T P): U^T w = b forward, L^T v = w backward, x = P^T v.
template <int N, class T>
KF_DEV void lu_solve_t(const T (&LU)[N][N], const int (&piv)[N], const T (&dinv)[N], T (&b)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int t = 0; t < i; ++t) b[i] -= LU[t][i] * b[t];
    b[i] *= dinv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i)
#pragma unroll
    for (int t = i + 1; t < N; ++t) b[i] -= LU[t][i] * b[t];
#pragma unroll
  for (int k = N - 1; k >= 0; --k)
#pragma unroll
    for (int r = k + 1; r < N; ++r) {
      const bool s = (piv[k] == r);
      const T a = b[k], c = b[r];
      b[k] = s ? c : a;
      b[r] = s ? a : c;
    }
}

// In-place Cholesky of a symmetric positive-definite S = L L^T; the lower
// triangle holds L, dinv[j] = 1 / L[j][j].
template <int N, class T>
KF_DEV void chol_factor(T (&S)[N][N], T (&dinv)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T d = S[j][j];
#pragma unroll
    for (int t = 0; t < j; ++t) d -= S[j][t] * S[j][t];
    T l = ksqrt(d);
    T inv = krcp(l);
    S[j][j] = l;
    dinv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T s = S[i][j];
#pragma unroll
      for (int t = 0; t < j; ++t) s -= S[i][t] * S[j][t];
      S[i][j] = s * inv;
    }
  }
}

// Solve (L L^T) X = B in place (B is N x K) from chol_factor's output.
template <int N, int K, class T>
KF_DEV void chol_solve(const T (&L)[N][N], const T (&dinv)[N], T (&B)[N][K]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int t = 0; t < i; ++t)
#pragma unroll
      for (int c = 0; c < K; ++c) B[i][c] -= L[i][t] * B[t][c];
#pragma unroll
    for (int c = 0; c < K; ++c) B[i][c] *= dinv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
#pragma unroll
    for (int t = i + 1; t < N; ++t)
#pragma unroll
      for (int c = 0; c < K; ++c) B[i][c] -= L[t][i] * B[t][c];
#pragma unroll
    for (int c = 0; c < K; ++c) B[i][c] *= dinv[i];
  }
}

// C = A B (A: R x K, B: K x C2), accumulated in type Acc.
template <int R, int K, int C2, class Acc, class TA, class TB>
KF_DEV void mm(const TA (&A)[R][K], const TB (&B)[K][C2], Acc (&C)[R][C2]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < C2; ++j) {
      Acc s = Acc(A[i][0]) * Acc(B[0][j]);
#pragma unroll
      for (int t = 1; t < K; ++t) s += Acc(A[i][t]) * Acc(B[t][j]);
      C[i][j] = s;
    }
}

// y = A x
template <int R, int K, class Acc, class TA, class TX>
KF_DEV void mv(const TA (&A)[R][K], const TX (&x)[K], Acc (&y)[R]) {
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Acc s = Acc(A[i][0]) * Acc(x[0]);
#pragma unroll
    for (int t = 1; t < K; ++t) s += Acc(A[i][t]) * Acc(x[t]);
    y[i] = s;
  }
}

// y = A^T x  (A: K x R)
template <int K, int R, class Acc, class TA, class TX>
KF_DEV void mtv(const TA (&A)[K][R], const TX (&x)[K], Acc (&y)[R]) {
#pragma unroll
  for (int i = 0; i < R; ++i) {
    Acc s = Acc(A[0][i]) * Acc(x[0]);
#pragma unroll
    for (int t = 1; t < K; ++t) s += Acc(A[t][i]) * Acc(x[t]);
    y[i] = s;
  }
}

// S = X Y^T + D for a result known to be symmetric: only the upper triangle
// is formed (in Acc) and mirrored, so S is exactly symmetric.
template <int N, int K, class Acc, class TO, class TX, class TY, class TD>
KF_DEV void sym_xyt_plus(const TX (&X)[N][K], const TY (&Y)[N][K], const TD (&D)[N][N],
                         TO (&S)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      Acc s = Acc(D[i][j]);
#pragma unroll
      for (int t = 0; t < K; ++t) s += Acc(X[i][t]) * Acc(Y[j][t]);
      S[i][j] = TO(s);
      S[j][i] = TO(s);
    }
}

// S = X^T Y + D for a symmetric result (X, Y: K x N), upper triangle mirrored.
template <int N, int K, class Acc, class TO, class TX, class TY, class TD>
KF_DEV void sym_xty_plus(const TX (&X)[K][N], const TY (&Y)[K][N], const TD (&D)[N][N],
                         TO (&S)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      Acc s = Acc(D[i][j]);
#pragma unroll
      for (int t = 0; t < K; ++t) s += Acc(X[t][i]) * Acc(Y[t][j]);
      S[i][j] = TO(s);
      S[j][i] = TO(s);
    }
}

template <int R, int C2, class TO, class TI>
KF_DEV void copy_mat(const TI (&A)[R][C2], TO (&B)[R][C2]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < C2; ++j) B[i][j] = TO(A[i][j]);
}

template <int R, class TO, class TI>
KF_DEV void copy_vec(const TI (&a)[R], TO (&b)[R]) {
#pragma unroll
  for (int i = 0; i < R; ++i) b[i] = TO(a[i]);
}

}  // namespace kfs

/*
 * kf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential FP64 reference for the linear-Gaussian state-space
 * model of Sarkka & Garcia-Fernandez, "On the performance of prefix-sum
 * parallel Kalman filters and smoothers on GPUs" (arXiv 2511.10363).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library; the product path never does.
 * It shares no code, header or table with the GPU library.
 *
 * Two families of routines live here:
 *   1. The textbook sequential recursions (Sec. III): Kalman filter
 *      (eqs. KF_mean_pred..KF_cov_upd), RTS smoother (Sec. III-B, forward-
 *      backward smoother), backward information filter (eqs. tf_vector_pred
 *      ..tf_matrix_upd) and two-filter combination (eqs. mean_tf_combination,
 *      cov_tf_combination).  These are the plain definition of the posterior
 *      moments that every parallel routine must reproduce.
 *   2. The paper's parallel-form building blocks (Sec. IV): filtering
 *      elements (eqs. pkf_init1..pkf_init3), the filtering operator
 *      (Lemma 1), smoothing elements (eqs. prts_init1, prts_init2) and the
 *      smoothing operator (Lemma 2).  Tests fold them sequentially; by
 *      associativity any scan order gives the same result.
 *
 * Conventions (reading C1 of the design notes): the prior is x_{0|0},P_{0|0};
 * step k=1..T predicts with F_{k-1},Q_{k-1},u_{k-1} then updates with y_k,
 * H_k,R_k,d_k.  Outputs for step k are stored at row k-1.  Model arrays are
 * either shared (stride 0) or per step (stride = matrix size); entry j of a
 * per-step F/Q/u array is F_j/Q_j/u_j (j=0..T-1), entry k-1 of a per-step
 * H/R/d array is H_k/R_k/d_k.  u and d may be NULL (zero).
 * All matrices are dense row-major.  Every covariance-like output is
 * symmetrised, (P+P^T)/2, after it is formed (reading C8).
 *
 * Return value: 0 on success, 1 on bad arguments, 2 on a failed
 * factorisation (non-positive Cholesky pivot or zero LU pivot).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KFO_MAXN 64

/* ---------------------------------------------------------------- */
/* small dense helpers (row-major)                                  */
/* ---------------------------------------------------------------- */

/* C(r x c) = A(r x k) * B(k x c) */
static void mat_mul(int r, int k, int c, const double *A, const double *B, double *C)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * c + j];
            C[i * c + j] = s;
        }
}

/* C(r x c) = A(r x k) * B(c x k)^T */
static void mat_mul_bt(int r, int k, int c, const double *A, const double *B, double *C)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += A[i * k + t] * B[j * k + t];
            C[i * c + j] = s;
        }
}

/* C(r x c) = A(k x r)^T * B(k x c) */
static void mat_mul_at(int r, int k, int c, const double *A, const double *B, double *C)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double s = 0.0;
            for (int t = 0; t < k; ++t) s += A[t * r + i] * B[t * c + j];
            C[i * c + j] = s;
        }
}

/* y(r) = A(r x c) x(c) */
static void mat_vec(int r, int c, const double *A, const double *x, double *y)
{
    for (int i = 0; i < r; ++i) {
        double s = 0.0;
        for (int j = 0; j < c; ++j) s += A[i * c + j] * x[j];
        y[i] = s;
    }
}

/* y(c) = A(r x c)^T x(r) */
static void mat_t_vec(int r, int c, const double *A, const double *x, double *y)
{
    for (int j = 0; j < c; ++j) {
        double s = 0.0;
        for (int i = 0; i < r; ++i) s += A[i * c + j] * x[i];
        y[j] = s;
    }
}

static void symmetrise(int n, double *P)
{
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double s = 0.5 * (P[i * n + j] + P[j * n + i]);
            P[i * n + j] = s;
            P[j * n + i] = s;
        }
}

static void identity(int n, double *I)
{
    memset(I, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
}

/* In-place Cholesky S = L L^T (lower triangle of S overwritten with L). */
static int cholesky(int n, double *S)
{
    for (int j = 0; j < n; ++j) {
        double d = S[j * n + j];
        for (int t = 0; t < j; ++t) d -= S[j * n + t] * S[j * n + t];
        if (!(d > 0.0)) return 2;
        double l = sqrt(d);
        S[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double s = S[i * n + j];
            for (int t = 0; t < j; ++t) s -= S[i * n + t] * S[j * n + t];
            S[i * n + j] = s / l;
        }
    }
    return 0;
}

/* Solve (L L^T) X = B in place, B is n x c. */
static void cholesky_solve(int n, int c, const double *L, double *B)
{
    for (int col = 0; col < c; ++col) {
        for (int i = 0; i < n; ++i) {              /* L z = b */
            double s = B[i * c + col];
            for (int t = 0; t < i; ++t) s -= L[i * n + t] * B[t * c + col];
            B[i * c + col] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {         /* L^T x = z */
            double s = B[i * c + col];
            for (int t = i + 1; t < n; ++t) s -= L[t * n + i] * B[t * c + col];
            B[i * c + col] = s / L[i * n + i];
        }
    }
}

/* In-place LU with partial pivoting: P A = L U, unit-lower L below the diagonal. */
static int lu_factor(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return 2;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            double l = A[i * n + k] / A[k * n + k];
            A[i * n + k] = l;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
        }
    }
    return 0;
}

/* Solve A X = B (B n x c, in place) from lu_factor's output. */
static void lu_solve(int n, int c, const double *LU, const int *piv, double *B)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k)
            for (int j = 0; j < c; ++j) {
                double t = B[k * c + j]; B[k * c + j] = B[piv[k] * c + j]; B[piv[k] * c + j] = t;
            }
    for (int col = 0; col < c; ++col) {
        for (int i = 0; i < n; ++i) {
            double s = B[i * c + col];
            for (int t = 0; t < i; ++t) s -= LU[i * n + t] * B[t * c + col];
            B[i * c + col] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = B[i * c + col];
            for (int t = i + 1; t < n; ++t) s -= LU[i * n + t] * B[t * c + col];
            B[i * c + col] = s / LU[i * n + i];
        }
    }
}

/* Solve A^T X = B (B n x c, in place) from lu_factor's output of A. */
static void lu_solve_t(int n, int c, const double *LU, const int *piv, double *B)
{
    for (int col = 0; col < c; ++col) {
        /* U^T z = b */
        for (int i = 0; i < n; ++i) {
            double s = B[i * c + col];
            for (int t = 0; t < i; ++t) s -= LU[t * n + i] * B[t * c + col];
            B[i * c + col] = s / LU[i * n + i];
        }
        /* L^T w = z */
        for (int i = n - 1; i >= 0; --i) {
            double s = B[i * c + col];
            for (int t = i + 1; t < n; ++t) s -= LU[t * n + i] * B[t * c + col];
            B[i * c + col] = s;
        }
    }
    /* x = P^T w : undo the row interchanges in reverse order */
    for (int k = n - 1; k >= 0; --k)
        if (piv[k] != k)
            for (int j = 0; j < c; ++j) {
                double t = B[k * c + j]; B[k * c + j] = B[piv[k] * c + j]; B[piv[k] * c + j] = t;
            }
}

/* Per-step model view. */
typedef struct {
    int nx, ny;
    const double *F, *Q, *H, *R, *u, *d;
    long sF, sQ, sH, sR; /* element strides between steps (0 = shared) */
    int u_step, d_step;  /* 1 if u/d are per step, 0 if shared            */
} model_t;

static const double *mF(const model_t *m, long j) { return m->F + j * m->sF; }
static const double *mQ(const model_t *m, long j) { return m->Q + j * m->sQ; }
static const double *mH(const model_t *m, long k) { return m->H + (k - 1) * m->sH; }
static const double *mR(const model_t *m, long k) { return m->R + (k - 1) * m->sR; }
/* u_j (j = 0..T-1) or NULL */
static const double *mU(const model_t *m, long j)
{
    return m->u ? m->u + (m->u_step ? j * m->nx : 0) : NULL;
}
/* d_k (k = 1..T) or NULL */
static const double *mD(const model_t *m, long k)
{
    return m->d ? m->d + (m->d_step ? (k - 1) * m->ny : 0) : NULL;
}

static int check_dims(int nx, int ny, long T)
{
    return (nx >= 1 && nx <= KFO_MAXN && ny >= 1 && ny <= KFO_MAXN && T >= 1) ? 0 : 1;
}

/* ---------------------------------------------------------------- */
/* 1. Sequential recursions (Sec. III)                              */
/* ---------------------------------------------------------------- */

/*
 * Kalman filter, Sec. III-A: prediction (eq. KF_mean_pred and the P_{k|k-1}
 * line), update (S_k, mean update, eq. KF_cov_upd), for k = 1..T from
 * x_{0|0} = m0, P_{0|0} = P0.  Writes x_{k|k}, P_{k|k} to m_f, P_f and,
 * when non-NULL, x_{k|k-1}, P_{k|k-1} to m_p, P_p (row k-1).
 */
int kfo_filter(int nx, int ny, long T,
               const double *F, long sF, const double *Q, long sQ,
               const double *H, long sH, const double *R, long sR,
               const double *u, int u_step, const double *d, int d_step,
               const double *m0, const double *P0, const double *y,
               double *m_f, double *P_f, double *m_p, double *P_p)
{
    if (check_dims(nx, ny, T)) return 1;
    model_t M = {nx, ny, F, Q, H, R, u, d, sF, sQ, sH, sR, u_step, d_step};
    const int n = nx, m = ny;
    double x[KFO_MAXN], P[KFO_MAXN * KFO_MAXN];
    double xp[KFO_MAXN], Pp[KFO_MAXN * KFO_MAXN], tmp[KFO_MAXN * KFO_MAXN];
    double S[KFO_MAXN * KFO_MAXN], HP[KFO_MAXN * KFO_MAXN], v[KFO_MAXN], w[KFO_MAXN];
    memcpy(x, m0, sizeof(double) * n);
    memcpy(P, P0, sizeof(double) * n * n);
    for (long k = 1; k <= T; ++k) {
        const double *Fk = mF(&M, k - 1), *Qk = mQ(&M, k - 1), *uk = mU(&M, k - 1);
        const double *Hk = mH(&M, k), *Rk = mR(&M, k), *dk = mD(&M, k);
        const double *yk = y + (k - 1) * m;
        /* predict */
        mat_vec(n, n, Fk, x, xp);
        if (uk) for (int i = 0; i < n; ++i) xp[i] += uk[i];
        mat_mul(n, n, n, Fk, P, tmp);
        mat_mul_bt(n, n, n, tmp, Fk, Pp);
        for (int i = 0; i < n * n; ++i) Pp[i] += Qk[i];
        symmetrise(n, Pp);
        if (m_p) memcpy(m_p + (k - 1) * n, xp, sizeof(double) * n);
        if (P_p) memcpy(P_p + (k - 1) * n * n, Pp, sizeof(double) * n * n);
        /* update: S = H Pp H^T + R */
        mat_mul(m, n, n, Hk, Pp, HP);               /* HP = H Pp (m x n) */
        mat_mul_bt(m, n, m, HP, Hk, S);
        for (int i = 0; i < m * m; ++i) S[i] += Rk[i];
        if (cholesky(m, S)) return 2;
        /* innovation v = y - H xp - d */
        mat_vec(m, n, Hk, xp, v);
        for (int i = 0; i < m; ++i) v[i] = yk[i] - v[i] - (dk ? dk[i] : 0.0);
        /* w = S^{-1} v ; x = xp + Pp H^T w = xp + (H Pp)^T w */
        memcpy(w, v, sizeof(double) * m);
        cholesky_solve(m, 1, S, w);
        mat_t_vec(m, n, HP, w, v);
        for (int i = 0; i < n; ++i) x[i] = xp[i] + v[i];
        /* P = Pp - Pp H^T S^{-1} H Pp = Pp - HP^T (S^{-1} HP) */
        memcpy(tmp, HP, sizeof(double) * m * n);
        cholesky_solve(m, n, S, tmp);                /* tmp = S^{-1} H Pp */
        mat_mul_at(n, m, n, HP, tmp, P);             /* P = HP^T tmp      */
        for (int i = 0; i < n * n; ++i) P[i] = Pp[i] - P[i];
        symmetrise(n, P);
        memcpy(m_f + (k - 1) * n, x, sizeof(double) * n);
        memcpy(P_f + (k - 1) * n * n, P, sizeof(double) * n * n);
    }
    return 0;
}

/*
 * RTS smoother, Sec. III-B (forward-backward smoother, linear-Gaussian case):
 * G_k = P_{k|k} F_k^T P_{k+1|k}^{-1}, mean and covariance recursions for
 * k = T-1..1, started from x_{T|T}, P_{T|T}.  Needs the filter's filtered and
 * predicted moments (kfo_filter with m_p, P_p).
 */
int kfo_rts(int nx, long T, const double *F, long sF,
            const double *m_f, const double *P_f, const double *m_p, const double *P_p,
            double *m_s, double *P_s)
{
    if (check_dims(nx, 1, T)) return 1;
    const int n = nx;
    /* an input u_k enters only through the predicted mean m_p */
    double G[KFO_MAXN * KFO_MAXN], L[KFO_MAXN * KFO_MAXN], tmp[KFO_MAXN * KFO_MAXN];
    double D[KFO_MAXN * KFO_MAXN], dv[KFO_MAXN], gv[KFO_MAXN];
    memcpy(m_s + (T - 1) * n, m_f + (T - 1) * n, sizeof(double) * n);
    memcpy(P_s + (T - 1) * n * n, P_f + (T - 1) * n * n, sizeof(double) * n * n);
    for (long k = T - 1; k >= 1; --k) {
        const double *Fk = F + k * sF;                      /* F_k */
        const double *Pf = P_f + (k - 1) * n * n;           /* P_{k|k} */
        const double *Pp1 = P_p + k * n * n;                /* P_{k+1|k} */
        const double *mp1 = m_p + k * n;                    /* x_{k+1|k} */
        /* G^T = P_{k+1|k}^{-1} F_k P_{k|k}  (P_{k+1|k} symmetric positive definite) */
        memcpy(L, Pp1, sizeof(double) * n * n);
        if (cholesky(n, L)) return 2;
        mat_mul(n, n, n, Fk, Pf, tmp);                      /* F P */
        cholesky_solve(n, n, L, tmp);                        /* tmp = G^T */
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) G[i * n + j] = tmp[j * n + i];
        /* mean */
        for (int i = 0; i < n; ++i) dv[i] = m_s[k * n + i] - mp1[i];
        mat_vec(n, n, G, dv, gv);
        for (int i = 0; i < n; ++i) m_s[(k - 1) * n + i] = m_f[(k - 1) * n + i] + gv[i];
        /* covariance */
        for (int i = 0; i < n * n; ++i) D[i] = P_s[k * n * n + i] - Pp1[i];
        mat_mul(n, n, n, G, D, tmp);
        mat_mul_bt(n, n, n, tmp, G, D);
        double *Ps = P_s + (k - 1) * n * n;
        for (int i = 0; i < n * n; ++i) Ps[i] = Pf[i] + D[i];
        symmetrise(n, Ps);
    }
    return 0;
}

/*
 * Backward information filter, Sec. III-B (two-filter smoother): start
 * eta_{T|T:T} = H_T^T R_T^{-1}(y_T - d_T), J_{T|T:T} = H_T^T R_T^{-1} H_T;
 * backward prediction (eq. tf_vector_pred and the J line) and update (through
 * eq. tf_matrix_upd).  Writes the predicted pair eta_{k|k+1:T}, J_{k|k+1:T}
 * for k = 1..T at row k-1; the pair at k = T carries no measurement and is 0.
 */
int kfo_backward_info(int nx, int ny, long T,
                      const double *F, long sF, const double *Q, long sQ,
                      const double *H, long sH, const double *R, long sR,
                      const double *u, int u_step, const double *d, int d_step,
                      const double *y, double *eta_out, double *J_out)
{
    if (check_dims(nx, ny, T)) return 1;
    model_t M = {nx, ny, F, Q, H, R, u, d, sF, sQ, sH, sR, u_step, d_step};
    const int n = nx, m = ny;
    double eta[KFO_MAXN], J[KFO_MAXN * KFO_MAXN];
    double Rl[KFO_MAXN * KFO_MAXN], RiH[KFO_MAXN * KFO_MAXN], Riy[KFO_MAXN];
    double Mi[KFO_MAXN * KFO_MAXN], tmp[KFO_MAXN * KFO_MAXN], tv[KFO_MAXN];
    int piv[KFO_MAXN];

    /* add H_k^T R_k^{-1} (y_k - d_k) and H_k^T R_k^{-1} H_k to (eta, J) */
#define KFO_INFO_UPDATE(k)                                                        \
    do {                                                                          \
        const double *Hk = mH(&M, (k)), *Rk = mR(&M, (k)), *dk = mD(&M, (k));     \
        const double *yk = y + ((k) - 1) * m;                                     \
        memcpy(Rl, Rk, sizeof(double) * m * m);                                   \
        if (cholesky(m, Rl)) return 2;                                            \
        memcpy(RiH, Hk, sizeof(double) * m * n);                                  \
        cholesky_solve(m, n, Rl, RiH);                      /* R^{-1} H */        \
        for (int i = 0; i < m; ++i) Riy[i] = yk[i] - (dk ? dk[i] : 0.0);          \
        cholesky_solve(m, 1, Rl, Riy);                      /* R^{-1}(y-d) */     \
        mat_t_vec(m, n, Hk, Riy, tv);                                             \
        for (int i = 0; i < n; ++i) eta[i] += tv[i];                              \
        mat_mul_at(n, m, n, Hk, RiH, tmp);                                        \
        for (int i = 0; i < n * n; ++i) J[i] += tmp[i];                           \
        symmetrise(n, J);                                                         \
    } while (0)

    memset(eta, 0, sizeof(double) * n);
    memset(J, 0, sizeof(double) * n * n);
    memset(eta_out + (T - 1) * n, 0, sizeof(double) * n);
    memset(J_out + (T - 1) * n * n, 0, sizeof(double) * n * n);
    KFO_INFO_UPDATE(T);
    for (long k = T; k >= 2; --k) {
        const double *Fk1 = mF(&M, k - 1), *Qk1 = mQ(&M, k - 1), *uk1 = mU(&M, k - 1);
        /* Mi = I + J Q_{k-1} */
        mat_mul(n, n, n, J, Qk1, Mi);
        for (int i = 0; i < n; ++i) Mi[i * n + i] += 1.0;
        if (lu_factor(n, Mi, piv)) return 2;
        /* eta_p = F^T Mi^{-1} (eta - J u) */
        memcpy(tv, eta, sizeof(double) * n);
        if (uk1) {
            double Ju[KFO_MAXN];
            mat_vec(n, n, J, uk1, Ju);
            for (int i = 0; i < n; ++i) tv[i] -= Ju[i];
        }
        lu_solve(n, 1, Mi, piv, tv);
        mat_t_vec(n, n, Fk1, tv, eta);
        /* J_p = F^T Mi^{-1} J F */
        mat_mul(n, n, n, J, Fk1, tmp);
        lu_solve(n, n, Mi, piv, tmp);
        mat_mul_at(n, n, n, Fk1, tmp, J);
        symmetrise(n, J);
        memcpy(eta_out + (k - 2) * n, eta, sizeof(double) * n);
        memcpy(J_out + (k - 2) * n * n, J, sizeof(double) * n * n);
        KFO_INFO_UPDATE(k - 1);
    }
#undef KFO_INFO_UPDATE
    return 0;
}

/*
 * Two-filter combination, eqs. mean_tf_combination and cov_tf_combination:
 * x_{k|T} = (I + P_{k|k} J)^{-1}(x_{k|k} + P_{k|k} eta), P_{k|T} = (I + P_{k|k} J)^{-1} P_{k|k}
 * with eta = eta_{k|k+1:T}, J = J_{k|k+1:T}.
 */
int kfo_tf_combine(int nx, long T, const double *m_f, const double *P_f,
                   const double *eta, const double *J, double *m_s, double *P_s)
{
    if (check_dims(nx, 1, T)) return 1;
    const int n = nx;
    double Mi[KFO_MAXN * KFO_MAXN], v[KFO_MAXN];
    int piv[KFO_MAXN];
    for (long k = 0; k < T; ++k) {
        const double *Pf = P_f + k * n * n, *Jk = J + k * n * n;
        mat_mul(n, n, n, Pf, Jk, Mi);
        for (int i = 0; i < n; ++i) Mi[i * n + i] += 1.0;
        if (lu_factor(n, Mi, piv)) return 2;
        mat_vec(n, n, Pf, eta + k * n, v);
        for (int i = 0; i < n; ++i) v[i] += m_f[k * n + i];
        lu_solve(n, 1, Mi, piv, v);
        memcpy(m_s + k * n, v, sizeof(double) * n);
        double *Ps = P_s + k * n * n;
        memcpy(Ps, Pf, sizeof(double) * n * n);
        lu_solve(n, n, Mi, piv, Ps);
        symmetrise(n, Ps);
    }
    return 0;
}

/* ---------------------------------------------------------------- */
/* 2. Parallel-form building blocks (Sec. IV)                       */
/* ---------------------------------------------------------------- */

/*
 * Filtering elements a_k = (A_k, b_k, C_k, eta_k, J_k), k = 1..T, Sec. IV-C:
 * k > 1 by eq. pkf_init1, k = 1 by eq. pkf_init2, (eta_k, J_k) by eq. pkf_init3
 * for every k.  Eq. pkf_init3 names S_k, which for k = 1 is defined twice; the
 * reading taken here (C4) uses S_k = H_k Q_{k-1} H_k^T + R_k for every k, the
 * S of p(y_k | x_{k-1}).  (A_1 = 0 makes eta_1, J_1 irrelevant downstream.)
 * Output layout per k: A [n*n], b [n], C [n*n], eta [n], J [n*n].
 */
int kfo_filter_elements(int nx, int ny, long T,
                        const double *F, long sF, const double *Q, long sQ,
                        const double *H, long sH, const double *R, long sR,
                        const double *u, int u_step, const double *d, int d_step,
                        const double *m0, const double *P0, const double *y,
                        double *A, double *b, double *C, double *eta, double *J)
{
    if (check_dims(nx, ny, T)) return 1;
    model_t M = {nx, ny, F, Q, H, R, u, d, sF, sQ, sH, sR, u_step, d_step};
    const int n = nx, m = ny;
    double S[KFO_MAXN * KFO_MAXN], HQ[KFO_MAXN * KFO_MAXN], Kt[KFO_MAXN * KFO_MAXN];
    double IKH[KFO_MAXN * KFO_MAXN], HF[KFO_MAXN * KFO_MAXN], SiHF[KFO_MAXN * KFO_MAXN];
    double r[KFO_MAXN], Sir[KFO_MAXN], tv[KFO_MAXN], xp[KFO_MAXN], Pp[KFO_MAXN * KFO_MAXN];
    double tmp[KFO_MAXN * KFO_MAXN];
    for (long k = 1; k <= T; ++k) {
        const double *Fk1 = mF(&M, k - 1), *Qk1 = mQ(&M, k - 1), *uk1 = mU(&M, k - 1);
        const double *Hk = mH(&M, k), *Rk = mR(&M, k), *dk = mD(&M, k);
        const double *yk = y + (k - 1) * m;
        double *Ak = A + (k - 1) * n * n, *bk = b + (k - 1) * n, *Ck = C + (k - 1) * n * n;
        double *ek = eta + (k - 1) * n, *Jk = J + (k - 1) * n * n;

        /* S_k = H Q H^T + R (the S of eq. pkf_init1, used by eq. pkf_init3) */
        mat_mul(m, n, n, Hk, Qk1, HQ);
        mat_mul_bt(m, n, m, HQ, Hk, S);
        for (int i = 0; i < m * m; ++i) S[i] += Rk[i];
        if (cholesky(m, S)) return 2;
        /* r = y - H u - d */
        if (uk1) mat_vec(m, n, Hk, uk1, r); else memset(r, 0, sizeof(double) * m);
        for (int i = 0; i < m; ++i) r[i] = yk[i] - r[i] - (dk ? dk[i] : 0.0);
        /* eta_k = F^T H^T S^{-1} r ; J_k = F^T H^T S^{-1} H F */
        mat_mul(m, n, n, Hk, Fk1, HF);
        memcpy(Sir, r, sizeof(double) * m);
        cholesky_solve(m, 1, S, Sir);
        mat_t_vec(m, n, HF, Sir, ek);
        memcpy(SiHF, HF, sizeof(double) * m * n);
        cholesky_solve(m, n, S, SiHF);
        mat_mul_at(n, m, n, HF, SiHF, Jk);
        symmetrise(n, Jk);

        if (k > 1) {
            /* K = Q H^T S^{-1}:  K^T = S^{-1} H Q */
            memcpy(Kt, HQ, sizeof(double) * m * n);
            cholesky_solve(m, n, S, Kt);
            /* IKH = I - K H */
            identity(n, IKH);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double s = 0.0;
                    for (int t = 0; t < m; ++t) s += Kt[t * n + i] * Hk[t * n + j];
                    IKH[i * n + j] -= s;
                }
            mat_mul(n, n, n, IKH, Fk1, Ak);                      /* A = (I-KH)F */
            mat_mul(n, n, n, IKH, Qk1, Ck);                      /* C = (I-KH)Q */
            symmetrise(n, Ck);
            /* b = u + K r */
            mat_t_vec(m, n, Kt, r, tv);
            for (int i = 0; i < n; ++i) bk[i] = (uk1 ? uk1[i] : 0.0) + tv[i];
        } else {
            /* eq. pkf_init2 */
            mat_vec(n, n, Fk1, m0, xp);
            if (uk1) for (int i = 0; i < n; ++i) xp[i] += uk1[i];
            mat_mul(n, n, n, Fk1, P0, tmp);
            mat_mul_bt(n, n, n, tmp, Fk1, Pp);
            for (int i = 0; i < n * n; ++i) Pp[i] += Qk1[i];
            symmetrise(n, Pp);
            double S1[KFO_MAXN * KFO_MAXN], HP[KFO_MAXN * KFO_MAXN], K1t[KFO_MAXN * KFO_MAXN];
            mat_mul(m, n, n, Hk, Pp, HP);
            mat_mul_bt(m, n, m, HP, Hk, S1);
            for (int i = 0; i < m * m; ++i) S1[i] += Rk[i];
            if (cholesky(m, S1)) return 2;
            memcpy(K1t, HP, sizeof(double) * m * n);
            cholesky_solve(m, n, S1, K1t);                      /* K1^T = S1^{-1} H Pp */
            memset(Ak, 0, sizeof(double) * n * n);
            mat_vec(m, n, Hk, xp, r);
            for (int i = 0; i < m; ++i) r[i] = yk[i] - r[i] - (dk ? dk[i] : 0.0);
            mat_t_vec(m, n, K1t, r, tv);
            for (int i = 0; i < n; ++i) bk[i] = xp[i] + tv[i];
            /* C1 = Pp - K1 S1 K1^T = Pp - (H Pp)^T S1^{-1} (H Pp) */
            mat_mul_at(n, m, n, HP, K1t, Ck);
            for (int i = 0; i < n * n; ++i) Ck[i] = Pp[i] - Ck[i];
            symmetrise(n, Ck);
        }
    }
    return 0;
}

/*
 * Filtering operator, Lemma 1: (A_i,b_i,C_i,eta_i,J_i) (x) (A_j,b_j,C_j,eta_j,J_j).
 * Element layout: A [n*n], b [n], C [n*n], eta [n], J [n*n] packed contiguously
 * (size 3n^2 + 2n).  out may alias neither input.
 */
int kfo_filter_combine(int nx, const double *ei, const double *ej, double *out)
{
    if (check_dims(nx, 1, 1)) return 1;
    const int n = nx, nn = n * n;
    const double *Ai = ei, *bi = ei + nn, *Ci = ei + nn + n, *ni = ei + 2 * nn + n, *Ji = ei + 2 * nn + 2 * n;
    const double *Aj = ej, *bj = ej + nn, *Cj = ej + nn + n, *nj = ej + 2 * nn + n, *Jj = ej + 2 * nn + 2 * n;
    double *Ao = out, *bo = out + nn, *Co = out + nn + n, *no = out + 2 * nn + n, *Jo = out + 2 * nn + 2 * n;
    double Mm[KFO_MAXN * KFO_MAXN], X[KFO_MAXN * KFO_MAXN], Y[KFO_MAXN * KFO_MAXN];
    double v[KFO_MAXN], w[KFO_MAXN];
    int piv[KFO_MAXN];
    /* M = I + C_i J_j ; the transposed system gives (I + J_j C_i)^{-1} = M^{-T} */
    mat_mul(n, n, n, Ci, Jj, Mm);
    for (int i = 0; i < n; ++i) Mm[i * n + i] += 1.0;
    if (lu_factor(n, Mm, piv)) return 2;
    /* A_ij = A_j M^{-1} A_i */
    memcpy(X, Ai, sizeof(double) * nn);
    lu_solve(n, n, Mm, piv, X);
    mat_mul(n, n, n, Aj, X, Ao);
    /* b_ij = A_j M^{-1} (b_i + C_i eta_j) + b_j */
    mat_vec(n, n, Ci, nj, v);
    for (int i = 0; i < n; ++i) v[i] += bi[i];
    lu_solve(n, 1, Mm, piv, v);
    mat_vec(n, n, Aj, v, bo);
    for (int i = 0; i < n; ++i) bo[i] += bj[i];
    /* C_ij = A_j M^{-1} C_i A_j^T + C_j */
    memcpy(X, Ci, sizeof(double) * nn);
    lu_solve(n, n, Mm, piv, X);
    mat_mul(n, n, n, Aj, X, Y);
    mat_mul_bt(n, n, n, Y, Aj, Co);
    for (int i = 0; i < nn; ++i) Co[i] += Cj[i];
    symmetrise(n, Co);
    /* eta_ij = A_i^T (I + J_j C_i)^{-1} (eta_j - J_j b_i) + eta_i */
    mat_vec(n, n, Jj, bi, v);
    for (int i = 0; i < n; ++i) w[i] = nj[i] - v[i];
    lu_solve_t(n, 1, Mm, piv, w);
    mat_t_vec(n, n, Ai, w, no);
    for (int i = 0; i < n; ++i) no[i] += ni[i];
    /* J_ij = A_i^T (I + J_j C_i)^{-1} J_j A_i + J_i */
    mat_mul(n, n, n, Jj, Ai, X);
    lu_solve_t(n, n, Mm, piv, X);
    mat_mul_at(n, n, n, Ai, X, Jo);
    for (int i = 0; i < nn; ++i) Jo[i] += Ji[i];
    symmetrise(n, Jo);
    return 0;
}

/*
 * Smoothing elements a_k = (E_k, g_k, L_k), Sec. IV-D: eq. prts_init1 for k < T
 * from the filter output, eq. prts_init2 at k = T.  Layout per k: E [n*n], g [n], L [n*n].
 */
int kfo_smooth_elements(int nx, long T, const double *F, long sF, const double *Q, long sQ,
                        const double *u, int u_step, const double *m_f, const double *P_f,
                        double *E, double *g, double *L)
{
    if (check_dims(nx, 1, T)) return 1;
    const int n = nx, nn = n * n;
    double FP[KFO_MAXN * KFO_MAXN], S[KFO_MAXN * KFO_MAXN], Et[KFO_MAXN * KFO_MAXN], v[KFO_MAXN];
    for (long k = 1; k <= T; ++k) {
        const double *Pk = P_f + (k - 1) * nn, *xk = m_f + (k - 1) * n;
        double *Ek = E + (k - 1) * nn, *gk = g + (k - 1) * n, *Lk = L + (k - 1) * nn;
        if (k == T) {
            memset(Ek, 0, sizeof(double) * nn);
            memcpy(gk, xk, sizeof(double) * n);
            memcpy(Lk, Pk, sizeof(double) * nn);
            continue;
        }
        const double *Fk = F + k * sF, *Qk = Q + k * sQ;
        const double *uk = u ? u + (u_step ? k * n : 0) : NULL;
        /* S = F P F^T + Q ; E = P F^T S^{-1}  <=>  E^T = S^{-1} F P */
        mat_mul(n, n, n, Fk, Pk, FP);
        mat_mul_bt(n, n, n, FP, Fk, S);
        for (int i = 0; i < nn; ++i) S[i] += Qk[i];
        symmetrise(n, S);
        if (cholesky(n, S)) return 2;
        memcpy(Et, FP, sizeof(double) * nn);
        cholesky_solve(n, n, S, Et);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Ek[i * n + j] = Et[j * n + i];
        /* g = x - E (F x + u) */
        mat_vec(n, n, Fk, xk, v);
        if (uk) for (int i = 0; i < n; ++i) v[i] += uk[i];
        mat_vec(n, n, Ek, v, gk);
        for (int i = 0; i < n; ++i) gk[i] = xk[i] - gk[i];
        /* L = P - E F P */
        mat_mul(n, n, n, Ek, FP, Lk);
        for (int i = 0; i < nn; ++i) Lk[i] = Pk[i] - Lk[i];
        symmetrise(n, Lk);
    }
    return 0;
}

/* Smoothing operator, Lemma 2.  Layout E [n*n], g [n], L [n*n]; out aliases no input. */
int kfo_smooth_combine(int nx, const double *ei, const double *ej, double *out)
{
    if (check_dims(nx, 1, 1)) return 1;
    const int n = nx, nn = n * n;
    const double *Ei = ei, *gi = ei + nn, *Li = ei + nn + n;
    const double *Ej = ej, *gj = ej + nn, *Lj = ej + nn + n;
    double *Eo = out, *go = out + nn, *Lo = out + nn + n;
    double X[KFO_MAXN * KFO_MAXN];
    mat_mul(n, n, n, Ei, Ej, Eo);
    mat_vec(n, n, Ei, gj, go);
    for (int i = 0; i < n; ++i) go[i] += gi[i];
    mat_mul(n, n, n, Ei, Lj, X);
    mat_mul_bt(n, n, n, X, Ei, Lo);
    for (int i = 0; i < nn; ++i) Lo[i] += Li[i];
    symmetrise(n, Lo);
    return 0;
}

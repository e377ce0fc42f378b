/*
 * kfscan.h -- C ABI of the MI355X (gfx950) parallel-in-time Kalman filter and
 * smoothers of Sarkka & Garcia-Fernandez, "On the performance of prefix-sum
 * parallel Kalman filters and smoothers on GPUs" (arXiv 2511.10363).
 *
 * Every entry point computes an all-prefix-sum (scan) over the paper's
 * associative elements on the GPU:
 *   kf_filter            Algorithm 5: filtering elements (A, b, C, eta, J) of
 *                        eqs. pkf_init1..pkf_init3, scanned with the operator
 *                        of Lemma 1; x_{k|k} = b_k^+, P_{k|k} = C_k^+.
 *   kf_smooth_rts        Algorithm 6: the filter pass, then smoothing elements
 *                        (E, g, L) of eqs. prts_init1/prts_init2 reverse-scanned
 *                        with the operator of Lemma 2; x_{k|T} = g_k^+, P_{k|T} = L_k^+.
 *   kf_smooth_twofilter  Algorithm 7: the filter pass, a reverse scan of
 *                        (a_2, ..., a_T, e) with the operator of Lemma 1 giving
 *                        eta_{k|k+1:T}, J_{k|k+1:T}, and the two-filter
 *                        combination (eqs. mean_tf_combination, cov_tf_combination).
 *
 * Model (Sec. III-A, eqs. transition_density_Kalman, measurement_density_Kalman,
 * with u = d = 0 and a time-invariant model):
 *   x_k = F x_{k-1} + q,  q ~ N(0, Q);   y_k = H x_k + r,  r ~ N(0, R);
 *   prior x_0 ~ N(m0, P0), i.e. m0 = x_{0|0}, P0 = P_{0|0}.  Step k = 1..T first
 *   predicts from x_{k-1|k-1}, then updates with y_k; results for step k are
 *   stored at row k-1.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller; the
 * library never allocates, frees or retains it.  Storage dtype of every array
 * is float64 for KF_PREC_F64 and float32 for the two other precisions.
 * Layouts are dense row-major:
 *   F, Q, P0 : [nx][nx]      H : [ny][nx]      R : [ny][ny]      m0 : [nx]
 *   y        : [nseq][T][ny]                   (sequences back to back)
 *   m_filt, m_smooth : [nseq][T][nx]
 *   P_filt, P_smooth : [nseq][T][nx][nx]      (exactly symmetric on output)
 * Q, R, P0 must be symmetric positive semi-definite with H Q H^T + R and the
 * predicted covariances positive definite (the smoothers factorise
 * F P_{k|k} F^T + Q).
 *
 * Numerical failures never abort a call.  A breakdown of a factorisation --
 * a non-positive Cholesky pivot of S_k (Sec. III-A) or of F P_{k|k} F^T + Q
 * (eq. prts_init1), a zero pivot of I + C_i J_j (Lemma 1) or of I + P J
 * (eq. cov_tf_combination) -- or a non-finite input makes that sequence's
 * results non-finite; it does not touch the other sequences.  With the
 * optional per-sequence status array (the `status` member of kf_problem,
 * kf_batch and kf_tv_problem, device uint32 [nseq], or NULL), the whole-call
 * entry points finish with a check of every output row: a sequence whose
 * outputs hold a non-finite value gets KF_SEQ_NONFINITE and all its output
 * rows overwritten with NaN; a ragged-batch entry that was skipped as invalid
 * gets KF_SEQ_INVALID (its rows are not touched).  The array is written in
 * full by every such call (no clearing needed) and is read after stream
 * synchronisation; kf_workspace_status then also reports KF_WS_NUMERIC and
 * returns KF_ERR_NUMERIC.  The check reads every output back once (about
 * w (n + n^2) bytes per step per output pair) in three small kernels, which
 * calls without a status array do not run.
 *
 * Workspace: device memory of at least kf_workspace_size() bytes, 256-byte
 * aligned, owned by the caller, with no initialisation required: the first
 * kernel of every call zeroes the workspace's control region (tile tickets,
 * look-back status words and payloads, pass epochs), so one workspace serves
 * any sequence of calls issued in order on one stream, whatever their shapes
 * and precisions.
 * Calls that may run concurrently need distinct workspaces.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Calls are asynchronous: they validate arguments on the host,
 * enqueue kernels and return; the caller synchronises.  No host memory is
 * read or written after return.
 *
 * Errors: argument checks happen on the host before anything is enqueued;
 * on any error nothing is launched and the outputs are untouched.
 */
#ifndef KFSCAN_H
#define KFSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KFSCAN_ABI_VERSION 5

typedef enum kf_status {
    KF_OK = 0,
    KF_ERR_INVALID_ARG = 1,  /* null pointer, bad size, unknown enum value       */
    KF_ERR_UNSUPPORTED = 2,  /* (nx, ny) or precision/scan combination not built */
    KF_ERR_WORKSPACE = 3,    /* workspace too small or misaligned                */
    KF_ERR_DEVICE = 4,       /* the HIP runtime rejected a launch                */
    KF_ERR_NUMERIC = 5       /* kf_workspace_status: a sequence of the last call
                                produced non-finite values (KF_WS_NUMERIC)       */
} kf_status;

/* Bits of the per-sequence status words (kf_problem::status etc.). */
#define KF_SEQ_NONFINITE 1u  /* non-finite output (breakdown or bad input); all rows NaN */
#define KF_SEQ_INVALID 2u    /* ragged batch: T[i] or offset[i] invalid, sequence skipped */

/* Bits reported by kf_workspace_status. */
#define KF_WS_TIMEOUT 1u     /* a look-back wait gave up                                  */
#define KF_WS_INVALID 2u     /* a ragged batch held invalid entries                       */
#define KF_WS_NUMERIC 4u     /* the status check found a sequence with non-finite outputs */

typedef enum kf_precision {
    KF_PREC_F64 = 0,          /* FP64 storage and arithmetic                        */
    KF_PREC_F32 = 1,          /* FP32 storage and arithmetic                        */
    KF_PREC_F32_F64SOLVE = 2  /* FP32 storage and scans; the (I + C_i J_j) and
                                 (I + P J) factorisations and solves, and the
                                 assembly of symmetric covariance blocks, in FP64   */
} kf_precision;

typedef enum kf_scan {
    KF_SCAN_AUTO = 0,             /* library default (KF_SCAN_LOOKBACK)              */
    KF_SCAN_LOOKBACK = 1,         /* single-pass tiled scan with decoupled look-back;
                                     the filtering-element scans use the
                                     time-invariant fold (see below)                 */
    KF_SCAN_BLELLOCH = 2,         /* Algorithm 2, one kernel per tree level          */
    KF_SCAN_HILLIS_STEELE = 3,    /* Algorithm 1, one kernel per doubling level      */
    KF_SCAN_LOOKBACK_GENERIC = 4, /* the look-back scan folding full elements step by
                                     step, with no use of time invariance            */
    KF_SCAN_SEQUENTIAL = 5,       /* no scan: the sequential recursions of Sec. III
                                     (Kalman filter; RTS, or backward information
                                     filter + two-filter combination), one GPU lane
                                     per sequence -- the baseline of the speedup
                                     experiment of Sec. VI.  Plain, batch and
                                     time-varying entry points; its workspace is 256
                                     bytes.  A ragged batch skips only the entries
                                     that are themselves invalid (status bit 1)     */
    KF_SCAN_LADNER_FISCHER = 6,   /* Algorithm 3 (in place), one kernel per level    */
    KF_SCAN_SENGUPTA_A = 7,       /* Algorithm 4 with N = 1, one kernel per level    */
    KF_SCAN_SENGUPTA_B = 8        /* Algorithm 4 with N = 16384 (Hillis-Steele on the
                                     top 16384 positions), one kernel per level     */
} kf_scan;
/* The one-kernel-per-level scans (_BLELLOCH, _HILLIS_STEELE, _LADNER_FISCHER,
 * _SENGUPTA_A, _SENGUPTA_B) keep every element in the workspace (Hillis-
 * Steele and Sengupta need two such arrays) and are offered for kf_problem and
 * kf_tv_problem with nseq <= 65535 and T <= 2^36, not for ragged batches. */

typedef struct kf_problem {
    int32_t nx;            /* state dimension n   (see kf_supported)              */
    int32_t ny;            /* measurement dimension m                             */
    int32_t precision;     /* kf_precision                                        */
    int32_t scan;          /* kf_scan                                             */
    int64_t T;             /* steps per sequence, >= 1                            */
    int64_t nseq;          /* number of sequences sharing the model, >= 1         */
    const void *F, *Q, *H, *R, *m0, *P0;  /* model, device                         */
    const void *y;                         /* measurements, device                  */
    void *m_filt, *P_filt;                 /* filter outputs, device                */
    void *m_smooth, *P_smooth;             /* smoother outputs, device (smoothers)  */
    uint32_t *status;                      /* device [nseq] or NULL (see above)     */
    int32_t items;                         /* 0, or steps per thread of the look-back
                                              scans (2, 4, 8 or 16), see below     */
} kf_problem;

/* A batch of independent sequences of different lengths (Sec. IV applies to
 * each one separately), packed into shared arrays, with one model for all or
 * one model per sequence:
 *   sequence i has T[i] steps; its measurements are rows offset[i] ..
 *   offset[i] + T[i] - 1 of y, and its results the same rows of the outputs.
 * All sequences share nx and ny. */
typedef struct kf_batch {
    int32_t nx;            /* state dimension n                                   */
    int32_t ny;            /* measurement dimension m                             */
    int32_t precision;     /* kf_precision                                        */
    int32_t scan;          /* _AUTO, _LOOKBACK, _LOOKBACK_GENERIC or _SEQUENTIAL  */
    int64_t nseq;          /* number of sequences, 1 .. 2^22                      */
    int64_t nmodels;       /* 1 (shared model) or nseq (model i for sequence i)   */
    int64_t total_steps;   /* rows of y and of the outputs, >= sum of T[i]        */
    const int64_t *T;      /* device [nseq], T[i] >= 1                            */
    const int64_t *offset; /* device [nseq], 0 <= offset[i] <= total_steps - T[i] */
    const void *F, *Q, *H, *R, *m0, *P0;  /* device, [nmodels] models back to back  */
    const void *y;                         /* device [total_steps][ny]               */
    void *m_filt, *P_filt;                 /* device [total_steps][nx], [..][nx][nx] */
    void *m_smooth, *P_smooth;             /* device, smoothers only                 */
    uint32_t *status;                      /* device [nseq] or NULL                  */
    int32_t items;                         /* 0, or steps per thread (see below)     */
} kf_batch;

/* A time-varying model with inputs (Sec. III-A with u, d; the model of the
 * paper's experiments, Sec. VI-A), shared by nseq sequences of T steps.  Row j
 * of the per-step arrays belongs to step j+1 (j = 0 .. T-1):
 *   F, Q [T][nx][nx]   F_j, Q_j: x_{j+1} = F_j x_j + u_j + q_j, q_j ~ N(0, Q_j)
 *   u    [T][nx]       u_j, or NULL for zero inputs
 *   H, R [T][ny][nx], [T][ny][ny]   H_{j+1}, R_{j+1}: y_{j+1} = H x_{j+1} + d + r
 *   d    [T][ny]       d_{j+1}, or NULL for zero offsets
 * The elements are built step by step from these arrays (eqs. pkf_init1..3,
 * prts_init1..2 with u, d).  KF_SCAN_AUTO and _LOOKBACK select the look-back
 * scan over full elements (_LOOKBACK_GENERIC); every other kf_scan is used as
 * asked (the one-kernel-per-level scans with nseq <= 65535). */
typedef struct kf_tv_problem {
    int32_t nx, ny, precision, scan;       /* any kf_scan                       */
    int64_t T;                             /* steps per sequence, >= 1          */
    int64_t nseq;                          /* sequences sharing the model, >= 1 */
    const void *F, *Q, *H, *R, *u, *d;     /* per-step model, device            */
    const void *m0, *P0;                   /* prior x_{0|0}, P_{0|0}, device    */
    const void *y;                         /* [nseq][T][ny], device             */
    void *m_filt, *P_filt;                 /* [nseq][T][nx], [nseq][T][nx][nx]  */
    void *m_smooth, *P_smooth;             /* smoothers only                    */
    uint32_t *status;                      /* device [nseq] or NULL             */
    int32_t items;                         /* 0, or steps per thread (see below) */
} kf_tv_problem;

/* Tile size of the look-back scans (`items` of kf_problem, kf_batch and
 * kf_tv_problem).  A tile is 256 threads (nx <= 4) times `items` steps.  0
 * lets the library choose (the time-invariant filter aims at one tile per
 * CU, the scans over full elements take the longest tiles; a ragged batch
 * always the longest); 2, 4, 8 or 16 asks for that many steps per thread in
 * both scans of the call, capped at the longest each kernel is built for
 * (16 for the time-invariant filter, 16 / 8 / 4 for the full-element scans at
 * nx <= 2 / <= 4 / wider).  The wide-state scans (nx > 4) have one built tile
 * size and ignore it.  Any other value is KF_ERR_INVALID_ARG.  Results do
 * not depend on the tile size beyond rounding; a ragged batch keeps each
 * sequence's results independent of the rest of the batch for any fixed
 * value.  The autotuner of the Python package picks it per workload. */

/* ABI version (KFSCAN_ABI_VERSION). */
int kf_abi_version(void);

/* Static description of a status code (never NULL). */
const char *kf_status_string(kf_status s);

/* 1 if kernels for (nx, ny, precision) are compiled in, else 0. */
int kf_supported(int32_t nx, int32_t ny, int32_t precision);

/* Bytes of workspace that kf_filter / kf_smooth_rts / kf_smooth_twofilter need
 * for this problem (the largest of the three, so one workspace serves all).
 * Only the size fields, precision and scan of *p are read. */
kf_status kf_workspace_size(const kf_problem *p, size_t *bytes);

/* Zero-fill `bytes` of device memory on `stream` with a fill kernel (a
 * convenience; workspaces need no clearing). */
kf_status kf_workspace_clear(void *workspace, size_t bytes, void *stream);

/* Copy `bytes` (a multiple of 16, both pointers 16-byte aligned) from device
 * memory src to device memory dst with one plain streaming kernel (k_copy16):
 * it reads and writes exactly `bytes`, which makes it the reference dispatch
 * for calibrating hardware traffic counters.  Asynchronous on `stream`. */
kf_status kf_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Diagnostic, synchronises `stream`: the error bits of the last call that
 * used this workspace, or-ed over its scans: KF_WS_TIMEOUT, a look-back wait
 * gave up (see kf_workspace_timed_out); KF_WS_INVALID, a ragged batch held a
 * sequence with T[i] < 1 or rows outside [0, total_steps), or lengths adding
 * up to more than total_steps.  Such sequences (all of them in the last case)
 * are skipped: no kernel reads or writes their rows, and their outputs are
 * left as they were; KF_WS_NUMERIC, the call had a status array and some
 * sequence's outputs held a non-finite value.  Returns KF_ERR_NUMERIC (with
 * *status filled) when KF_WS_NUMERIC is set, else KF_OK.  Needs at least the
 * first 32 bytes of the workspace. */
kf_status kf_workspace_status(const void *workspace, size_t workspace_bytes, uint32_t *status,
                              void *stream);

/* Diagnostic, synchronises `stream`: sets *timed_out to 1 if a look-back wait
 * in the last call that used this workspace gave up (a predecessor tile
 * never published within about a second, so that call's outputs are
 * invalid), else 0.  *p must describe that call. */
kf_status kf_workspace_timed_out(const kf_problem *p, const void *workspace,
                                 size_t workspace_bytes, int32_t *timed_out, void *stream);

/* Algorithm 5: writes m_filt, P_filt. */
kf_status kf_filter(const kf_problem *p, void *workspace, size_t workspace_bytes, void *stream);

/* Algorithm 6: writes m_filt, P_filt (the filter pass) and m_smooth, P_smooth. */
kf_status kf_smooth_rts(const kf_problem *p, void *workspace, size_t workspace_bytes,
                        void *stream);

/* Algorithm 7: writes m_filt, P_filt (the forward pass) and m_smooth, P_smooth. */
kf_status kf_smooth_twofilter(const kf_problem *p, void *workspace, size_t workspace_bytes,
                              void *stream);

/* ---- Ragged batches ----------------------------------------------------
 * The same three computations over a kf_batch.  The device arrays T and offset
 * are checked on the device (kf_workspace_status); everything else on the
 * host.  The tiling is chosen from the mean length total_steps / nseq.  The
 * one-kernel-per-level scans are not offered for batches
 * (KF_ERR_UNSUPPORTED).  Sequences whose output rows overlap give undefined
 * results in the overlap. */
kf_status kf_batch_workspace_size(const kf_batch *b, size_t *bytes);
kf_status kf_filter_batch(const kf_batch *b, void *workspace, size_t workspace_bytes,
                          void *stream);
kf_status kf_smooth_rts_batch(const kf_batch *b, void *workspace, size_t workspace_bytes,
                              void *stream);
kf_status kf_smooth_twofilter_batch(const kf_batch *b, void *workspace, size_t workspace_bytes,
                                    void *stream);

/* Instrumentation of the one-kernel-per-level scans: the number of
 * applications of the associative operator (*combines) and of dependent
 * parallel steps that apply it (*steps) in one scan over T elements of one
 * sequence, counted from the same launch plan the scan enqueues (padding
 * positions included).  The work and span of Algorithms 1-4 (Sec. II).
 * KF_ERR_UNSUPPORTED for the other scans, whose work depends on the data
 * (look-back) or which do not scan (sequential). */
kf_status kf_scan_counts(int32_t scan, int64_t T, int64_t *combines, int64_t *steps);

/* ---- Time-varying models ----------------------------------------------- */
kf_status kf_tv_workspace_size(const kf_tv_problem *p, size_t *bytes);
kf_status kf_filter_tv(const kf_tv_problem *p, void *workspace, size_t workspace_bytes,
                       void *stream);
kf_status kf_smooth_rts_tv(const kf_tv_problem *p, void *workspace, size_t workspace_bytes,
                           void *stream);
kf_status kf_smooth_twofilter_tv(const kf_tv_problem *p, void *workspace,
                                 size_t workspace_bytes, void *stream);

/* ---- Stage entry points ------------------------------------------------
 * For callers that schedule or time the passes themselves.  Each enqueues
 * exactly one kernel on `stream`:
 *   kf_prepare        derives the element constants of eqs. pkf_init1..3
 *                     from the model (FP64) into the workspace and zeroes the
 *                     workspace's control words;
 *   kf_pass_filter    the forward scan of Algorithm 5 (writes m_filt, P_filt);
 *   kf_pass_rts       the reverse scan of Algorithm 6 (reads m_filt, P_filt,
 *                     writes m_smooth, P_smooth);
 *   kf_pass_twofilter the backward scan and combination of Algorithm 7 (reads
 *                     y, m_filt, P_filt, writes m_smooth, P_smooth).
 * A pass needs a kf_prepare of the same problem earlier in stream order on
 * the same workspace; each pass advances an epoch word in the workspace that
 * tags everything it publishes, so passes may be repeated after one
 * kf_prepare (up to 2^30 times).
 * kf_filter = kf_prepare + kf_pass_filter;
 * kf_smooth_rts = kf_prepare + kf_pass_filter + kf_pass_rts;
 * kf_smooth_twofilter = kf_prepare + kf_pass_filter + kf_pass_twofilter. */
kf_status kf_prepare(const kf_problem *p, void *workspace, size_t workspace_bytes, void *stream);
kf_status kf_pass_filter(const kf_problem *p, void *workspace, size_t workspace_bytes,
                         void *stream);
kf_status kf_pass_rts(const kf_problem *p, void *workspace, size_t workspace_bytes, void *stream);
kf_status kf_pass_twofilter(const kf_problem *p, void *workspace, size_t workspace_bytes,
                            void *stream);

/* ---- An entry point that allocates nothing ------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * kf_smooth_rts_noalloc is kf_smooth_rts (Algorithm 6, same kernels, same
 * results) with its workspace in a static device array of
 * KF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; it calls no allocating routine.  The caller still
 * passes every input and output array.  A problem whose kf_workspace_size
 * exceeds KF_NOALLOC_SCRATCH_BYTES is refused with KF_ERR_WORKSPACE before
 * anything is enqueued (16 MiB covers the nx = 4 tracking workload up to about
 * T = 2^25 in FP32).  The array is shared by every call on a GPU and keeps the
 * last call's contents (the call re-initialises what it needs): calls that
 * may overlap on one GPU (other streams, other host threads) race and must
 * use kf_smooth_rts with their own workspaces.  `stream` must belong to the
 * current device. */
#define KF_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
kf_status kf_smooth_rts_noalloc(const kf_problem *p, void *stream);

/* ---- Self-test of the scan skeleton ------------------------------------
 * The single-pass look-back drivers of the scans above (fold, wavefront scan,
 * windowed decoupled look-back with anchors, step walk): group = 1 runs the
 * thread driver of the nx <= 4 scans (256 threads x items steps per tile),
 * group = 8 or 16 the group driver of the wide-state scans (groups of that
 * many lanes, 256 / 128 threads, items steps per group), each with an exact,
 * associative, non-commutative operator, so that its all-prefix-sums and
 * reversed all-prefix-sums (Sec. II-B) can be compared bit for bit with a
 * host scan.  An element is the affine map (A, b, C) acting on pairs (v, M)
 * with v in Z_p^2, M in Z_p^{2x2}: v -> A v + b, M -> A M + C, mod p, where
 * p = 33554393 for KF_PREC_F64 (values stored as float64) and p = 2039 for
 * KF_PREC_F32 (float32).
 *   elems  : device [nseq][T][10]: A row-major (4), b (2), C row-major (4),
 *            integers in [0, p); element 0 (forward) or T-1 (reverse) of
 *            each sequence must have A = 0, which anchors every prefix
 *   states : device [nseq][T][6], written: (b, C) of the composed map
 *            forward:  row k = a_1 then a_2 ... then a_{k+1}
 *            reverse:  row k = a_T then a_{T-1} ... then a_{k+1}
 *            (1-based a; the composition of a_i then a_j is
 *             (A_j A_i, A_j b_i + b_j, A_j C_i + C_j))
 * reverse is 0 or 1; items (2, 4, 8 or 16) is the steps per thread of the
 * tiles (256 threads).  Values outside [0, p) give undefined results (never
 * a fault).  The workspace (kf_selftest_scan_workspace bytes, 256-byte
 * aligned) needs no initialisation.  Asynchronous on `stream`. */
kf_status kf_selftest_scan_workspace(int32_t precision, int32_t group, int32_t items, int64_t T,
                                     int64_t nseq, size_t *bytes);
kf_status kf_selftest_scan(int32_t precision, int32_t group, int32_t reverse, int32_t items,
                           int64_t T, int64_t nseq, const void *elems, void *states,
                           void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KFSCAN_H */

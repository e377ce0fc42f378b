// kf_api.hip -- the C-ABI entry points declared in include/kfscan.h.
//
// Host-side only: validate arguments, size and carve the caller's workspace,
// and hand the launches to the per-precision instantiations.  Nothing here
// allocates device memory or synchronises the stream.
#include <cstdint>

#include "kf_inst.hpp"
#include "kf_plan.hpp"

namespace kfs {

__global__ void k_fill_zero(unsigned* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Streaming device copy, 16 bytes per lane per iteration, grid-stride.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Per-sequence numeric status (the optional status array of a call).
//
// k_status_init writes every word: KF_SEQ_INVALID for a ragged-batch entry
// that the scans skipped (the validity rule of k_batch_tiles: 1 <= T[i],
// rows inside [0, total_steps), valid lengths adding up to at most
// total_steps), else 0.  One block when the batch arrays are given, a
// grid-stride fill otherwise.
// k_status_check reads every output value of every valid sequence and raises
// KF_SEQ_NONFINITE on a non-finite one (plus KF_WS_NUMERIC in the workspace's
// error word); k_status_fill then overwrites every output value of such a
// sequence with NaN.  Both walk (sequence, chunk) pairs grid-stride; a
// sequence's values are one contiguous range per output array.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_status_init(const int64_t* __restrict__ len,
                                                       const int64_t* __restrict__ row, long nseq,
                                                       long total_steps,
                                                       uint32_t* __restrict__ status) {
  if (!len) {
    for (long i = blockIdx.x * (long)BLOCK + threadIdx.x; i < nseq; i += (long)gridDim.x * BLOCK)
      status[i] = 0u;
    return;
  }
  __shared__ long long s_sum[BLOCK];
  const int tid = threadIdx.x;
  auto valid = [&](long i) {
    const long T = (long)len[i], r = (long)row[i];
    return T >= 1 && T <= total_steps && r >= 0 && r <= total_steps - T;
  };
  long long part = 0;
  for (long i = tid; i < nseq; i += BLOCK)
    if (valid(i)) part += (long long)len[i];
  s_sum[tid] = part;
  __syncthreads();
  for (int o = BLOCK / 2; o > 0; o >>= 1) {
    if (tid < o) s_sum[tid] += s_sum[tid + o];
    __syncthreads();
  }
  const bool over = s_sum[0] > (long long)total_steps;
  for (long i = tid; i < nseq; i += BLOCK)
    status[i] = (over || !valid(i)) ? KF_SEQ_INVALID : 0u;
}

// Values of sequence q in one output array of `width` scalars per row.
struct SeqRange {
  long begin, count;
};
KF_DEV SeqRange seq_range(const int64_t* __restrict__ len, const int64_t* __restrict__ row,
                          long T, long q, long width) {
  if (len) return SeqRange{(long)row[q] * width, (long)len[q] * width};
  return SeqRange{q * T * width, T * width};
}

template <class R> struct StatusArgs {
  R* out[4];             // m_filt, P_filt, m_smooth, P_smooth (the last two may be null)
  const int64_t* len;    // ragged batch (null for equal-length sequences)
  const int64_t* row;
  long T, nseq, chunks;  // chunks: blocks' worth of work per sequence
  int nx;
  uint32_t* status;
  unsigned* ws_err;
};

template <class R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_status_check(StatusArgs<R> a) {
  const long work = a.nseq * a.chunks;
  for (long b = blockIdx.x; b < work; b += gridDim.x) {
    const long q = b / a.chunks, c = b - q * a.chunks;
    if (a.status[q] & KF_SEQ_INVALID) continue;
    int bad = 0;
#pragma unroll 1
    for (int o = 0; o < 4; ++o) {
      const R* __restrict__ p = a.out[o];
      if (!p) continue;
      const long width = (o & 1) ? (long)a.nx * a.nx : (long)a.nx;
      const SeqRange rg = seq_range(a.len, a.row, a.T, q, width);
      const long per = (rg.count + a.chunks - 1) / a.chunks;
      const long lo = c * per, hi = (lo + per < rg.count) ? lo + per : rg.count;
      for (long i = lo + threadIdx.x; i < hi; i += BLOCK) bad |= !__builtin_isfinite(p[rg.begin + i]);
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) {
      atomicOr(a.status + q, KF_SEQ_NONFINITE);
      atomicOr(a.ws_err, KF_WS_NUMERIC);
    }
  }
}

template <class R, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_status_fill(StatusArgs<R> a) {
  const long work = a.nseq * a.chunks;
  const R nan = __builtin_nan("");
  for (long b = blockIdx.x; b < work; b += gridDim.x) {
    const long q = b / a.chunks, c = b - q * a.chunks;
    if ((a.status[q] & (KF_SEQ_NONFINITE | KF_SEQ_INVALID)) != KF_SEQ_NONFINITE) continue;
#pragma unroll 1
    for (int o = 0; o < 4; ++o) {
      R* __restrict__ p = a.out[o];
      if (!p) continue;
      const long width = (o & 1) ? (long)a.nx * a.nx : (long)a.nx;
      const SeqRange rg = seq_range(a.len, a.row, a.T, q, width);
      const long per = (rg.count + a.chunks - 1) / a.chunks;
      const long lo = c * per, hi = (lo + per < rg.count) ? lo + per : rg.count;
      for (long i = lo + threadIdx.x; i < hi; i += BLOCK) p[rg.begin + i] = nan;
    }
  }
}

template <class R>
static kf_status enqueue_status(Op op, const Job& j, char* ws, const Layout& L, hipStream_t st) {
  constexpr int B = 256;
  const long nseq = j.nseq;
  if (j.batch)
    hipLaunchKernelGGL((k_status_init<1024>), dim3(1), dim3(1024), 0, st, j.len, j.row, nseq,
                       j.total_steps, j.status);
  else
    hipLaunchKernelGGL((k_status_init<B>), dim3((unsigned)((nseq + B - 1) / B < 4096
                                                               ? (nseq + B - 1) / B : 4096)),
                       dim3(B), 0, st, (const int64_t*)nullptr, (const int64_t*)nullptr, nseq,
                       j.total_steps, j.status);
  StatusArgs<R> a{};
  a.out[0] = static_cast<R*>(j.m_filt);
  a.out[1] = static_cast<R*>(j.P_filt);
  if (op != OP_FILTER) {
    a.out[2] = static_cast<R*>(j.m_smooth);
    a.out[3] = static_cast<R*>(j.P_smooth);
  }
  a.len = j.batch ? j.len : nullptr;
  a.row = j.batch ? j.row : nullptr;
  a.T = j.T;
  a.nseq = nseq;
  a.nx = j.nx;
  // about 64K values of one output pair per (sequence, chunk), by the mean length
  const long mean_rows = j.batch ? (j.total_steps + nseq - 1) / nseq : j.T;
  long chunks = (mean_rows * (long)(j.nx + j.nx * j.nx) + 65535) / 65536;
  a.chunks = chunks < 1 ? 1 : (chunks > 4096 ? 4096 : chunks);
  a.status = j.status;
  a.ws_err = reinterpret_cast<unsigned*>(ws + L.ctr[0]) + 2;
  const long work = nseq * a.chunks;
  const dim3 grid((unsigned)(work < 65536 ? work : 65536));
  hipLaunchKernelGGL((k_status_check<R, B>), grid, dim3(B), 0, st, a);
  hipLaunchKernelGGL((k_status_fill<R, B>), grid, dim3(B), 0, st, a);
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

bool wide_shape_built(int nx, int ny) {
#define KFS_TEST(n, m) \
  if (nx == n && ny == m) return true;
  KFS_WIDE_SHAPES(KFS_TEST)
#undef KFS_TEST
  return false;
}

bool shape_built(int nx, int ny) {
#define KFS_TEST(n, m) \
  if (nx == n && ny == m) return true;
  KFS_SHAPES(KFS_TEST)
#undef KFS_TEST
  return wide_shape_built(nx, ny);
}

static kf_status check_common(int nx, int ny, int precision, int scan) {
  if (nx < 1 || ny < 1) return KF_ERR_INVALID_ARG;
  if (precision < KF_PREC_F64 || precision > KF_PREC_F32_F64SOLVE) return KF_ERR_INVALID_ARG;
  if (scan < KF_SCAN_AUTO || scan > KF_SCAN_SENGUPTA_B) return KF_ERR_INVALID_ARG;
  if (!shape_built(nx, ny)) return KF_ERR_UNSUPPORTED;
  // wide states: the look-back scan over full elements only
  if (is_wide(nx) && scan != KF_SCAN_AUTO && scan != KF_SCAN_LOOKBACK &&
      scan != KF_SCAN_LOOKBACK_GENERIC)
    return KF_ERR_UNSUPPORTED;
  return KF_OK;
}

static kf_status check_layout(const Job& j) {
  if (j.items != 0 && j.items != 2 && j.items != 4 && j.items != 8 && j.items != 16)
    return KF_ERR_INVALID_ARG;
  const Layout L = make_layout(j);
  if (L.grid[0] > 2147483647L || L.grid[1] > 2147483647L) return KF_ERR_INVALID_ARG;
  return KF_OK;
}

static kf_status check_sizes(const kf_problem* p) {
  if (!p) return KF_ERR_INVALID_ARG;
  if (p->T < 1 || p->nseq < 1) return KF_ERR_INVALID_ARG;
  // tile counts and element offsets stay well inside 32-bit grid limits
  if (p->T > (int64_t(1) << 40) || p->nseq > (int64_t(1) << 31)) return KF_ERR_INVALID_ARG;
  kf_status s = check_common(p->nx, p->ny, p->precision, p->scan);
  if (s != KF_OK) return s;
  // the tree scans put sequences on the grid's y dimension and positions on x
  if (is_tree_scan(p->scan) && (p->nseq > 65535 || p->T > (int64_t(1) << 36)))
    return KF_ERR_UNSUPPORTED;
  return check_layout(job_of(*p));
}

static kf_status check_batch(const kf_batch* b) {
  if (!b) return KF_ERR_INVALID_ARG;
  if (b->nseq < 1 || b->nseq > (int64_t(1) << 22)) return KF_ERR_INVALID_ARG;
  if (b->nmodels != 1 && b->nmodels != b->nseq) return KF_ERR_INVALID_ARG;
  if (b->total_steps < 1 || b->total_steps > (int64_t(1) << 40)) return KF_ERR_INVALID_ARG;
  kf_status s = check_common(b->nx, b->ny, b->precision, b->scan);
  if (s != KF_OK) return s;
  if (is_tree_scan(b->scan)) return KF_ERR_UNSUPPORTED;
  return check_layout(job_of(*b));
}

static kf_status check_tv(const kf_tv_problem* p) {
  if (!p) return KF_ERR_INVALID_ARG;
  if (p->T < 1 || p->nseq < 1) return KF_ERR_INVALID_ARG;
  if (p->T > (int64_t(1) << 40) || p->nseq > (int64_t(1) << 31)) return KF_ERR_INVALID_ARG;
  kf_status s = check_common(p->nx, p->ny, p->precision, p->scan);
  if (s != KF_OK) return s;
  if (is_wide(p->nx)) return KF_ERR_UNSUPPORTED;
  if (is_tree_scan(p->scan) && (p->nseq > 65535 || p->T > (int64_t(1) << 36)))
    return KF_ERR_UNSUPPORTED;
  return check_layout(job_of(*p));
}

static kf_status run_job(Op op, int stages, const Job& j, void* ws, size_t ws_bytes,
                         void* stream) {
  if ((stages & ST_PREPARE) && (!j.F || !j.Q || !j.H || !j.R || !j.m0 || !j.P0))
    return KF_ERR_INVALID_ARG;
  if ((stages & (ST_FORWARD | ST_BACKWARD)) && (!j.y || !j.m_filt || !j.P_filt))
    return KF_ERR_INVALID_ARG;
  if (op != OP_FILTER && (stages & ST_BACKWARD) && (!j.m_smooth || !j.P_smooth))
    return KF_ERR_INVALID_ARG;
  if (j.batch && (!j.len || !j.row)) return KF_ERR_INVALID_ARG;
  const Layout L = make_layout(j);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L.total)
    return KF_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  kf_status s;
  switch (j.precision) {
    case KF_PREC_F64: s = run_f64(op, stages, j, w, L, st); break;
    case KF_PREC_F32: s = run_f32(op, stages, j, w, L, st); break;
    default: s = run_mixed(op, stages, j, w, L, st); break;
  }
  // the status check follows whole calls only (the stage entry points leave it)
  if (s != KF_OK || !j.status || stages != ST_ALL) return s;
  return j.precision == KF_PREC_F64 ? enqueue_status<double>(op, j, w, L, st)
                                    : enqueue_status<float>(op, j, w, L, st);
}

static kf_status run(Op op, int stages, const kf_problem* p, void* ws, size_t ws_bytes,
                     void* stream) {
  kf_status s = check_sizes(p);
  if (s != KF_OK) return s;
  return run_job(op, stages, job_of(*p), ws, ws_bytes, stream);
}

kf_status run_problem(Op op, const kf_problem* p, void* ws, size_t ws_bytes, void* stream,
                      size_t* ws_needed) {
  kf_status s = check_sizes(p);
  if (s != KF_OK) return s;
  const size_t need = make_layout(job_of(*p)).total;
  if (ws_needed) *ws_needed = need;
  if (ws_bytes < need) return KF_ERR_WORKSPACE;
  return run_job(op, ST_ALL, job_of(*p), ws, ws_bytes, stream);
}

static kf_status run_tv(Op op, const kf_tv_problem* p, void* ws, size_t ws_bytes, void* stream) {
  kf_status s = check_tv(p);
  if (s != KF_OK) return s;
  return run_job(op, ST_ALL, job_of(*p), ws, ws_bytes, stream);
}

static kf_status run_batch(Op op, const kf_batch* b, void* ws, size_t ws_bytes, void* stream) {
  kf_status s = check_batch(b);
  if (s != KF_OK) return s;
  return run_job(op, ST_ALL, job_of(*b), ws, ws_bytes, stream);
}

static kf_status read_error_words(const void* ws, size_t ws_bytes, unsigned (&words)[2],
                                  void* stream) {
  if (!ws || ws_bytes < 8 * sizeof(unsigned)) return KF_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int slot = 0; slot < 2; ++slot) {
    // the control words of scan slot s start at byte 16 s (kf_plan.hpp)
    const char* src = static_cast<const char*>(ws) + 16 * slot + 2 * sizeof(unsigned);
    if (hipMemcpyAsync(&words[slot], src, sizeof(unsigned), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return KF_ERR_DEVICE;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return KF_ERR_DEVICE;
  return KF_OK;
}

}  // namespace kfs

extern "C" {

int kf_abi_version(void) { return KFSCAN_ABI_VERSION; }

const char* kf_status_string(kf_status s) {
  switch (s) {
    case KF_OK: return "ok";
    case KF_ERR_INVALID_ARG: return "invalid argument";
    case KF_ERR_UNSUPPORTED: return "unsupported shape, precision or scan";
    case KF_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case KF_ERR_DEVICE: return "HIP launch failed";
    case KF_ERR_NUMERIC: return "a sequence produced non-finite values";
  }
  return "unknown status";
}

int kf_supported(int32_t nx, int32_t ny, int32_t precision) {
  if (precision < KF_PREC_F64 || precision > KF_PREC_F32_F64SOLVE) return 0;
  return kfs::shape_built(nx, ny) ? 1 : 0;
}

kf_status kf_workspace_size(const kf_problem* p, size_t* bytes) {
  if (!bytes) return KF_ERR_INVALID_ARG;
  kf_status s = kfs::check_sizes(p);
  if (s != KF_OK) return s;
  *bytes = kfs::make_layout(kfs::job_of(*p)).total;
  return KF_OK;
}

kf_status kf_batch_workspace_size(const kf_batch* b, size_t* bytes) {
  if (!bytes) return KF_ERR_INVALID_ARG;
  kf_status s = kfs::check_batch(b);
  if (s != KF_OK) return s;
  *bytes = kfs::make_layout(kfs::job_of(*b)).total;
  return KF_OK;
}

kf_status kf_tv_workspace_size(const kf_tv_problem* p, size_t* bytes) {
  if (!bytes) return KF_ERR_INVALID_ARG;
  kf_status s = kfs::check_tv(p);
  if (s != KF_OK) return s;
  *bytes = kfs::make_layout(kfs::job_of(*p)).total;
  return KF_OK;
}

kf_status kf_scan_counts(int32_t scan, int64_t T, int64_t* combines, int64_t* steps) {
  if (!combines || !steps || T < 1 || T > (int64_t(1) << 40)) return KF_ERR_INVALID_ARG;
  if (scan < KF_SCAN_AUTO || scan > KF_SCAN_SENGUPTA_B) return KF_ERR_INVALID_ARG;
  if (!kfs::is_tree_scan(scan)) return KF_ERR_UNSUPPORTED;
  int64_t c = 0, n = 0;
  for (const kfs::TreeStep& t : kfs::tree_plan(scan, T))
    if (t.threads > 0 && t.combines > 0) {
      c += t.combines;
      ++n;
    }
  *combines = c;
  *steps = n;
  return KF_OK;
}

kf_status kf_filter_tv(const kf_tv_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run_tv(kfs::OP_FILTER, p, ws, ws_bytes, stream);
}

kf_status kf_smooth_rts_tv(const kf_tv_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run_tv(kfs::OP_RTS, p, ws, ws_bytes, stream);
}

kf_status kf_smooth_twofilter_tv(const kf_tv_problem* p, void* ws, size_t ws_bytes,
                                 void* stream) {
  return kfs::run_tv(kfs::OP_TWOFILTER, p, ws, ws_bytes, stream);
}

kf_status kf_workspace_clear(void* workspace, size_t bytes, void* stream) {
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 3u) != 0) return KF_ERR_INVALID_ARG;
  const size_t n = bytes / 4;
  if (n == 0) return KF_OK;
  const unsigned grid = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(kfs::k_fill_zero, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<unsigned*>(workspace), n);
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

kf_status kf_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15u) != 0 || ((reinterpret_cast<uintptr_t>(dst) |
                                             reinterpret_cast<uintptr_t>(src)) & 15u) != 0)
    return KF_ERR_INVALID_ARG;
  const size_t n = bytes / 16;
  if (n == 0) return KF_OK;
  const unsigned grid = (unsigned)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
  hipLaunchKernelGGL(kfs::k_copy16, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  return hipGetLastError() == hipSuccess ? KF_OK : KF_ERR_DEVICE;
}

kf_status kf_workspace_status(const void* ws, size_t ws_bytes, uint32_t* status, void* stream) {
  if (!status) return KF_ERR_INVALID_ARG;
  unsigned words[2] = {0u, 0u};
  kf_status s = kfs::read_error_words(ws, ws_bytes, words, stream);
  if (s != KF_OK) return s;
  *status = words[0] | words[1];
  return (*status & KF_WS_NUMERIC) ? KF_ERR_NUMERIC : KF_OK;
}

kf_status kf_workspace_timed_out(const kf_problem* p, const void* ws, size_t ws_bytes,
                                 int32_t* timed_out, void* stream) {
  if (!timed_out) return KF_ERR_INVALID_ARG;
  kf_status s = kfs::check_sizes(p);
  if (s != KF_OK) return s;
  if (ws_bytes < kfs::make_layout(kfs::job_of(*p)).total) return KF_ERR_WORKSPACE;
  unsigned words[2] = {0u, 0u};
  s = kfs::read_error_words(ws, ws_bytes, words, stream);
  if (s != KF_OK) return s;
  *timed_out = ((words[0] | words[1]) & 1u) ? 1 : 0;
  return KF_OK;
}

kf_status kf_filter_batch(const kf_batch* b, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run_batch(kfs::OP_FILTER, b, ws, ws_bytes, stream);
}

kf_status kf_smooth_rts_batch(const kf_batch* b, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run_batch(kfs::OP_RTS, b, ws, ws_bytes, stream);
}

kf_status kf_smooth_twofilter_batch(const kf_batch* b, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run_batch(kfs::OP_TWOFILTER, b, ws, ws_bytes, stream);
}

kf_status kf_filter(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_FILTER, kfs::ST_ALL, p, ws, ws_bytes, stream);
}

kf_status kf_smooth_rts(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_RTS, kfs::ST_ALL, p, ws, ws_bytes, stream);
}

kf_status kf_smooth_twofilter(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_TWOFILTER, kfs::ST_ALL, p, ws, ws_bytes, stream);
}

kf_status kf_prepare(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_FILTER, kfs::ST_PREPARE, p, ws, ws_bytes, stream);
}

kf_status kf_pass_filter(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_FILTER, kfs::ST_FORWARD, p, ws, ws_bytes, stream);
}

kf_status kf_pass_rts(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_RTS, kfs::ST_BACKWARD, p, ws, ws_bytes, stream);
}

kf_status kf_pass_twofilter(const kf_problem* p, void* ws, size_t ws_bytes, void* stream) {
  return kfs::run(kfs::OP_TWOFILTER, kfs::ST_BACKWARD, p, ws, ws_bytes, stream);
}

}  // extern "C"

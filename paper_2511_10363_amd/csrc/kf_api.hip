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

bool shape_built(int nx, int ny) {
#define KFS_TEST(n, m) \
  if (nx == n && ny == m) return true;
  KFS_SHAPES(KFS_TEST)
#undef KFS_TEST
  return false;
}

static kf_status check_sizes(const kf_problem* p) {
  if (!p) return KF_ERR_INVALID_ARG;
  if (p->nx < 1 || p->ny < 1 || p->T < 1 || p->nseq < 1) return KF_ERR_INVALID_ARG;
  if (p->precision < KF_PREC_F64 || p->precision > KF_PREC_F32_F64SOLVE) return KF_ERR_INVALID_ARG;
  if (p->scan < KF_SCAN_AUTO || p->scan > KF_SCAN_LOOKBACK_GENERIC) return KF_ERR_INVALID_ARG;
  // tile counts and element offsets stay well inside 32-bit grid limits
  if (p->T > (int64_t(1) << 40) || p->nseq > (int64_t(1) << 31)) return KF_ERR_INVALID_ARG;
  if (!shape_built(p->nx, p->ny)) return KF_ERR_UNSUPPORTED;
  // the tree scans put sequences on the grid's y dimension
  if (is_tree_scan(p->scan) && p->nseq > 65535) return KF_ERR_UNSUPPORTED;
  const Layout L = make_layout(p->nx, p->ny, p->precision, p->scan, p->T, p->nseq);
  if ((double)L.ntiles[0] * (double)p->nseq > 2147483647.0 ||
      (double)L.ntiles[1] * (double)p->nseq > 2147483647.0)
    return KF_ERR_INVALID_ARG;
  return KF_OK;
}

static kf_status run(Op op, int stages, const kf_problem* p, void* ws, size_t ws_bytes,
                     void* stream) {
  kf_status s = check_sizes(p);
  if (s != KF_OK) return s;
  if ((stages & ST_PREPARE) && (!p->F || !p->Q || !p->H || !p->R || !p->m0 || !p->P0))
    return KF_ERR_INVALID_ARG;
  if ((stages & (ST_FORWARD | ST_BACKWARD)) && (!p->y || !p->m_filt || !p->P_filt))
    return KF_ERR_INVALID_ARG;
  if (op != OP_FILTER && (stages & ST_BACKWARD) && (!p->m_smooth || !p->P_smooth))
    return KF_ERR_INVALID_ARG;
  const Layout L = make_layout(p->nx, p->ny, p->precision, p->scan, p->T, p->nseq);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0 || ws_bytes < L.total)
    return KF_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  switch (p->precision) {
    case KF_PREC_F64: return run_f64(op, stages, *p, w, L, st);
    case KF_PREC_F32: return run_f32(op, stages, *p, w, L, st);
    default: return run_mixed(op, stages, *p, w, L, st);
  }
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
  *bytes = kfs::make_layout(p->nx, p->ny, p->precision, p->scan, p->T, p->nseq).total;
  return KF_OK;
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

kf_status kf_workspace_timed_out(const kf_problem* p, const void* ws, size_t ws_bytes,
                                 int32_t* timed_out, void* stream) {
  if (!timed_out) return KF_ERR_INVALID_ARG;
  kf_status s = kfs::check_sizes(p);
  if (s != KF_OK) return s;
  const kfs::Layout L = kfs::make_layout(p->nx, p->ny, p->precision, p->scan, p->T, p->nseq);
  if (!ws || ws_bytes < L.total) return KF_ERR_WORKSPACE;
  unsigned words[2] = {0u, 0u};
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int slot = 0; slot < 2; ++slot) {
    const char* src = static_cast<const char*>(ws) + L.ctr[slot] + 2 * sizeof(unsigned);
    if (hipMemcpyAsync(&words[slot], src, sizeof(unsigned), hipMemcpyDeviceToHost, st) != hipSuccess)
      return KF_ERR_DEVICE;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return KF_ERR_DEVICE;
  *timed_out = (words[0] | words[1]) ? 1 : 0;
  return KF_OK;
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

// kf_noalloc.hip -- kf_smooth_rts_noalloc: kf_smooth_rts with its workspace
// in a static device array instead of caller memory, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The array lives in the library's code object: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  In
// host code the array's name is only a host-side handle, so its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept; kernels receive that address, exactly as they
// receive a caller's workspace.  Nothing here allocates, frees or calls an
// allocating routine.
#include <cstdint>
#include <mutex>

#include "kf_plan.hpp"

namespace kfs {

// KF_NOALLOC_SCRATCH_BYTES (16 MiB): the workspace of the tracking workload
// up to about T = 2^25 in FP32 at nx = 4 (kf_workspace_size gives the exact
// need of a problem).
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices];

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, which must be current).
static kf_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices)
    return KF_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KF_ERR_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KF_OK;
}

}  // namespace kfs

extern "C" {

kf_status kf_smooth_rts_noalloc(const kf_problem* p, void* stream) {
  void* ws = nullptr;
  const kf_status s = kfs::scratch_address(&ws);
  if (s != KF_OK) return s;
  return kfs::run_problem(kfs::OP_RTS, p, ws, kfs::kNoAllocScratchBytes, stream, nullptr);
}

}  // extern "C"

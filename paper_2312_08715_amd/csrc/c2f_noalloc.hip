// b3d_c2f_step for callers that cannot allocate device memory: its
// workspace (the stage's hypotheses, their scores, the draws) lives in a
// fixed file-scope device array instead of a caller-provided buffer.
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code it names a host-side stand-in): its device address is taken
// with hipGetSymbolAddress once per device, with that device current, and
// kept in g_scratch.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_internal.hpp"

using namespace b3d_api;

namespace {

__device__ __align__(256) unsigned char scratch[B3D_C2F_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's array (looked up on its first use).
b3d_status scratch_ptr(void** out) {
  int dev = -1;
  B3D_CHECK_HIP(hipGetDevice(&dev), "c2f_step_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(B3D_ENOTSUP, "c2f_step_noalloc: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "c2f_step_noalloc");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return B3D_OK;
}

}  // namespace

extern "C" b3d_status b3d_c2f_step_noalloc(const b3d_scene* scene, const float* center, const b3d_schedule* s,
                                           int32_t K, uint64_t seed, float* weights_out, float* poses_out,
                                           float* logq_out, int32_t* idx_out, void* stream) {
  size_t need = 0;
  if (b3d_status st = b3d_c2f_workspace_size(s, K, &need)) return st;
  if (need > (size_t)B3D_C2F_SCRATCH_BYTES)
    return fail(B3D_ESHAPE, "c2f_step_noalloc: the schedule needs %zu bytes of workspace, above the %zu-byte limit", need,
                (size_t)B3D_C2F_SCRATCH_BYTES);
  void* ws = nullptr;
  if (b3d_status st = scratch_ptr(&ws)) return st;
  // the stage loop writes every workspace word before reading it: nothing to clear
  return b3d_c2f_step(scene, center, s, K, seed, ws, (size_t)B3D_C2F_SCRATCH_BYTES, weights_out, poses_out, logq_out,
                      idx_out, stream);
}

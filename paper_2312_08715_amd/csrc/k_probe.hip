// Microbenchmarks of the chip's peaks, built into their own library
// (libb3d_probe.so) for the benchmark; nothing in libb3d.so uses them.
//
// Peak probe: FP32 vector FMA throughput, for placing the kernels on the
// chip's measured (not only published) VALU roofline.  Every lane runs 8
// independent FMA chains; the result is stored so that nothing is elided.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "b3d_probe.h"

namespace {

__global__ __launch_bounds__(256) void k_probe_fma(float* __restrict__ out, int iters, float a, float b) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = __builtin_fmaf(x[k], a, b);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_probe_fma(float* out, int blocks, int iters, hipStream_t st) {
  hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, st, out, iters, 0.999999f, 1e-7f);
  return hipGetLastError();
}

// Peak probe: HBM bandwidth by a triad c = a + s b over float4s, one pass,
// grid-stride (3 x 16 bytes per element moved).
__global__ __launch_bounds__(256) void k_probe_triad(const float4* __restrict__ a, const float4* __restrict__ b,
                                                     float4* __restrict__ c, long long n, float s) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 x = a[i], y = b[i];
    c[i] = make_float4(x.x + s * y.x, x.y + s * y.y, x.z + s * y.z, x.w + s * y.w);
  }
}

hipError_t launch_probe_triad(const float* a, const float* b, float* c, long long n4, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_probe_triad, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float4*>(a),
                     reinterpret_cast<const float4*>(b), reinterpret_cast<float4*>(c), n4, 1.5f);
  return hipGetLastError();
}

// Peak probe: LDS read bandwidth.  Each lane reads 16-byte words of a 32 KB
// LDS array at addresses that walk the banks without conflicts, iters x 32
// times; the sum is stored so that nothing is elided.
__global__ __launch_bounds__(256) void k_probe_lds(float* __restrict__ out, int iters) {
  __shared__ float4 buf[2048];
  for (int i = threadIdx.x; i < 2048; i += 256) buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  int k = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
      const float4 v = buf[(k + r * 64) & 2047];
      acc.x += v.x;
      acc.y += v.y;
      acc.z += v.z;
      acc.w += v.w;
    }
    k = (k + 7) & 2047;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

hipError_t launch_probe_lds(float* out, int blocks, int iters, hipStream_t st) {
  hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(256), 0, st, out, iters);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int32_t b3d_probe_fma(float* out, int32_t blocks, int32_t iters, void* stream) {
  if (!out || blocks < 1 || iters < 1 || blocks > (1 << 20) || iters > (1 << 20)) return -1;
  return launch_probe_fma(out, blocks, iters, (hipStream_t)stream) == hipSuccess ? 0 : -3;
}

int32_t b3d_probe_hbm(const float* a, const float* b, float* c, int64_t n, void* stream) {
  if (!a || !b || !c || n < 4 || (n % 4) != 0) return -1;
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -3;
  return launch_probe_triad(a, b, c, n / 4, cus * 8, (hipStream_t)stream) == hipSuccess ? 0 : -3;
}

int32_t b3d_probe_lds(float* out, int32_t blocks, int32_t iters, void* stream) {
  if (!out || blocks < 1 || iters < 1 || blocks > (1 << 20) || iters > (1 << 20)) return -1;
  return launch_probe_lds(out, blocks, iters, (hipStream_t)stream) == hipSuccess ? 0 : -3;
}

}  // extern "C"

// Peak probe: FP32 vector FMA throughput, for placing the kernels on the
// chip's measured (not only published) VALU roofline.  Every lane runs 8
// independent FMA chains; the result is stored so that nothing is elided.
#include "b3d_launch.hpp"

namespace b3d {

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

}  // namespace b3d

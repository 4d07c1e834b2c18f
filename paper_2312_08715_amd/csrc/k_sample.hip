// Hypothesis grids, normalisation and Gumbel-max sampling, and the
// coarse-to-fine region update.  Random numbers come from Philox4x32-10
// (Salmon et al., SC'11), a counter-based generator, so a draw depends only
// on (seed, counter) and never on the launch shape.
#include "b3d_launch.hpp"

namespace b3d {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    if (i > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    U4 o;
    o.x = hi1 ^ c.y ^ k0;
    o.y = lo1;
    o.z = hi0 ^ c.w ^ k1;
    o.w = lo0;
    c = o;
  }
  return c;
}

// Odd multiple of 2^-24 from the top 23 bits: exact in binary32, in (0, 1).
__device__ __forceinline__ float to_unit(uint32_t x) { return (float)(2u * (x >> 9) + 1u) * 5.9604644775390625e-8f; }

__device__ void perturbation(uint32_t k0, uint32_t k1, uint32_t stage, int r, float max_angle, float* R) {
  if (r == 0) {
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0f : 0.0f;
    return;
  }
  U4 c = {(uint32_t)r, stage, 0u, 1u};
  const U4 o = philox4x32_10(c, k0, k1);
  const float u0 = to_unit(o.x), u1 = to_unit(o.y), u2 = to_unit(o.z);
  const float z = 1.0f - 2.0f * u0, ph = 6.283185307179586f * u1;
  const float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  const float kx = s * cosf(ph), ky = s * sinf(ph), kz = z;
  const float th = max_angle * u2;
  const float sn = sinf(th), cs = 1.0f - cosf(th);
  // I + sin(th) [k]x + (1 - cos th) [k]x^2, with [k]x^2 = k k^T - I
  R[0] = 1.0f + cs * (kx * kx - 1.0f);
  R[1] = -sn * kz + cs * kx * ky;
  R[2] = sn * ky + cs * kx * kz;
  R[3] = sn * kz + cs * kx * ky;
  R[4] = 1.0f + cs * (ky * ky - 1.0f);
  R[5] = -sn * kx + cs * ky * kz;
  R[6] = -sn * ky + cs * kx * kz;
  R[7] = sn * kx + cs * ky * kz;
  R[8] = 1.0f + cs * (kz * kz - 1.0f);
}

__device__ __forceinline__ float grid_offset(int i, int n, float h, int cell) {
  if (n <= 1) return 0.0f;
  if (cell) return -h + (2.0f * i + 1.0f) * h / (float)n;
  return -h + 2.0f * h * (float)i / (float)(n - 1);
}

// One thread per (segment p, hypothesis n): pose p*N + n.
__global__ void k_enumerate(GridDev g, const float* __restrict__ centres, int P, uint32_t k0, uint32_t k1,
                            uint32_t stage, float* __restrict__ poses) {
  const int nt = g.count[0] * g.count[1] * g.count[2];
  const long long N = (long long)nt * g.n_rot;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= N * P) return;
  const int p = (int)(i / N);
  const int n = (int)(i - (long long)p * N);
  const int r = n / nt, tr = n - r * nt;
  const int ix = tr / (g.count[1] * g.count[2]);
  const int iy = (tr / g.count[2]) % g.count[1];
  const int iz = tr % g.count[2];
  const float* C = centres ? centres + 16 * (size_t)p : g.center;
  float dR[9];
  if (g.rots) {
    for (int k = 0; k < 9; ++k) dR[k] = g.rots[9 * r + k];
  } else {
    perturbation(k0, k1, stage, r, g.max_angle, dR);
  }
  float* out = poses + 16 * (size_t)i;
  const float off[3] = {grid_offset(ix, g.count[0], g.half[0], g.cell_centres),
                        grid_offset(iy, g.count[1], g.half[1], g.cell_centres),
                        grid_offset(iz, g.count[2], g.half[2], g.cell_centres)};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b)
      out[4 * a + b] = dR[3 * a + 0] * C[b] + dR[3 * a + 1] * C[4 + b] + dR[3 * a + 2] * C[8 + b];
    out[4 * a + 3] = C[4 * a + 3] + off[a];
  }
  out[12] = 0.0f;
  out[13] = 0.0f;
  out[14] = 0.0f;
  out[15] = 1.0f;
}

hipError_t launch_enumerate(const GridDev& g, const float* centres, int P, uint32_t key0, uint32_t key1,
                            uint32_t stage, float* poses, hipStream_t st) {
  const long long N = (long long)g.count[0] * g.count[1] * g.count[2] * g.n_rot * P;
  const int blocks = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_enumerate, dim3(blocks), dim3(256), 0, st, g, centres, P, key0, key1, stage, poses);
  return hipGetLastError();
}

// Block (p, k): logsumexp of segment p and its draw k by Gumbel-max.
__global__ __launch_bounds__(kBlock) void k_sample(const float* __restrict__ logL, int P, int N, int K, uint32_t k0,
                                                   uint32_t k1, uint32_t stage, uint32_t kbase, float* __restrict__ w,
                                                   int* __restrict__ idx, float* __restrict__ logw) {
  __shared__ float rv[kWaves];
  __shared__ int ri[kWaves];
  __shared__ float red[kWaves];
  const int blk = blockIdx.x;
  const int p = blk / K, k = blk - p * K;
  const float* L = logL + (size_t)p * N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // max
  float m = -INFINITY;
  for (int n = threadIdx.x; n < N; n += kBlock) m = fmaxf(m, L[n]);
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wave] = m;
  __syncthreads();
  m = red[0];
  for (int i = 1; i < kWaves; ++i) m = fmaxf(m, red[i]);
  __syncthreads();
  // sum of exp(l - m), fixed order
  float s = 0.0f;
  for (int n = threadIdx.x; n < N; n += kBlock) s += expf(L[n] - m);
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  s = red[0];
  for (int i = 1; i < kWaves; ++i) s += red[i];
  const float lse = m + logf(s);
  if (k == 0 && w)
    for (int n = threadIdx.x; n < N; n += kBlock) w[(size_t)p * N + n] = expf(L[n] - lse);
  // argmax of l + G, ties to the lowest index
  const uint32_t draw = kbase + (uint32_t)(p * K + k);
  float bv = -INFINITY;
  int bi = -1;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    U4 c = {(uint32_t)n, draw, stage, 0u};
    const float u = to_unit(philox4x32_10(c, k0, k1).x);
    const float v = L[n] - logf(-logf(u));
    if (bi < 0 || v > bv) {
      bv = v;
      bi = n;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (oi >= 0 && (bi < 0 || ov > bv || (ov == bv && oi < bi))) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    rv[wave] = bv;
    ri[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bv = rv[0];
    bi = ri[0];
    for (int i = 1; i < kWaves; ++i)
      if (ri[i] >= 0 && (bi < 0 || rv[i] > bv || (rv[i] == bv && ri[i] < bi))) {
        bv = rv[i];
        bi = ri[i];
      }
    idx[(size_t)p * K + k] = bi;
    if (logw) logw[(size_t)p * K + k] = L[bi] - lse;
  }
}

hipError_t launch_sample(const float* logL, int P, int N, int K, uint32_t key0, uint32_t key1, uint32_t stage,
                         uint32_t k0, float* w, int* idx, float* logw, hipStream_t st) {
  hipLaunchKernelGGL(k_sample, dim3(P * K), dim3(kBlock), 0, st, logL, P, N, K, key0, key1, stage, k0, w, idx, logw);
  return hipGetLastError();
}

// After a stage: particle k moves to its drawn cell.  Stage 0 (accumulate =
// 0): one segment with K draws, centre k = poses[idx[k]], logq = logw.
// Later stages: K segments with one draw each, centre k = poses[k N +
// idx[k]], logq += logw.
__global__ void k_c2f_update(const float* __restrict__ poses, int P, int N, const int* __restrict__ idx,
                             const float* __restrict__ logw, int K, int accumulate, float* __restrict__ centres,
                             float* __restrict__ logq, int* __restrict__ idx_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int i = idx[k];
  const size_t src = (P == 1) ? (size_t)i : (size_t)k * N + i;
  for (int e = 0; e < 16; ++e) centres[16 * (size_t)k + e] = poses[16 * src + e];
  logq[k] = accumulate ? logq[k] + logw[k] : logw[k];
  if (idx_out) idx_out[k] = i;
}

hipError_t launch_c2f_update(const float* poses, int P, int N, const int* idx, const float* logw, int K, int accumulate,
                             float* centres, float* logq, int* idx_out, hipStream_t st) {
  hipLaunchKernelGGL(k_c2f_update, dim3((K + 63) / 64), dim3(64), 0, st, poses, P, N, idx, logw, K, accumulate,
                     centres, logq, idx_out);
  return hipGetLastError();
}

}  // namespace b3d

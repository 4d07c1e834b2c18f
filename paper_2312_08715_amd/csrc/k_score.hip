// Split-path likelihood kernels over point images in device memory: the
// windowed robust likelihood of eq. (1) (one workgroup per hypothesis,
// rendered rows staged through LDS with a halo of the window half-width),
// its adjoint, and the per-pixel background terms with their summed-area
// tables used by the fused path.
#include "b3d_launch.hpp"

namespace b3d {

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }

// Stage rows [y0, y1) of a point image into LDS as three planes, with 16-byte
// loads for the aligned middle of the span.
__device__ __forceinline__ void put_plane(float* sx, float* sy, float* sz, int f, float v) {
  const int p = f / 3, comp = f - 3 * p;
  (comp == 0 ? sx : (comp == 1 ? sy : sz))[p] = v;
}

__device__ __forceinline__ void stage_rows(const float* __restrict__ img, int W, int y0, int y1, float* sx, float* sy,
                                           float* sz) {
  const int nf = (y1 - y0) * W * 3;
  const float* src = img + (size_t)y0 * W * 3;
  const int head = (int)(((16 - ((uintptr_t)src & 15)) & 15) / 4);
  const int h0 = min(head, nf);
  for (int f = threadIdx.x; f < h0; f += kBlock) put_plane(sx, sy, sz, f, src[f]);
  const int nv = (nf - h0) / 4;
  const float4* v4 = reinterpret_cast<const float4*>(src + h0);
  for (int i = threadIdx.x; i < nv; i += kBlock) {
    const float4 v = v4[i];
    const int f = h0 + 4 * i;
    put_plane(sx, sy, sz, f, v.x);
    put_plane(sx, sy, sz, f + 1, v.y);
    put_plane(sx, sy, sz, f + 2, v.z);
    put_plane(sx, sy, sz, f + 3, v.w);
  }
  for (int f = h0 + 4 * nv + threadIdx.x; f < nf; f += kBlock) put_plane(sx, sy, sz, f, src[f]);
}

// Window sums S = sum_j exp2(-D c2) and T = sum_j exp2(-D c2) D of the
// observed point (ox, oy, oz) at pixel (r, c) over staged rows starting at y0
// (rows outside [0, H) and columns outside [0, W) do not exist).  HH > 0:
// half-width known at compile time (rows rolled, columns unrolled,
// predicated); HH = 0: any h.
template <int HH, bool WANT_T>
__device__ __forceinline__ void window_sums(const ScoreConsts& sc, int H, int W, int r, int c, float ox, float oy,
                                            float oz, const float* sx, const float* sy, const float* sz, int y0,
                                            float& S, float& T) {
  S = 0.0f;
  T = 0.0f;
  if (HH > 0) {
    constexpr int n = 2 * HH + 1;
    int cc[n];
    bool cv[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const int cj = c - HH + k;
      cv[k] = cj >= 0 && cj < W;
      cc[k] = min(max(cj, 0), W - 1);
    }
#pragma unroll 1
    for (int j = 0; j < n; ++j) {
      const int rj = r - HH + j;
      if (rj < 0 || rj >= H) continue;
      const int base = (rj - y0) * W;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const float qz = sz[base + cc[k]];
        const bool ok = cv[k] && qz > 0.0f;
        const float ex = ox - sx[base + cc[k]], ey = oy - sy[base + cc[k]], ez = oz - qz;
        const float D = ok ? ex * ex + ey * ey + ez * ez : 0.0f;
        const float e = ok ? fast_exp2(-D * sc.c2) : 0.0f;
        S += e;
        if (WANT_T) T += e * D;
      }
    }
  } else {
    const int r0 = max(r - sc.h, 0), r1 = min(r + sc.h, H - 1);
    const int c0 = max(c - sc.h, 0), c1 = min(c + sc.h, W - 1);
    for (int rj = r0; rj <= r1; ++rj) {
      const int base = (rj - y0) * W;
      for (int cj = c0; cj <= c1; ++cj) {
        const float qz = sz[base + cj];
        if (!(qz > 0.0f)) continue;
        const float ex = ox - sx[base + cj], ey = oy - sy[base + cj], ez = oz - qz;
        const float D = ex * ex + ey * ey + ez * ez;
        const float e = fast_exp2(-D * sc.c2);
        S += e;
        if (WANT_T) T += e * D;
      }
    }
  }
}

template <bool WANT_T>
__device__ __forceinline__ void window_sums_h(const ScoreConsts& sc, int H, int W, int r, int c, float ox, float oy,
                                              float oz, const float* sx, const float* sy, const float* sz, int y0,
                                              float& S, float& T) {
  switch (sc.h) {
    case 1:
      window_sums<1, WANT_T>(sc, H, W, r, c, ox, oy, oz, sx, sy, sz, y0, S, T);
      break;
    case 2:
      window_sums<2, WANT_T>(sc, H, W, r, c, ox, oy, oz, sx, sy, sz, y0, S, T);
      break;
    default:
      window_sums<0, WANT_T>(sc, H, W, r, c, ox, oy, oz, sx, sy, sz, y0, S, T);
  }
}

__global__ __launch_bounds__(kBlock) void k_score(const float* __restrict__ obs, const float* __restrict__ rend, int N,
                                                  int H, int W, ScoreConsts sc, float* __restrict__ logL, int cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* red = reinterpret_cast<float*>(smem);
  float* sx = red + 64;
  const int n = blockIdx.x;
  if (n >= N) return;
  const float* rn = rend + (size_t)n * H * W * 3;
  const int h = sc.h;
  const int band = max(cap / (3 * W) - 2 * h, 1);
  float acc[1] = {0.0f};
  for (int a = 0; a < H; a += band) {
    const int b = min(a + band, H);
    const int y0 = max(a - h, 0), y1 = min(b + h, H);
    const int np = (y1 - y0) * W;
    float* sy = sx + np;
    float* sz = sy + np;
    stage_rows(rn, W, y0, y1, sx, sy, sz);
    __syncthreads();
    for (int k = threadIdx.x; k < (b - a) * W; k += kBlock) {
      const int r = a + k / W, c = k - (k / W) * W;
      const float* q = obs + 3 * ((size_t)r * W + c);
      const float oz = q[2];
      if (!(oz > 0.0f)) continue;
      float S, T;
      window_sums_h<false>(sc, H, W, r, c, q[0], q[1], oz, sx, sy, sz, y0, S, T);
      acc[0] += fast_ln(sc.a + sc.bn * S);
    }
    __syncthreads();
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) logL[n] = acc[0];
}

hipError_t launch_score(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc, float* logL,
                        int cap, hipStream_t st) {
  const size_t lds = sizeof(float) * (64 + (size_t)cap);
  hipLaunchKernelGGL(k_score, dim3(N), dim3(kBlock), lds, st, obs, rend, N, H, W, sc, logL, cap);
  return hipGetLastError();
}

// Adjoint of k_score.  Per band of output rows [a, b): rendered rows
// [a - 2h, b + 2h) and the weights w_i = (b/L_i) of observed rows
// [a - h, b + h) go to LDS; then every rendered pixel gathers
// sum_i w_i K_ij (q~_i - q_j) / sigma^2 over its window (the window is
// symmetric, so no atomics are needed).
__global__ __launch_bounds__(kBlock) void k_score_backward(const float* __restrict__ obs, const float* __restrict__ rend,
                                                           int N, int H, int W, ScoreConsts sc,
                                                           const float* __restrict__ dlogL, float* __restrict__ d_rend,
                                                           float* __restrict__ d_sigma, float* __restrict__ d_pout,
                                                           int cap) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* red = reinterpret_cast<float*>(smem);
  float* sx = red + 64;
  const int n = blockIdx.x;
  if (n >= N) return;
  const float g = dlogL ? dlogL[n] : 1.0f;
  const float* rn = rend + (size_t)n * H * W * 3;
  float* dn = d_rend ? d_rend + (size_t)n * H * W * 3 : nullptr;
  const int h = sc.h;
  // LDS: 3 planes of (band + 4h) rows and 1 plane of (band + 2h) rows
  const int band = max(cap / (4 * W) - 4 * h, 1);
  float acc[2] = {0.0f, 0.0f};  // d/dsigma, d/dp_out
  for (int a = 0; a < H; a += band) {
    const int b = min(a + band, H);
    const int y0 = max(a - 2 * h, 0), y1 = min(b + 2 * h, H);
    const int wa = max(a - h, 0), wb = min(b + h, H);
    const int np = (y1 - y0) * W;
    float* sy = sx + np;
    float* sz = sy + np;
    float* sw = sz + np;
    stage_rows(rn, W, y0, y1, sx, sy, sz);
    __syncthreads();
    for (int k = threadIdx.x; k < (wb - wa) * W; k += kBlock) {
      const int r = wa + k / W, c = k - (k / W) * W;
      const float* q = obs + 3 * ((size_t)r * W + c);
      const float oz = q[2];
      float w = 0.0f;
      if (oz > 0.0f) {
        float S, T;
        window_sums_h<true>(sc, H, W, r, c, q[0], q[1], oz, sx, sy, sz, y0, S, T);
        const float L = sc.a + sc.bn * S;
        w = sc.bn / L;
        if (r >= a && r < b) {
          acc[0] += w * (T * sc.inv_s3 - 3.0f * S * sc.inv_s);
          acc[1] += (sc.invV - sc.normM * S) / L;
        }
      }
      sw[k] = w;
    }
    __syncthreads();
    if (dn) {
      const float scale = g * sc.inv_s2;
      for (int k = threadIdx.x; k < (b - a) * W; k += kBlock) {
        const int r = a + k / W, c = k - (k / W) * W;
        const int pj = (r - y0) * W + c;
        const float qz = sz[pj];
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        if (qz > 0.0f) {
          const float qx = sx[pj], qy = sy[pj];
          const int r0 = max(r - h, 0), r1 = min(r + h, H - 1);
          const int c0 = max(c - h, 0), c1 = min(c + h, W - 1);
          for (int ri = r0; ri <= r1; ++ri) {
            for (int ci = c0; ci <= c1; ++ci) {
              const float w = sw[(ri - wa) * W + ci];
              if (w == 0.0f) continue;
              const float* q = obs + 3 * ((size_t)ri * W + ci);
              const float ex = q[0] - qx, ey = q[1] - qy, ez = q[2] - qz;
              const float e = w * fast_exp2(-(ex * ex + ey * ey + ez * ez) * sc.c2);
              gx += e * ex;
              gy += e * ey;
              gz += e * ez;
            }
          }
        }
        float* o = dn + 3 * ((size_t)r * W + c);
        o[0] = gx * scale;
        o[1] = gy * scale;
        o[2] = gz * scale;
      }
    }
    __syncthreads();
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    if (d_sigma) d_sigma[n] = g * acc[0];
    if (d_pout) d_pout[n] = g * acc[1];
  }
}

hipError_t launch_score_backward(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc,
                                 const float* dlogL, float* d_rend, float* d_sigma, float* d_pout, int cap,
                                 hipStream_t st) {
  const size_t lds = sizeof(float) * (64 + (size_t)cap);
  hipLaunchKernelGGL(k_score_backward, dim3(N), dim3(kBlock), lds, st, obs, rend, N, H, W, sc, dlogL, d_rend, d_sigma,
                     d_pout, cap);
  return hipGetLastError();
}

// Per-pixel likelihood terms of the background alone (double precision):
// terms[0][p] = l_p, terms[1][p] = dl_p/dp_out, terms[2][p] = dl_p/dsigma,
// zero for invalid observed pixels.
__global__ void k_bg_terms(SceneDev s, double* __restrict__ terms) {
  const int H = s.cam.H, W = s.cam.W;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= H * W) return;
  const int r = p / W, c = p - r * W;
  const float* q = s.obs + 3 * (size_t)p;
  double l = 0.0, dp = 0.0, ds = 0.0;
  if (q[2] > 0.0f) {
    double S = 0.0, T = 0.0;
    if (s.bg) {
      const int h = s.sc.h;
      for (int rj = max(r - h, 0); rj <= min(r + h, H - 1); ++rj)
        for (int cj = max(c - h, 0); cj <= min(c + h, W - 1); ++cj) {
          const unsigned long long k = s.bg[(size_t)rj * W + cj];
          if (k == kEmptyKey) continue;
          const double z = (double)key_depth(k);
          const double ex = (double)q[0] - z * (double)ray_x(s.cam, cj);
          const double ey = (double)q[1] - z * (double)ray_y(s.cam, rj);
          const double ez = (double)q[2] - z;
          const double D = ex * ex + ey * ey + ez * ez;
          const double e = exp(-D * s.sc.dc);
          S += e;
          T += e * D;
        }
    }
    const double L = s.sc.da + s.sc.dbn * S;
    l = log(L);
    dp = (s.sc.dinvV - s.sc.dnormM * S) / L;
    ds = (s.sc.dbn / L) * (T * s.sc.dinv_s3 - 3.0 * S * s.sc.dinv_s);
  }
  const size_t HW = (size_t)H * W;
  terms[p] = l;
  terms[HW + p] = dp;
  terms[2 * HW + p] = ds;
}

// Summed-area tables: sat[k][(r)(W+1) + c] = sum of terms[k] over rows < r, cols < c.
__global__ void k_sat_rows(const double* __restrict__ terms, int H, int W, double* __restrict__ sat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (k, row) pairs, row in [0, H]
  if (i >= 3 * (H + 1)) return;
  const int k = i / (H + 1), r = i - k * (H + 1);
  double* o = sat + (size_t)k * (H + 1) * (W + 1) + (size_t)r * (W + 1);
  o[0] = 0.0;
  double run = 0.0;
  for (int c = 0; c < W; ++c) {
    if (r > 0) run += terms[(size_t)k * H * W + (size_t)(r - 1) * W + c];
    o[c + 1] = run;
  }
}

__global__ void k_sat_cols(int H, int W, double* __restrict__ sat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // (k, col) pairs
  if (i >= 3 * (W + 1)) return;
  const int k = i / (W + 1), c = i - k * (W + 1);
  double* o = sat + (size_t)k * (H + 1) * (W + 1);
  double run = 0.0;
  for (int r = 0; r <= H; ++r) {
    run += o[(size_t)r * (W + 1) + c];
    o[(size_t)r * (W + 1) + c] = run;
  }
}

hipError_t launch_background_terms(const SceneDev& s, double* terms, hipStream_t st) {
  const int H = s.cam.H, W = s.cam.W;
  double* sat = const_cast<double*>(s.sat);
  hipLaunchKernelGGL(k_bg_terms, dim3((H * W + 255) / 256), dim3(256), 0, st, s, terms);
  hipLaunchKernelGGL(k_sat_rows, dim3((3 * (H + 1) + 63) / 64), dim3(64), 0, st, terms, H, W, sat);
  hipLaunchKernelGGL(k_sat_cols, dim3((3 * (W + 1) + 63) / 64), dim3(64), 0, st, H, W, sat);
  return hipGetLastError();
}

}  // namespace b3d

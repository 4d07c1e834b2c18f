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

// ---- split path over a ring of rows --------------------------------------
//
// The rendered point image of a hypothesis is streamed from top to bottom
// exactly once: an LDS ring holds, in their stored x, y, z order, the rows a
// window can still reach, and the next R rows are loaded into registers
// (kRingPF 16-byte words per thread) while the current R rows are scored, so
// that the loads stay in flight across the arithmetic and the barriers.  A
// row y sits in slot y mod nrows.  Needs W a multiple of 4 and 16-byte
// aligned images (rows are then whole 16-byte words); the host checks both.

// A workgroup barrier that orders LDS only: the ring kernels keep global
// loads (the next rows) and stores (gradients) in flight across it, where
// __syncthreads would first wait for all of them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kRingPF = 8;  // float4 words per thread per step, score
constexpr int kRingPP = 8;  // output pixels per thread per step, score
constexpr int kRingQP = kRingPP / 4;  // ... as quads
constexpr int kBackPF = 8;  // float4 words per thread per step, adjoint
constexpr int kBackPP = 4;  // list entries per thread per step, adjoint

typedef float f4v __attribute__((ext_vector_type(4)));

template <int PF>
__device__ __forceinline__ void rows_load(const float* __restrict__ img, int wpr, int y0, int y1, f4v (&v)[PF]) {
  // every lane loads PF words (beyond the span: its last word again), so the
  // registers are written unconditionally; rows_store drops the extra ones
  const int nw = y1 > y0 ? (y1 - y0) * wpr : 0;
  if (nw == 0) return;
  const f4v* src = reinterpret_cast<const f4v*>(img) + (size_t)y0 * wpr;
  const int rounds = (nw + kBlock - 1) / kBlock;  // uniform: whole rounds past the span are skipped
#pragma unroll
  for (int i = 0; i < PF; ++i)
    if (i < rounds) v[i] = src[min((int)threadIdx.x + i * kBlock, nw - 1)];
}

template <int PF>
__device__ __forceinline__ void rows_store(float* ring, int nrows, int wpr, int y0, int y1, const f4v (&v)[PF]) {
  const int nw = y1 > y0 ? (y1 - y0) * wpr : 0;
  if (nw == 0) return;
  f4v* dst = reinterpret_cast<f4v*>(ring);
  // word k = tid + i kBlock of the span sits in row (k / wpr), column (k mod
  // wpr); both advance by fixed amounts from one i to the next
  const int dq = kBlock / wpr, dm = kBlock - dq * wpr;
  int ro = (int)threadIdx.x / wpr;
  int col = (int)threadIdx.x - ro * wpr;
  int slot = (y0 + ro) % nrows;
  const int rounds = (nw + kBlock - 1) / kBlock;
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    if (i >= rounds) break;
    if ((int)threadIdx.x + i * kBlock < nw) dst[slot * wpr + col] = v[i];
    col += dm;
    int carry = dq;
    if (col >= wpr) {
      col -= wpr;
      ++carry;
    }
    slot += carry;
    while (slot >= nrows) slot -= nrows;
  }
}

// Window sums S = sum_j exp2(-D c2) (and T = sum_j exp2(-D c2) D) of the
// observed point o at pixel (r, c) over the rendered rows held in the ring.
template <int HH, bool WANT_T>
__device__ __forceinline__ void window_ring(const ScoreConsts& sc, int H, int W, int nrows, int r, int c, float ox,
                                            float oy, float oz, const float* ring, float& S, float& T) {
  const int h = HH > 0 ? HH : sc.h;
  S = 0.0f;
  T = 0.0f;
  int slot = (r - h + nrows) % nrows;
  if (HH > 0) {
    constexpr int n = 2 * HH + 1;
    int cc[n];
    bool cv[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const int cj = c - HH + k;
      cv[k] = cj >= 0 && cj < W;
      cc[k] = 3 * min(max(cj, 0), W - 1);
    }
#pragma unroll 1
    for (int j = 0; j < n; ++j) {
      const int rj = r - HH + j;
      if (rj >= 0 && rj < H) {
        const float* row = ring + slot * 3 * W;
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const float qz = row[cc[k] + 2];
          const bool ok = cv[k] && qz > 0.0f;
          const float ex = ox - row[cc[k]], ey = oy - row[cc[k] + 1], ez = oz - qz;
          const float D = ok ? ex * ex + ey * ey + ez * ez : 0.0f;
          const float e = ok ? fast_exp2(-D * sc.c2) : 0.0f;
          S += e;
          if (WANT_T) T += e * D;
        }
      }
      slot = slot + 1 == nrows ? 0 : slot + 1;
    }
  } else {
    const int c0 = max(c - h, 0), c1 = min(c + h, W - 1);
    for (int rj = r - h; rj <= r + h; ++rj) {
      if (rj >= 0 && rj < H) {
        const float* row = ring + slot * 3 * W;
        for (int cj = c0; cj <= c1; ++cj) {
          const float qz = row[3 * cj + 2];
          if (!(qz > 0.0f)) continue;
          const float ex = ox - row[3 * cj], ey = oy - row[3 * cj + 1], ez = oz - qz;
          const float D = ex * ex + ey * ey + ez * ez;
          const float e = fast_exp2(-D * sc.c2);
          S += e;
          if (WANT_T) T += e * D;
        }
      }
      slot = slot + 1 == nrows ? 0 : slot + 1;
    }
  }
}

// Work compaction inside a wave.  Only some pixels take the window
// arithmetic (valid observed points; drawn rendered points): lanes push
// those items into their wave's LDS queue (kQueueItems float4 slots) and the
// whole wave processes 64 of them at a time, one per lane, so that a wave
// does not run the window for one valid pixel among 63 idle lanes.  Items
// leave the queue in the order they were pushed (lane order within a push),
// so every lane's order of accumulation is fixed by the input alone.
constexpr int kQueueItems = 128;

struct WaveQueue {
  float4* q;  // this wave's kQueueItems slots
  int n;      // items queued (uniform across the wave)
};

template <class F>
__device__ __forceinline__ void wq_push(WaveQueue& w, bool valid, const float4& item, F&& process) {
  const int lane = threadIdx.x & 63;
  const unsigned long long m = __ballot(valid);
  if (valid) w.q[w.n + __popcll(m & ((1ull << lane) - 1ull))] = item;
  w.n += __popcll(m);
  if (w.n >= 64) {
    __builtin_amdgcn_wave_barrier();
    const float4 mine = w.q[lane];
    const bool more = lane + 64 < w.n;
    float4 rest = mine;
    if (more) rest = w.q[lane + 64];
    __builtin_amdgcn_wave_barrier();
    if (more) w.q[lane] = rest;
    w.n -= 64;
    process(mine, true);
  }
}

template <class F>
__device__ __forceinline__ void wq_flush(WaveQueue& w, F&& process) {
  if (w.n > 0) {
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_wave_barrier();
    const bool act = lane < w.n;
    float4 mine = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (act) mine = w.q[lane];
    w.n = 0;
    process(mine, act);
  }
}

// ---- the observed image's valid pixels, listed once per call -------------
//
// Every hypothesis is scored against the same observed image, so its valid
// pixels (z > 0) are listed once, row-major, in the caller's workspace:
// rows[r] = index of row r's first entry (rows[H] = number of entries),
// list[e] = (x, y, z, pixel index as int bits).  The scoring kernels then
// take only those pixels, densely, instead of every pixel of a row.

__device__ __forceinline__ int block_excl_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;  // inclusive scan within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < kWaves; ++w) {
    off += w < wave ? wsum[w] : 0;
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Block r counts the valid pixels of row r into rows[r + 1].
__global__ __launch_bounds__(kBlock) void k_obs_count(const float* __restrict__ obs, int H, int W, int* rows) {
  __shared__ int wsum[kWaves];
  const int r = blockIdx.x;
  int n = 0;
  for (int c = threadIdx.x; c < W; c += kBlock) n += obs[3 * ((size_t)r * W + c) + 2] > 0.0f ? 1 : 0;
  int total;
  (void)block_excl_scan(n, wsum, &total);
  if (threadIdx.x == 0) rows[r + 1] = total;
  if (r == 0 && threadIdx.x == 0) rows[0] = 0;
}

// One block: rows[1..H] from counts to running totals.
__global__ __launch_bounds__(kBlock) void k_obs_scan(int H, int* rows) {
  __shared__ int wsum[kWaves];
  int carry = 0;
  for (int base = 1; base <= H; base += kBlock) {
    const int r = base + (int)threadIdx.x;
    const int v = r <= H ? rows[r] : 0;
    int total;
    const int ex = block_excl_scan(v, wsum, &total);
    if (r <= H) rows[r] = carry + ex + v;
    carry += total;
  }
}

// Block r writes row r's valid pixels, in column order, from rows[r].
__global__ __launch_bounds__(kBlock) void k_obs_fill(const float* __restrict__ obs, int H, int W,
                                                     const int* __restrict__ rows, float4* __restrict__ list) {
  __shared__ int wsum[kWaves];
  const int r = blockIdx.x;
  int at = rows[r];
  for (int base = 0; base < W; base += kBlock) {
    const int c = base + (int)threadIdx.x;
    const float* q = obs + 3 * ((size_t)r * W + min(c, W - 1));
    const bool v = c < W && q[2] > 0.0f;
    int total;
    const int ex = block_excl_scan(v ? 1 : 0, wsum, &total);
    if (v) list[at + ex] = make_float4(q[0], q[1], q[2], __int_as_float(r * W + c));
    at += total;
  }
}

size_t score_workspace_bytes(int H, int W) {
  return (((size_t)(H + 1) * sizeof(int) + 15) & ~(size_t)15) + sizeof(float4) * (size_t)H * W;
}

hipError_t launch_obs_list(const float* obs, int H, int W, void* workspace, hipStream_t st) {
  int* rows = reinterpret_cast<int*>(workspace);
  float4* list = reinterpret_cast<float4*>(reinterpret_cast<char*>(workspace) +
                                           (((size_t)(H + 1) * sizeof(int) + 15) & ~(size_t)15));
  hipLaunchKernelGGL(k_obs_count, dim3(H), dim3(kBlock), 0, st, obs, H, W, rows);
  hipLaunchKernelGGL(k_obs_scan, dim3(1), dim3(kBlock), 0, st, H, rows);
  hipLaunchKernelGGL(k_obs_fill, dim3(H), dim3(kBlock), 0, st, obs, H, W, rows, list);
  return hipGetLastError();
}

// Entries [e0, e1) of the list into registers, kRingPP per thread at most
// (beyond e1: z = 0, which no step scores).
template <int PP>
__device__ __forceinline__ void entries_load(const float4* __restrict__ list, int e0, int e1, f4v (&v)[PP]) {
  const f4v* src = reinterpret_cast<const f4v*>(list);
  const int rounds = (e1 - e0 + kBlock - 1) / kBlock;  // uniform
#pragma unroll
  for (int i = 0; i < PP; ++i) {
    if (i < rounds) {
      const int e = e0 + (int)threadIdx.x + i * kBlock;
      f4v x = src[min(e, max(e1 - 1, 0))];
      if (e >= e1) x.z = 0.0f;
      v[i] = x;
    }
  }
}

// logL of one hypothesis per workgroup; rows [a, a + R) per step, the ring
// holding rendered rows [a - h, a + R + h), the step's valid observed pixels
// taken from the list, one per lane.
template <int HH>
__global__ __launch_bounds__(kBlock) void k_score_ring(const int* __restrict__ rows, const float4* __restrict__ list,
                                                       const float* __restrict__ rend, int N, int H, int W,
                                                       ScoreConsts sc, int R, float* __restrict__ logL) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* red = reinterpret_cast<float*>(smem);
  float* ring = red + 64;
  const int n = blockIdx.x;
  if (n >= N) return;
  const int h = HH > 0 ? HH : sc.h;
  const int nrows = R + 2 * h, wpr = 3 * W / 4;
  const float* rn = rend + (size_t)n * H * W * 3;
  f4v v[kRingPF], cur[kRingPP];
  rows_load<kRingPF>(rn, wpr, 0, min(h, H), v);
  rows_store<kRingPF>(ring, nrows, wpr, 0, min(h, H), v);
  rows_load<kRingPF>(rn, wpr, min(h, H), min(h + R, H), v);
  float acc[1] = {0.0f};
  for (int a = 0; a < H; a += R) {
    const int ya = min(a + h, H), yb = min(a + R + h, H);
    const int e0 = rows[a], e1 = rows[min(a + R, H)];
    lds_barrier();
    rows_store<kRingPF>(ring, nrows, wpr, ya, yb, v);
    // this step's entries (issued before the next rows, so that waiting for
    // them does not wait for those)
    entries_load<kRingPP>(list, e0, e1, cur);
    lds_barrier();
    rows_load<kRingPF>(rn, wpr, yb, min(yb + R, H), v);  // the next step's rows, in flight while these are scored
    const int rounds = (e1 - e0 + kBlock - 1) / kBlock;
#pragma unroll 1
    for (int i = 0; i < rounds; ++i) {
      const f4v it = cur[0];
#pragma unroll
      for (int t = 0; t + 1 < kRingPP; ++t) cur[t] = cur[t + 1];
      if (it.z > 0.0f) {
        const int p = __float_as_int(it.w);
        const int r = p / W;
        float S, T;
        window_ring<HH, false>(sc, H, W, nrows, r, p - r * W, it.x, it.y, it.z, ring, S, T);
        acc[0] += fast_ln(sc.a + sc.bn * S);
      }
    }
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) logL[n] = acc[0];
}

int score_ring_rows(int H, int W, int h) {
  if (W % 4 != 0) return 0;
  const int wpr = 3 * W / 4;
  int R = std::min(kRingPF * kBlock / wpr, kRingPP * kBlock / W);
  // five workgroups per CU
  while (R > 0 && sizeof(float) * (64 + (size_t)(R + 2 * h) * 3 * W) > 32768) --R;
  if (R < std::max(h, 1)) return 0;  // the prologue loads h rows in one step
  return std::min(R, H);
}

hipError_t launch_score_ring(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc, int R,
                             void* workspace, float* logL, hipStream_t st) {
  if (hipError_t e = launch_obs_list(obs, H, W, workspace, st)) return e;
  const int* rows = reinterpret_cast<const int*>(workspace);
  const float4* list = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(workspace) +
                                                       (((size_t)(H + 1) * sizeof(int) + 15) & ~(size_t)15));
  const size_t lds = sizeof(float) * (64 + (size_t)(R + 2 * sc.h) * 3 * W);
  switch (sc.h) {
    case 1:
      hipLaunchKernelGGL(k_score_ring<1>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R, logL);
      break;
    case 2:
      hipLaunchKernelGGL(k_score_ring<2>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R, logL);
      break;
    default:
      hipLaunchKernelGGL(k_score_ring<0>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R, logL);
  }
  return hipGetLastError();
}

// Adjoint of k_score_ring.  Step a: rendered rows [a, a + R + 2h) in one
// ring; in a second, for the observed rows [a - h, a + R + h), each pixel's
// observed point and window weight w_i = g b / L_i as one 16-byte word
// (zeros for invalid pixels).  The weights of rows [a + h, a + R + h) are
// computed from the list (with the sigma and p_out sums of those rows), then
// every rendered pixel of rows [a, a + R) gathers
// sum_i w_i K_ij (q~_i - q_j) / sigma^2 over its window (the window is
// symmetric: a gather, no atomics) and is written once: a drawn pixel by the
// lane that processes it from its wave's queue, the others as zeros, by
// whole empty quads where they can.
template <int HH>
__global__ __launch_bounds__(kBlock) void k_score_backward_ring(const int* __restrict__ rows,
                                                                const float4* __restrict__ list,
                                                                const float* __restrict__ rend, int N, int H, int W,
                                                                ScoreConsts sc, int R, const float* __restrict__ dlogL,
                                                                float* __restrict__ d_rend, float* __restrict__ d_sigma,
                                                                float* __restrict__ d_pout) {
  extern __shared__ __align__(16) unsigned char smem[];
  float* red = reinterpret_cast<float*>(smem);
  const int h = HH > 0 ? HH : sc.h;
  const int nrows = R + 2 * h, wpr = 3 * W / 4;
  float4* queues = reinterpret_cast<float4*>(red + 64);
  float* rr = reinterpret_cast<float*>(queues + kWaves * kQueueItems);  // rendered ring
  f4v* wo = reinterpret_cast<f4v*>(rr + (size_t)nrows * 3 * W);        // (observed point, weight) ring
  const int n = blockIdx.x;
  if (n >= N) return;
  const float g = dlogL ? dlogL[n] : 1.0f;
  const float gb = g * sc.bn;
  const float* rn = rend + (size_t)n * H * W * 3;
  float* dn = d_rend ? d_rend + (size_t)n * H * W * 3 : nullptr;
  WaveQueue wq{queues + (threadIdx.x >> 6) * kQueueItems, 0};
  float acc[2] = {0.0f, 0.0f};  // d/dsigma, d/dp_out (times g at the end)
  f4v vr[kBackPF], cur[kBackPP];
  const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};

  // weights of the observed rows [y0, y1): clear their slots, then each
  // valid pixel of the list (in cur) writes its point and weight
  auto weights = [&](int y0, int y1, int e0, int e1) {
    for (int k = threadIdx.x; k < (y1 - y0) * W; k += kBlock) {
      const int dr = k / W;
      wo[((y0 + dr) % nrows) * W + (k - dr * W)] = zero;
    }
    lds_barrier();
    const int rounds = (e1 - e0 + kBlock - 1) / kBlock;
#pragma unroll 1
    for (int i = 0; i < rounds; ++i) {
      const f4v it = cur[0];
#pragma unroll
      for (int t = 0; t + 1 < kBackPP; ++t) cur[t] = cur[t + 1];
      if (it.z > 0.0f) {
        const int p = __float_as_int(it.w);
        const int r = p / W, c = p - r * W;
        float S, T;
        window_ring<HH, true>(sc, H, W, nrows, r, c, it.x, it.y, it.z, rr, S, T);
        const float L = sc.a + sc.bn * S;
        acc[0] += (sc.bn / L) * (T * sc.inv_s3 - 3.0f * S * sc.inv_s);
        acc[1] += (sc.invV - sc.normM * S) / L;
        f4v o = it;
        o.w = gb / L;
        wo[(r % nrows) * W + c] = o;
      }
    }
  };

  // prologue: rendered rows [0, 2h), weights of observed rows [0, h)
  const int p1 = min(2 * h, H), p2 = min(h, H);
  rows_load<kBackPF>(rn, wpr, 0, p1, vr);
  entries_load<kBackPP>(list, rows[0], rows[p2], cur);
  rows_store<kBackPF>(rr, nrows, wpr, 0, p1, vr);
  lds_barrier();
  weights(0, p2, rows[0], rows[p2]);
  rows_load<kBackPF>(rn, wpr, p1, min(p1 + R, H), vr);
  const float scale = sc.inv_s2;
  for (int a = 0; a < H; a += R) {
    const int ra = min(a + 2 * h, H), rb = min(a + R + 2 * h, H);  // rendered rows arriving
    const int oa = min(a + h, H), ob = min(a + R + h, H);          // observed rows weighted now
    lds_barrier();
    rows_store<kBackPF>(rr, nrows, wpr, ra, rb, vr);
    // this step's entries, then the next step's rows (in flight while this
    // step runs; waiting for the entries does not wait for them)
    entries_load<kBackPP>(list, rows[oa], rows[ob], cur);
    rows_load<kBackPF>(rn, wpr, rb, min(rb + R, H), vr);
    weights(oa, ob, rows[oa], rows[ob]);
    lds_barrier();
    if (dn) {
      auto gather = [&](const float4& it, bool act) {
        if (act) {
          const int p = __float_as_int(it.w);
          const int r = p / W, c = p - r * W;
          const float qx = it.x, qy = it.y, qz = it.z;
          float gx = 0.0f, gy = 0.0f, gz = 0.0f;
          const int c0 = max(c - h, 0), c1 = min(c + h, W - 1);
          int slot = (r - h + nrows) % nrows;
          for (int ri = r - h; ri <= r + h; ++ri) {
            if (ri >= 0 && ri < H) {
              const f4v* row = wo + slot * W;
              for (int ci = c0; ci <= c1; ++ci) {
                const f4v o = row[ci];
                if (o.w == 0.0f) continue;
                const float ex = o.x - qx, ey = o.y - qy, ez = o.z - qz;
                const float e = o.w * fast_exp2(-(ex * ex + ey * ey + ez * ez) * sc.c2);
                gx += e * ex;
                gy += e * ey;
                gz += e * ez;
              }
            }
            slot = slot + 1 == nrows ? 0 : slot + 1;
          }
          float* o = dn + 3 * (size_t)p;
          o[0] = gx * scale;
          o[1] = gy * scale;
          o[2] = gz * scale;
        }
      };
      // quads with no drawn pixel are written as zeros, three 16-byte words
      // each; the other quads' empty pixels are written one by one below
      const int np = (min(a + R, H) - a) * W, nq = np / 4;
      for (int q = threadIdx.x; q < nq; q += kBlock) {
        const int p0 = a * W + 4 * q;
        const float* qj = rr + (((p0 / W) % nrows) * W + (p0 % W)) * 3;
        if (!(qj[2] > 0.0f || qj[5] > 0.0f || qj[8] > 0.0f || qj[11] > 0.0f)) {
          f4v* o = reinterpret_cast<f4v*>(dn + 3 * (size_t)p0);
          o[0] = zero;
          o[1] = zero;
          o[2] = zero;
        }
      }
      for (int b0 = 0; b0 < np; b0 += kBlock) {
        const int k = b0 + (int)threadIdx.x;
        bool drawn = false;
        float4 it = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (k < np) {
          const int dr = k / W;
          const int r = a + dr, c = k - dr * W;
          const float* row = rr + (r % nrows) * W * 3;
          const float* qj = row + c * 3;
          it = make_float4(qj[0], qj[1], qj[2], __int_as_float(r * W + c));
          drawn = it.z > 0.0f;
          const int c4 = c & ~3;
          const bool quad_drawn = row[3 * c4 + 2] > 0.0f || row[3 * c4 + 5] > 0.0f || row[3 * c4 + 8] > 0.0f ||
                                  row[3 * c4 + 11] > 0.0f;
          if (!drawn && quad_drawn) {
            float* o = dn + 3 * ((size_t)r * W + c);
            o[0] = 0.0f;
            o[1] = 0.0f;
            o[2] = 0.0f;
          }
        }
        wq_push(wq, drawn, it, gather);
      }
      wq_flush(wq, gather);
    }
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    if (d_sigma) d_sigma[n] = g * acc[0];
    if (d_pout) d_pout[n] = g * acc[1];
  }
}

constexpr size_t kQueueBytes = sizeof(float4) * kWaves * kQueueItems;

int score_backward_ring_rows(int H, int W, int h) {
  if (W % 4 != 0) return 0;
  const int wpr = 3 * W / 4;
  int R = std::min(kBackPF * kBlock / wpr, kBackPP * kBlock / W);
  // three workgroups per CU
  while (R > 0 && sizeof(float) * 64 + kQueueBytes + sizeof(float) * (size_t)(R + 2 * h) * 7 * W > 54272) --R;
  if (R < std::max(2 * h, 1)) return 0;  // the prologue loads 2h rendered rows in one step
  return std::min(R, H);
}

hipError_t launch_score_backward_ring(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc,
                                      int R, void* workspace, const float* dlogL, float* d_rend, float* d_sigma,
                                      float* d_pout, hipStream_t st) {
  if (hipError_t e = launch_obs_list(obs, H, W, workspace, st)) return e;
  const int* rows = reinterpret_cast<const int*>(workspace);
  const float4* list = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(workspace) +
                                                       (((size_t)(H + 1) * sizeof(int) + 15) & ~(size_t)15));
  const size_t lds = sizeof(float) * 64 + kQueueBytes + sizeof(float) * (size_t)(R + 2 * sc.h) * 7 * W;
  switch (sc.h) {
    case 1:
      hipLaunchKernelGGL(k_score_backward_ring<1>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R,
                         dlogL, d_rend, d_sigma, d_pout);
      break;
    case 2:
      hipLaunchKernelGGL(k_score_backward_ring<2>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R,
                         dlogL, d_rend, d_sigma, d_pout);
      break;
    default:
      hipLaunchKernelGGL(k_score_backward_ring<0>, dim3(N), dim3(kBlock), lds, st, rows, list, rend, N, H, W, sc, R,
                         dlogL, d_rend, d_sigma, d_pout);
  }
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

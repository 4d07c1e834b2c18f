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
                            uint32_t stage, float* __restrict__ poses, const float* __restrict__ hscale) {
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
  const float sc = hscale ? *hscale : 1.0f;  // translation half extents scaled (a widened search)
  const float off[3] = {grid_offset(ix, g.count[0], g.half[0] * sc, g.cell_centres),
                        grid_offset(iy, g.count[1], g.half[1] * sc, g.cell_centres),
                        grid_offset(iz, g.count[2], g.half[2] * sc, g.cell_centres)};
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
                            uint32_t stage, float* poses, hipStream_t st, const float* hscale) {
  const long long N = (long long)g.count[0] * g.count[1] * g.count[2] * g.n_rot * P;
  const int blocks = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_enumerate, dim3(blocks), dim3(256), 0, st, g, centres, P, key0, key1, stage, poses, hscale);
  return hipGetLastError();
}

// Block (p, k): logsumexp of segment p and its draw k by Gumbel-max, BS
// threads (each block reads its segment three times; a draw is one block, so
// long segments take the larger block to cut each thread's serial share).
template <int BS>
__global__ __launch_bounds__(BS) void k_sample(const float* __restrict__ logL, int P, int N, int K, uint32_t k0,
                                               uint32_t k1, uint32_t stage, uint32_t kbase, float* __restrict__ w,
                                               int* __restrict__ idx, float* __restrict__ logw) {
  constexpr int NW = BS / 64;
  __shared__ float rv[NW];
  __shared__ int ri[NW];
  __shared__ float red[NW];
  const int blk = blockIdx.x;
  const int p = blk / K, k = blk - p * K;
  const float* L = logL + (size_t)p * N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // max
  float m = -INFINITY;
  for (int n = threadIdx.x; n < N; n += BS) m = fmaxf(m, L[n]);
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wave] = m;
  __syncthreads();
  m = red[0];
  for (int i = 1; i < NW; ++i) m = fmaxf(m, red[i]);
  __syncthreads();
  // sum of exp(l - m), fixed order
  float s = 0.0f;
  for (int n = threadIdx.x; n < N; n += BS) s += expf(L[n] - m);
  s = wave_sum(s);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  s = red[0];
  for (int i = 1; i < NW; ++i) s += red[i];
  const float lse = m + logf(s);
  if (k == 0 && w)
    for (int n = threadIdx.x; n < N; n += BS) w[(size_t)p * N + n] = expf(L[n] - lse);
  // argmax of l + G, ties to the lowest index
  const uint32_t draw = kbase + (uint32_t)(p * K + k);
  float bv = -INFINITY;
  int bi = -1;
  for (int n = threadIdx.x; n < N; n += BS) {
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
    for (int i = 1; i < NW; ++i)
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
  if (N > 2048)
    hipLaunchKernelGGL(k_sample<1024>, dim3(P * K), dim3(1024), 0, st, logL, P, N, K, key0, key1, stage, k0, w, idx,
                       logw);
  else
    hipLaunchKernelGGL(k_sample<kBlock>, dim3(P * K), dim3(kBlock), 0, st, logL, P, N, K, key0, key1, stage, k0, w,
                       idx, logw);
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

// ---- table-contact placement and the SMC sampler's per-particle steps ----

// Camera-frame pose of an object resting on face f, turned by th about the
// table normal and moved by (dx, dy): T [Rz(th) R | Rz(th) d + (dx, dy, 0)].
__device__ void contact_pose(const ContactDev& C, const FaceDev& f, float dx, float dy, float th,
                             float* __restrict__ out) {
  float s, c;
  sincosf(th, &s, &c);
  float Rt[9], tt[3];
  for (int j = 0; j < 3; ++j) {
    Rt[j] = c * f.R[j] - s * f.R[3 + j];
    Rt[3 + j] = s * f.R[j] + c * f.R[3 + j];
    Rt[6 + j] = f.R[6 + j];
  }
  tt[0] = c * f.d[0] - s * f.d[1] + dx;
  tt[1] = s * f.d[0] + c * f.d[1] + dy;
  tt[2] = f.d[2];
  for (int r = 0; r < 3; ++r) {
    const float* T = C.T + 4 * r;
    for (int j = 0; j < 3; ++j) out[4 * r + j] = T[0] * Rt[j] + T[1] * Rt[3 + j] + T[2] * Rt[6 + j];
    out[4 * r + 3] = T[0] * tt[0] + T[1] * tt[1] + T[2] * tt[2] + T[3];
  }
  out[12] = 0.0f;
  out[13] = 0.0f;
  out[14] = 0.0f;
  out[15] = 1.0f;
}

__global__ void k_contact_poses(ContactDev C, const int* __restrict__ place, const float* __restrict__ dphi, int N,
                                float* __restrict__ poses) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int o = min(max(place[2 * n], 0), C.n_types - 1), c = min(max(place[2 * n + 1], 0), 5);
  contact_pose(C, C.faces[6 * o + c], dphi[3 * n], dphi[3 * n + 1], dphi[3 * n + 2], poses + 16 * (size_t)n);
}

hipError_t launch_contact_poses(const ContactDev& C, const int* place, const float* dphi, int N, float* poses,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_contact_poses, dim3((N + 63) / 64), dim3(64), 0, st, C, place, dphi, N, poses);
  return hipGetLastError();
}

// Split cell j = (ix ny + iy) nt + it of [lo, hi) into nx x ny x nt cells.
__device__ __forceinline__ CellDev split_cell(const CellDev& p, int nx, int ny, int nt, int j) {
  const int i[3] = {j / (ny * nt), (j / nt) % ny, j % nt};
  const int n[3] = {nx, ny, nt};
  CellDev q;
  q.type = p.type;
  q.face = p.face;
  for (int k = 0; k < 3; ++k) {
    const float step = (p.hi[k] - p.lo[k]) / (float)n[k];
    q.lo[k] = p.lo[k] + (float)i[k] * step;
    q.hi[k] = p.lo[k] + (float)(i[k] + 1) * step;
  }
  return q;
}

__global__ void k_contact_enumerate(ContactDev C, const CellDev* __restrict__ cells, int P, int nx, int ny, int nt,
                                    float* __restrict__ poses) {
  const int n = nx * ny * nt;
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (long long)P * n) return;
  const int p = (int)(id / n), j = (int)(id - (long long)p * n);
  const CellDev q = split_cell(cells[p], nx, ny, nt, j);
  contact_pose(C, C.faces[6 * q.type + q.face], 0.5f * (q.lo[0] + q.hi[0]), 0.5f * (q.lo[1] + q.hi[1]),
               0.5f * (q.lo[2] + q.hi[2]), poses + 16 * id);
}

hipError_t launch_contact_enumerate(const ContactDev& C, const CellDev* cells, int P, int nx, int ny, int nt,
                                    float* poses, hipStream_t st) {
  const long long n = (long long)P * nx * ny * nt;
  hipLaunchKernelGGL(k_contact_enumerate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C, cells, P, nx, ny,
                     nt, poses);
  return hipGetLastError();
}

__global__ void k_contact_choose(const CellDev* __restrict__ roots, int nx, int ny, int nt, const int* __restrict__ idx,
                                 const float* __restrict__ logw, int M, CellDev* __restrict__ cells,
                                 double* __restrict__ clogq, int* __restrict__ choice) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int n = idx[m], ns = nx * ny * nt;
  const CellDev parent = roots ? roots[n / ns] : cells[m];
  cells[m] = split_cell(parent, nx, ny, nt, roots ? n % ns : n);
  clogq[m] = (roots ? 0.0 : clogq[m]) + (double)logw[m];
  if (choice) choice[m] = n;
}

hipError_t launch_contact_choose(const CellDev* roots, int nx, int ny, int nt, const int* idx, const float* logw, int M,
                                 CellDev* cells, double* clogq, int* choice, hipStream_t st) {
  hipLaunchKernelGGL(k_contact_choose, dim3((M + 63) / 64), dim3(64), 0, st, roots, nx, ny, nt, idx, logw, M, cells,
                     clogq, choice);
  return hipGetLastError();
}

__global__ void k_contact_draw(ContactDev C, const CellDev* __restrict__ cells, int M, uint32_t k0, uint32_t k1,
                               uint32_t i, const double* __restrict__ clogq, float* __restrict__ dphi,
                               float* __restrict__ poses, double* __restrict__ logq) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const CellDev q = cells[m];
  U4 c = {(uint32_t)m, i, 0u, 2u};
  const U4 o = philox4x32_10(c, k0, k1);
  const float u[3] = {to_unit(o.x), to_unit(o.y), to_unit(o.z)};
  float x[3];
  double vol = 1.0;
  for (int k = 0; k < 3; ++k) {
    x[k] = q.lo[k] + u[k] * (q.hi[k] - q.lo[k]);
    vol *= (double)q.hi[k] - (double)q.lo[k];
    dphi[3 * m + k] = x[k];
  }
  logq[m] = clogq[m] - log(vol);
  contact_pose(C, C.faces[6 * q.type + q.face], x[0], x[1], x[2], poses + 16 * (size_t)m);
}

hipError_t launch_contact_draw(const ContactDev& C, const CellDev* cells, int M, uint32_t key0, uint32_t key1,
                               uint32_t i, const double* clogq, float* dphi, float* poses, double* logq,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_contact_draw, dim3((M + 63) / 64), dim3(64), 0, st, C, cells, M, key0, key1, i, clogq, dphi,
                     poses, logq);
  return hipGetLastError();
}

__global__ void k_noise_draw(const int* __restrict__ nidx, const float* __restrict__ nlogw, int M, int A, int B,
                             float sigma_max, uint32_t k0, uint32_t k1, uint32_t i, float* __restrict__ noise,
                             double* __restrict__ logq) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int k = nidx[m], a = k / B, b = k - (k / B) * B;
  U4 c = {(uint32_t)m, i, 1u, 2u};
  const U4 o = philox4x32_10(c, k0, k1);
  noise[2 * m] = sigma_max * ((float)a + to_unit(o.x)) / (float)A;
  noise[2 * m + 1] = ((float)b + to_unit(o.y)) / (float)B;
  logq[m] += (double)nlogw[m] - log((double)sigma_max / ((double)A * B));
}

hipError_t launch_noise_draw(const int* nidx, const float* nlogw, int M, int A, int B, float sigma_max,
                             uint32_t key0, uint32_t key1, uint32_t i, float* noise, double* logq, hipStream_t st) {
  hipLaunchKernelGGL(k_noise_draw, dim3((M + 63) / 64), dim3(64), 0, st, nidx, nlogw, M, A, B, sigma_max, key0, key1,
                     i, noise, logq);
  return hipGetLastError();
}

// Block m: the posterior over type of particle m's stage-0 cells, marginal
// over face and placement: post[m][o] = sum over type o's cells of
// exp(logL - LSE), the cells of type o being [o per_type, (o + 1) per_type).
__global__ __launch_bounds__(kBlock) void k_type_posterior(const float* __restrict__ logL, int N, int n_types,
                                                           int per_type, float* __restrict__ post) {
  __shared__ double red[kBlock];
  const float* L = logL + (size_t)blockIdx.x * N;
  double mx = -INFINITY;
  for (int n = threadIdx.x; n < N; n += kBlock) mx = fmax(mx, (double)L[n]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  __shared__ double typ[kMaxTypes];
  for (int o = 0; o < n_types; ++o) {
    double s = 0.0;
    for (int n = o * per_type + threadIdx.x; n < (o + 1) * per_type; n += kBlock) s += exp((double)L[n] - mx);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) typ[o] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int o = 0; o < n_types; ++o) tot += typ[o];
    for (int o = 0; o < n_types; ++o) post[(size_t)blockIdx.x * n_types + o] = (float)(typ[o] / tot);
  }
}

hipError_t launch_type_posterior(const float* logL, int M, int N, int n_types, int per_type, float* post,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_type_posterior, dim3(M), dim3(kBlock), 0, st, logL, N, n_types, per_type, post);
  return hipGetLastError();
}

// Fixed-order block reductions of doubles (whole block, kBlock threads).
__device__ double block_max_d(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_sum_d(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kBlock) void k_smc_reweight(ContactDev C, int M, int i, double log_smax, PartDev in,
                                                         StageDev sd, float* __restrict__ lw_shift) {
  __shared__ double red[kBlock];
  double mx = -INFINITY;
  for (int m = threadIdx.x; m < M; m += kBlock) {
    const CellDev q = sd.cells[m];
    const double lpr = in.lprior[m] + C.faces[6 * q.type + q.face].lprior;
    const double lp = (double)sd.logL[m] + lpr - log_smax;
    const double back = i > 1 ? -log_smax : 0.0;
    const double lw = in.logW[m] + lp - in.logp[m] - sd.logq[m] + back;
    sd.lprior[m] = lpr;
    sd.logp[m] = lp;
    sd.logW_pre[m] = lw;
    mx = fmax(mx, lw);
  }
  mx = block_max_d(mx, red);
  for (int m = threadIdx.x; m < M; m += kBlock) lw_shift[m] = (float)(sd.logW_pre[m] - mx);
}

hipError_t launch_smc_reweight(const ContactDev& C, int M, int i, double log_sigma_max, const PartDev& in,
                               const StageDev& sd, float* lw_shift, hipStream_t st) {
  hipLaunchKernelGGL(k_smc_reweight, dim3(1), dim3(kBlock), 0, st, C, M, i, log_sigma_max, in, sd, lw_shift);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_smc_resample(int M, int n, int k, float threshold, PartDev in,
                                                         StageDev sd, const int* __restrict__ drawn, PartDev out,
                                                         int* __restrict__ ancestors, double* __restrict__ ess) {
  __shared__ double red[kBlock];
  double mx = -INFINITY;
  for (int m = threadIdx.x; m < M; m += kBlock) mx = fmax(mx, sd.logW_pre[m]);
  mx = block_max_d(mx, red);
  double s1 = 0.0, s2 = 0.0;
  for (int m = threadIdx.x; m < M; m += kBlock) {
    const double e = exp(sd.logW_pre[m] - mx);
    s1 += e;
    s2 += e * e;
  }
  s1 = block_sum_d(s1, red);
  s2 = block_sum_d(s2, red);
  const double e_ss = s1 * s1 / s2;
  const bool resample = e_ss < (double)threshold * M;
  const double mean_lw = mx + log(s1) - log((double)M);
  for (int m = threadIdx.x; m < M; m += kBlock) {
    const int src = resample ? drawn[m] : m;
    ancestors[m] = src;
    for (int j = 0; j < k; ++j) {
      const size_t a = (size_t)src * n + j, b = (size_t)m * n + j;
      for (int e = 0; e < 2; ++e) out.place[2 * b + e] = in.place[2 * a + e];
      for (int e = 0; e < 3; ++e) out.dphi[3 * b + e] = in.dphi[3 * a + e];
      for (int e = 0; e < 16; ++e) out.poses[16 * b + e] = in.poses[16 * a + e];
    }
    const size_t b = (size_t)m * n + k;
    out.place[2 * b] = sd.cells[src].type;
    out.place[2 * b + 1] = sd.cells[src].face;
    for (int e = 0; e < 3; ++e) out.dphi[3 * b + e] = sd.dphi[3 * src + e];
    for (int e = 0; e < 16; ++e) out.poses[16 * b + e] = sd.poses[16 * (size_t)src + e];
    out.noise[2 * m] = sd.noise[2 * src];
    out.noise[2 * m + 1] = sd.noise[2 * src + 1];
    out.logL[m] = sd.logL[src];
    out.logp[m] = sd.logp[src];
    out.lprior[m] = sd.lprior[src];
    out.logW[m] = resample ? mean_lw : sd.logW_pre[m];
  }
  if (threadIdx.x == 0) *ess = e_ss;
}

hipError_t launch_smc_resample(int M, int n_slots, int k, float threshold, const PartDev& in, const StageDev& sd,
                               const int* drawn, PartDev out, int* ancestors, double* ess, hipStream_t st) {
  hipLaunchKernelGGL(k_smc_resample, dim3(1), dim3(kBlock), 0, st, M, n_slots, k, threshold, in, sd, drawn, out,
                     ancestors, ess);
  return hipGetLastError();
}

}  // namespace b3d

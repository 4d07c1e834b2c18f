// Fused render + windowed likelihood (+ adjoint), one workgroup per pose
// hypothesis.  Nothing but the per-hypothesis results leaves the CU:
//   1. the object's conservative pixel rectangle under the pose is found;
//   2. an LDS depth/id buffer covering that rectangle plus twice the window
//      half-width is initialised from the static background and the mesh is
//      rasterised into it (cluster by cluster, vertices transformed once into
//      LDS, 64-bit atomicMin on packed (depth, id) keys);
//   3. every observed pixel whose window can see the object evaluates eq. (1)
//      over its window, reading rendered depths from LDS and turning them into
//      points on their pixel rays;
//   4. (adjoint) the window weights b/L_i are kept in LDS and every object
//      pixel gathers d logL/d z_j over its window, then maps it through the
//      ray/plane intersection of its triangle onto (dt, dw);
//   5. pixels whose window cannot see the object contribute their
//      background-only terms, read from double-precision summed-area tables.
// When the rectangle does not fit the LDS budget it is processed in bands of
// rows, re-rasterising per band.
#include "b3d_launch.hpp"
#include <type_traits>

namespace b3d {

__device__ __forceinline__ float f_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float f_ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }

__device__ __forceinline__ double rect_sum(const double* sat, int W, const Rect& r) {
  if (r.empty()) return 0.0;
  const int p = W + 1;
  return sat[(size_t)r.y1 * p + r.x1] - sat[(size_t)r.y0 * p + r.x1] - sat[(size_t)r.y1 * p + r.x0] +
         sat[(size_t)r.y0 * p + r.x0];
}

// LDS: rasteriser scratch (once the depth buffer is complete: the window
// weights, then the drawn-pixel list) | depth keys [zcap] | reduction [64] |
// ray tables of columns [-2h, W + 2h) and rows [-2h, H + 2h).
size_t fused_lds_bytes(const SceneDev& s) {
  return kRasterLdsBytes + sizeof(float) * (64 + s.cam.W + s.cam.H + 8 * s.sc.h) + kFusedBytesPerKey * (size_t)s.zcap;
}

// One round of block-wide stream compaction: the threads whose flag is set
// append their value to list[n ...] in thread order; returns how many did.
// Whole block; `wcnt` holds kWaves ints of LDS.
__device__ __forceinline__ int append_flagged(bool flag, int value, unsigned short* __restrict__ list, int n,
                                              int* wcnt) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  if (lane == 0) wcnt[wave] = __popcll(m);
  __syncthreads();
  int off = n, sum = 0;
  for (int w = 0; w < kWaves; ++w) {
    off += w < wave ? wcnt[w] : 0;
    sum += wcnt[w];
  }
  if (flag) list[off + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned short)value;
  __syncthreads();
  return sum;
}

// Row-major list of the buffer slots [k0, k1) that hold a surface of the mesh
// (triangle id < T); returns its length.  Whole block.
__device__ __forceinline__ int list_drawn(const unsigned long long* __restrict__ zbuf, int k0, int k1, uint32_t T,
                                          unsigned short* __restrict__ list, int* wcnt) {
  int n = 0;
  for (int base = k0; base < k1; base += kBlock) {
    const int k = base + (int)threadIdx.x;
    n += append_flagged(k < k1 && key_id(zbuf[k]) < T, k, list, n, wcnt);
  }
  return n;
}

// Window sums for observed point (ox, oy, oz) at pixel (r, c) over the LDS
// depth rectangle L (pitch lw), which holds the whole window (positions
// outside the image are empty slots): S = sum_j exp(-D_ij/(2 sigma^2)) and
// T = sum_j exp(-D_ij/(2 sigma^2)) D_ij over the rendered points of the
// window.  HH > 0: the window half-width known at compile time, each row
// unrolled and branch-free: an empty slot's far depth makes its term exactly
// 0.  HH = 0: any h, empty slots skipped.
template <int HH, bool GRAD, bool COUNT>
__device__ __forceinline__ void window_sums(const unsigned long long* __restrict__ zbuf, const Rect& L, int lw,
                                            const float* __restrict__ dxt, const float* __restrict__ dyt, int r,
                                            int c, int h, float ox, float oy, float oz, float c2, float& S, float& T,
                                            unsigned& pairs) {
  S = 0.0f;
  T = 0.0f;
  if (HH > 0) {
    constexpr int n = 2 * HH + 1;
    float dxs[n];
#pragma unroll
    for (int k = 0; k < n; ++k) dxs[k] = dxt[c - HH + k];
    const unsigned long long* zr = zbuf + (r - HH - L.y0) * lw + (c - HH - L.x0);
#pragma unroll 1
    for (int j = 0; j < n; ++j, zr += lw) {
      const float dy = dyt[r - HH + j];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const unsigned long long key = zr[k];
        const float z = key_depth(key);
        const float ex = ox - z * dxs[k], ey = oy - z * dy, ez = oz - z;
        const float D = ex * ex + ey * ey + ez * ez;
        const float e = f_exp2(-D * c2);
        S += e;
        if (GRAD) T += e * D;
        if (COUNT) pairs += key != kEmptyKey ? 1u : 0u;
      }
    }
  } else {
    const int r0 = max(r - h, L.y0), r1 = min(r + h, L.y1 - 1);
    const int c0 = max(c - h, L.x0), c1 = min(c + h, L.x1 - 1);
    for (int rj = r0; rj <= r1; ++rj) {
      const float dy = dyt[rj];
      const unsigned long long* zr = zbuf + (rj - L.y0) * lw - L.x0;
      for (int cj = c0; cj <= c1; ++cj) {
        const unsigned long long key = zr[cj];
        if (key == kEmptyKey) continue;
        const float z = key_depth(key);
        const float ex = ox - z * dxt[cj], ey = oy - z * dy, ez = oz - z;
        const float D = ex * ex + ey * ey + ez * ez;
        const float e = f_exp2(-D * c2);
        S += e;
        if (GRAD) T += e * D;
        if (COUNT) ++pairs;
      }
    }
  }
}

// d logL / d z_j of an object pixel (r, c) with point q = z (dx, dy, 1):
// sum over observed i in its window of w_i exp(-D_ij/(2 sigma^2)) (q~_i - q).d,
// with w_i = b/L_i from the LDS buffer of observed rows [wa, ...) and region
// columns (0 for invalid observed pixels).  Returns the sum before the
// 1/sigma^2 factor.  HH as for window_sums.
template <int HH>
__device__ __forceinline__ float window_grad(const float* __restrict__ wbuf, int wa, int wb, const Rect& region,
                                             const float* __restrict__ obs, int W, int r, int c, int h, float qx,
                                             float qy, float qz, float dx, float dy, float c2) {
  const int rw = region.w();
  float g = 0.0f;
  if (HH > 0) {
    constexpr int n = 2 * HH + 1;
    if (r - HH >= wa && r + HH < wb && c - HH >= region.x0 && c + HH < region.x1) {
      // the whole window inside the weights' rows and the region's columns
      // (every pixel away from the image border): no clamping, one address
      // per window row; the same terms in the same order as below
      const float* wr = wbuf + (r - HH - wa) * rw + (c - HH - region.x0);
      const float* orow = obs + 3 * ((size_t)(r - HH) * W + (c - HH));
#pragma unroll 1
      for (int j = 0; j < n; ++j, wr += rw, orow += 3 * (size_t)W) {
#pragma unroll
        for (int k = 0; k < n; ++k) {
          const float wv = wr[k];
          const float* q = orow + 3 * k;
          const float ex = q[0] - qx, ey = q[1] - qy, ez = q[2] - qz;
          const float e = f_exp2(-(ex * ex + ey * ey + ez * ez) * c2);
          g += wv * e * __builtin_fmaf(ex, dx, __builtin_fmaf(ey, dy, ez));
        }
      }
      return g;
    }
    int cc[n];
    bool cv[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const int ci = c - HH + k;
      cv[k] = ci >= region.x0 && ci < region.x1;
      cc[k] = min(max(ci, region.x0), region.x1 - 1);
    }
#pragma unroll 1
    for (int j = 0; j < n; ++j) {
      const int ri = r - HH + j;
      const bool rv = ri >= wa && ri < wb;
      const int rc = min(max(ri, wa), wb - 1);
      const float* wr = wbuf + (rc - wa) * rw - region.x0;
      const float* orow = obs + 3 * (size_t)rc * W;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const float wv = (rv && cv[k]) ? wr[cc[k]] : 0.0f;
        const float* q = orow + 3 * cc[k];
        const float ex = q[0] - qx, ey = q[1] - qy, ez = q[2] - qz;
        const float e = f_exp2(-(ex * ex + ey * ey + ez * ez) * c2);
        g += wv * e * __builtin_fmaf(ex, dx, __builtin_fmaf(ey, dy, ez));
      }
    }
  } else {
    const int r0 = max(r - h, wa), r1 = min(r + h, wb - 1);
    const int c0 = max(c - h, region.x0), c1 = min(c + h, region.x1 - 1);
    for (int ri = r0; ri <= r1; ++ri) {
      const float* wr = wbuf + (ri - wa) * rw - region.x0;
      for (int ci = c0; ci <= c1; ++ci) {
        const float wv = wr[ci];
        if (wv == 0.0f) continue;
        const float* q = obs + 3 * ((size_t)ri * W + ci);
        const float ex = q[0] - qx, ey = q[1] - qy, ez = q[2] - qz;
        const float e = f_exp2(-(ex * ex + ey * ey + ez * ez) * c2);
        g += wv * e * __builtin_fmaf(ex, dx, __builtin_fmaf(ey, dy, ez));
      }
    }
  }
  return g;
}

// Row r and column c of slot k (0 <= k < 2^20) of a rectangle of width w,
// given inv_w = 1/w correctly rounded: (k + 1/2) inv_w is formed with one
// rounding, a relative error below 2^-22, so it lies within 1/(4w) of
// (k + 1/2)/w, whose fractional part is in [1/(2w), 1 - 1/(2w)]: truncating it
// gives floor(k/w) exactly, with no integer division.
__device__ __forceinline__ void row_col(int k, int w, float inv_w, int& r, int& c) {
  r = (int)__builtin_fmaf((float)k, inv_w, 0.5f * inv_w);
  c = k - __mul24(r, w);
}

// First local index k >= 0 with (base + k) mod kBlock == t.
__device__ __forceinline__ int first_of(unsigned t, int base) {
  return ((int)t - base % kBlock + kBlock) % kBlock;
}

// The depth buffer of one band: the LDS rectangle L (pitch L.w(), rows and
// columns possibly beyond the image, which stay empty) initialised from the
// background keys, the mesh rasterised into its image part, then the depth of
// every slot the mesh drew recomputed on its triangle's plane.  Whole block.
template <bool COUNT, int RM = kRasterAny>
__device__ __forceinline__ void raster_band(const SceneDev& s, const Pose& P, const Rect& L,
                                            unsigned long long* zbuf, unsigned char* smem, float* red, unsigned* cnt) {
  const Cam& cam = s.cam;
  const int H = cam.H, W = cam.W, lw = L.w();
  const int nk = L.h() * lw;
  const float inv_lw = 1.0f / (float)lw;
  for (int k = threadIdx.x; k < nk; k += kBlock) {
    int r, c;
    row_col(k, lw, inv_lw, r, c);
    r += L.y0;
    c += L.x0;
    const bool in = r >= 0 && r < H && c >= 0 && c < W;
    zbuf[k] = (in && s.bg) ? s.bg[(size_t)r * W + c] : kEmptyKey;
  }
  __syncthreads();
  raster_mesh_mode<COUNT, RM>(s.mesh, P, cam, 0u, grow_clip(L, 0, W, H), L, zbuf, carve_raster_lds(smem), cnt);
  // the slots this mesh drew (listed in the free scratch, which holds more
  // entries than the buffer has slots), then their depths on the planes
  unsigned short* rlist = reinterpret_cast<unsigned short*>(smem);
  const int nr = list_drawn(zbuf, 0, nk, (uint32_t)s.mesh.T, rlist, reinterpret_cast<int*>(red));
  for (int k = threadIdx.x; k < nr; k += kBlock) {
    const int off = rlist[k];
    const unsigned long long key = zbuf[off];
    int r, c;
    row_col(off, lw, inv_lw, r, c);
    zbuf[off] = pack_key(plane_depth(s.mesh, P, cam, key_id(key), L.y0 + r, L.x0 + c), key_id(key));
  }
  __syncthreads();
}

// One hypothesis: pose16 (16 floats), writes *logL_out and, when GRAD,
// grad_out[0..8).  Must be called by the whole block; `smem` is at least
// fused_lds_bytes(s).
template <bool GRAD, bool COUNT = false, int RM = kRasterAny>
__device__ __forceinline__ void render_score_one(const SceneDev& s, const float* __restrict__ pose16,
                                                 float* __restrict__ logL_out, float* __restrict__ grad_out,
                                                 unsigned char* smem, unsigned* cnt = nullptr, int row_lo = -1,
                                                 int row_hi = -1) {
  unsigned c_pair = 0, c_obs = 0, c_adj = 0;
  float* wbuf = reinterpret_cast<float*>(smem);  // after rasterisation
  unsigned long long* zbuf = reinterpret_cast<unsigned long long*>(smem + kRasterLdsBytes);
  float* red = reinterpret_cast<float*>(zbuf + s.zcap);

  const Cam& cam = s.cam;
  const ScoreConsts& sc = s.sc;
  const int H = cam.H, W = cam.W, h = sc.h;
  // ray tables indexed by column in [-2h, W + 2h) and row in [-2h, H + 2h)
  float* dxt = red + 64 + 2 * h;
  float* dyt = dxt + W + 4 * h;
  const Pose P = load_pose(pose16);
  for (int i = (int)threadIdx.x - 2 * h; i < W + 2 * h; i += kBlock) dxt[i] = ray_x(cam, i);
  for (int i = (int)threadIdx.x - 2 * h; i < H + 2 * h; i += kBlock) dyt[i] = ray_y(cam, i);

  const Rect obj = object_rect(s.mesh, P, cam);
  // observed pixels whose window can see the object (none when nothing is drawn)
  Rect region = grow_clip(obj, h, W, H);
  if (obj.empty()) region.x1 = region.x0;
  // acc: l, d(dt) x3, d(dw) x3, d sigma, d p_out
  float acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (!obj.empty()) {
    // the depth buffer spans the object rectangle grown by 2h, past the image
    // edges if need be (those slots stay empty), so every window is inside it
    const Rect lds = grow(obj, 2 * h);
    const int lw = lds.w(), rw = region.w();
    const int ow = obj.w();
    int band = s.zcap / lw - 4 * h;
    // the window weights ((band + 2h) x rw floats) leave at least one round
    // (kBlock entries) of the drawn-pixel list in the scratch
    if (GRAD) band = min(band, min(s.wcap, (int)(kRasterLdsBytes - 2 * kBlock) / 4) / rw - 2 * h);
    band = max(band, 1);
    int gcarry = 0;  // drawn pixels of earlier bands' own rows
    // with a row range: only the region's rows in [row_lo, row_hi) (the
    // adjoint's weights still span the whole region's halo rows)
    const int ya = row_lo >= 0 ? max(region.y0, row_lo) : region.y0;
    const int yb = row_lo >= 0 ? min(region.y1, row_hi) : region.y1;
    for (int a = ya; a < yb; a += band) {
      const int b = min(a + band, yb);
      Rect L = lds;
      L.y0 = a - 2 * h;
      L.y1 = b + 2 * h;
      raster_band<COUNT, RM>(s, P, L, zbuf, smem, red, cnt);
      // likelihood over observed rows [wa, wb); rows [a, b) are this band's own
      const int wa = GRAD ? max(a - h, region.y0) : a;
      const int wb = GRAD ? min(b + h, region.y1) : b;
      const int nw = (wb - wa) * rw;

      // pixel g of the region (row-major from its corner) always goes to
      // thread g mod kBlock, so every thread adds its terms in the same order
      // however the rows are banded: results do not depend on the band height
      const float inv_rw = 1.0f / (float)rw;
      for (int k = first_of(threadIdx.x, (wa - region.y0) * rw); k < nw; k += kBlock) {
        int r, c;
        row_col(k, rw, inv_rw, r, c);
        r += wa;
        c += region.x0;
        const float* q = s.obs + 3 * ((size_t)r * W + c);
        const float ox = q[0], oy = q[1], oz = q[2];
        float wv = 0.0f;
        if (oz > 0.0f) {
          float S, T;
          unsigned pairs = 0;
          switch (h) {
            case 1:
              window_sums<1, GRAD, COUNT>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, sc.c2, S, T, pairs);
              break;
            case 2:
              window_sums<2, GRAD, COUNT>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, sc.c2, S, T, pairs);
              break;
            default:
              window_sums<0, GRAD, COUNT>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, sc.c2, S, T, pairs);
          }
          if (COUNT && r >= a && r < b) c_pair += pairs;
          const float Li = sc.a + sc.bn * S;
          const float iL = __builtin_amdgcn_rcpf(Li);  // 1 / L_i, hardware reciprocal (1 ulp)
          const float bL = sc.bn * iL;
          if (r >= a && r < b) {
            if (COUNT && S > 0.0f) ++c_obs;
            acc[0] += f_ln(Li);
            if (GRAD) {
              acc[7] += bL * (T * sc.inv_s3 - 3.0f * S * sc.inv_s);
              acc[8] += (sc.invV - sc.normM * S) * iL;
            }
          }
          wv = bL;
        }
        if (GRAD) wbuf[k] = wv;
      }

      if (GRAD) {
        __syncthreads();
        // d logL / d z_j of drawn pixel (r, c) over its window, onto (dt, dw)
        auto gather = [&](int r, int c, unsigned long long key) {
          const uint32_t id = key_id(key);
          if (COUNT) ++c_adj;
          const float z = key_depth(key);
          const float dx = dxt[c], dy = dyt[r];
          const float qx = z * dx, qy = z * dy, qz = z;
          float g;
          switch (h) {
            case 1:
              g = window_grad<1>(wbuf, wa, wb, region, s.obs, W, r, c, h, qx, qy, qz, dx, dy, sc.c2);
              break;
            case 2:
              g = window_grad<2>(wbuf, wa, wb, region, s.obs, W, r, c, h, qx, qy, qz, dx, dy, sc.c2);
              break;
            default:
              g = window_grad<0>(wbuf, wa, wb, region, s.obs, W, r, c, h, qx, qy, qz, dx, dy, sc.c2);
          }
          g *= sc.inv_s2;
          const float4 no = s.mesh.normals[id];
          const float3 nn = rotate(P, no.x, no.y, no.z);
          const float sg = g * __builtin_amdgcn_rcpf(nn.x * dx + nn.y * dy + nn.z);
          const float tx = P.t[0] - qx, ty = P.t[1] - qy, tz = P.t[2] - qz;
          acc[1] += sg * nn.x;
          acc[2] += sg * nn.y;
          acc[3] += sg * nn.z;
          acc[4] += sg * (nn.y * tz - nn.z * ty);
          acc[5] += sg * (nn.z * tx - nn.x * tz);
          acc[6] += sg * (nn.x * ty - nn.y * tx);
        };
        // the drawn pixels of this band's own rows, listed chunk by chunk in the
        // scratch after the window weights; the i-th of them over all bands and
        // chunks (row-major) goes to thread i mod kBlock, so each thread's
        // order does not depend on banding
        const int ga = max(a, obj.y0), gb = min(b, obj.y1);
        const int ng = max(gb - ga, 0) * ow;
        const float inv_ow = 1.0f / (float)ow;
        unsigned short* glist = reinterpret_cast<unsigned short*>(smem + 4 * nw);
        const int gcap = ((int)kRasterLdsBytes - 4 * nw) / 2;
        for (int pos = 0; pos < ng;) {
          int n = 0;
          // compaction rounds while a whole round still fits
          for (; pos < ng && n + kBlock <= gcap; pos += kBlock) {
            const int k = pos + (int)threadIdx.x;
            bool d = false;
            if (k < ng) {
              int r, c;
              row_col(k, ow, inv_ow, r, c);
              r += ga;
              c += obj.x0;
              d = key_id(zbuf[(r - L.y0) * lw + (c - L.x0)]) < (uint32_t)s.mesh.T;
            }
            n += append_flagged(d, k, glist, n, reinterpret_cast<int*>(red));
          }
          for (int i = first_of(threadIdx.x, gcarry); i < n; i += kBlock) {
            int r, c;
            row_col(glist[i], ow, inv_ow, r, c);
            r += ga;
            c += obj.x0;
            gather(r, c, zbuf[(r - L.y0) * lw + (c - L.x0)]);
          }
          gcarry += n;
          __syncthreads();  // the list is rewritten by the next chunk
        }
      }
      __syncthreads();
    }
  }
  if (COUNT) {
    atomicAdd(&cnt[kCntPair], c_pair);
    atomicAdd(&cnt[kCntObs], c_obs);
    atomicAdd(&cnt[kCntAdj], c_adj);
  }
  block_sum<9>(acc, red);
  if (row_lo >= 0) {  // the rows' own terms only, no background outside the region
    if (threadIdx.x == 0) {
      *logL_out = acc[0];
      if (GRAD)
        for (int k = 0; k < 8; ++k) grad_out[k] = acc[1 + k];
    }
    return;
  }
  if (threadIdx.x == 0) {
    const size_t stride = (size_t)(H + 1) * (W + 1);
    Rect all;
    all.x0 = 0;
    all.x1 = W;
    all.y0 = 0;
    all.y1 = H;
    const double outside_l = rect_sum(s.sat, W, all) - rect_sum(s.sat, W, region);
    *logL_out = (float)((double)acc[0] + outside_l);
    if (GRAD) {
      const double outside_dp = rect_sum(s.sat + stride, W, all) - rect_sum(s.sat + stride, W, region);
      const double outside_ds = rect_sum(s.sat + 2 * stride, W, all) - rect_sum(s.sat + 2 * stride, W, region);
      float* g = grad_out;
      for (int k = 0; k < 6; ++k) g[k] = acc[1 + k];
      g[6] = (float)((double)acc[7] + outside_ds);
      g[7] = (float)((double)acc[8] + outside_dp);
    }
  }
}

// RM: the rasteriser compiled in (the launcher picks it from the mesh, so
// that meshes without large primitives run the plain one alone).
template <bool GRAD, int RM>
__global__ __launch_bounds__(kBlock, 4) void k_render_score(SceneDev s, const float* __restrict__ poses, int N,
                                                         float* __restrict__ logL, float* __restrict__ grad) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = blockIdx.x;
  if (n >= N) return;
  render_score_one<GRAD, false, RM>(s, poses + 16 * (size_t)n, logL + n, GRAD ? grad + 8 * (size_t)n : nullptr,
                                    smem);
}

// A group of scenes in one launch, one workgroup per (scene, hypothesis)
// item.  Items are numbered scene by scene in the order the host chose
// (costliest hypotheses first), so the expensive scenes start early and the
// cheap ones fill the tail; the hardware dispatcher hands them out in order.
// The item's scene is copied from the argument member by member at constant
// positions: indexing the argument with the scene number would move it to
// scratch memory.  No static LDS either, which would cost a resident block
// per CU at the default tile.
template <bool GRAD, int RM>
__global__ __launch_bounds__(kBlock, 4) void k_batch(const BatchGroupDev G) {
  extern __shared__ __align__(16) unsigned char smem[];
  const long long w = blockIdx.x;
  if (w >= G.first[G.S]) return;
  int k = 0;
  for (int j = 1; j < G.S; ++j) k = G.first[j] <= w ? j : k;
  SceneDev s;
  const float* poses = nullptr;
  float *logL = nullptr, *grad = nullptr;
  long long first = 0;
#pragma unroll
  for (int j = 0; j < kBatchGroup; ++j)
    if (k == j) {
      s = G.s[j];
      poses = G.poses[j];
      logL = G.logL[j];
      grad = G.grad[j];
      first = G.first[j];
    }
  const long long n = w - first;
  render_score_one<GRAD, false, RM>(s, poses + 16 * n, logL + n, GRAD ? grad + 8 * n : nullptr, smem);
}

hipError_t launch_batch(const BatchGroupDev& g, bool grad, size_t lds, hipStream_t st) {
  bool big = false;
  for (int k = 0; k < g.S; ++k) big = big || g.s[k].mesh.has_big != 0;
  const dim3 grid((unsigned)g.first[g.S]);
  if (grad && big)
    hipLaunchKernelGGL((k_batch<true, kRasterAny>), grid, dim3(kBlock), lds, st, g);
  else if (grad)
    hipLaunchKernelGGL((k_batch<true, kRasterSmall>), grid, dim3(kBlock), lds, st, g);
  else if (big)
    hipLaunchKernelGGL((k_batch<false, kRasterAny>), grid, dim3(kBlock), lds, st, g);
  else
    hipLaunchKernelGGL((k_batch<false, kRasterSmall>), grid, dim3(kBlock), lds, st, g);
  return hipGetLastError();
}

// The same work drained by a persistent grid instead: as many workgroups as
// fit the chip, each pulling the next item from a device counter (reset by
// a one-thread kernel, not a memset, so that launches can be captured) and
// exiting once the counter passes the group's total.  Its loop keeps more
// state live (some of it spills) and `work` takes static LDS, so it loses
// where items are short, but it keeps every slot busy to the end of long
// launches of long items.
template <bool GRAD, int RM>
__global__ __launch_bounds__(kBlock, 4) void k_batch_queue(const BatchGroupDev G,
                                                           unsigned long long* __restrict__ counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ long long work;
  const long long total = G.first[G.S];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) work = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    // the same value in every lane: keep it (and the scene it selects) scalar
    const unsigned long long wr = (unsigned long long)work;
    const long long w = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(wr >> 32)) << 32) |
                                    (unsigned)__builtin_amdgcn_readfirstlane((unsigned)wr));
    if (w >= total) break;
    int k = 0;
    for (int j = 1; j < G.S; ++j) k = G.first[j] <= w ? j : k;
    const long long n = w - G.first[k];
    render_score_one<GRAD, false, RM>(G.s[k], G.poses[k] + 16 * n, G.logL[k] + n, GRAD ? G.grad[k] + 8 * n : nullptr,
                                      smem);
  }
}

__global__ void k_reset_counter(unsigned long long* c) {
  if (threadIdx.x == 0) c[threadIdx.x] = 0ull;
}

hipError_t batch_queue_occupancy(bool grad, size_t lds, int* blocks_per_cu) {
  // every raster variant has the same launch bounds and LDS
  if (grad)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_queue<true, kRasterSmall>, kBlock, lds);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_batch_queue<false, kRasterSmall>, kBlock, lds);
}

hipError_t launch_batch_queue(const BatchGroupDev& g, unsigned long long* counter, bool grad, size_t lds, int blocks,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
  bool big = false;
  for (int k = 0; k < g.S; ++k) big = big || g.s[k].mesh.has_big != 0;
  if (grad && big)
    hipLaunchKernelGGL((k_batch_queue<true, kRasterAny>), dim3(blocks), dim3(kBlock), lds, st, g, counter);
  else if (grad)
    hipLaunchKernelGGL((k_batch_queue<true, kRasterSmall>), dim3(blocks), dim3(kBlock), lds, st, g, counter);
  else if (big)
    hipLaunchKernelGGL((k_batch_queue<false, kRasterAny>), dim3(blocks), dim3(kBlock), lds, st, g, counter);
  else
    hipLaunchKernelGGL((k_batch_queue<false, kRasterSmall>), dim3(blocks), dim3(kBlock), lds, st, g, counter);
  return hipGetLastError();
}

// n_refine Adam steps on each of N poses of a scene, one workgroup per pose:
// the fused render + score + adjoint, then the update, with the pose kept in
// LDS between steps (the same arithmetic as render_score + adam_pose launched
// in turn, starting from zero moments).
__global__ __launch_bounds__(kBlock) void k_refine_pose(SceneDev s, float* __restrict__ poses, int N, int n_refine,
                                                        float lr_t, float lr_r, float b1, float b2, float eps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float P[16];
  __shared__ float g[8];
  __shared__ float L;
  const int n = blockIdx.x;
  if (n >= N) return;
  float* pose = poses + 16 * (size_t)n;
  float m[6] = {0, 0, 0, 0, 0, 0}, v[6] = {0, 0, 0, 0, 0, 0};  // used by thread 0
  if (threadIdx.x < 16) P[threadIdx.x] = pose[threadIdx.x];
  __syncthreads();
  for (int it = 1; it <= n_refine; ++it) {
    render_score_one<true>(s, P, &L, g, smem);
    if (threadIdx.x == 0) adam_update(P, g, m, v, it, lr_t, lr_r, b1, b2, eps);
    __syncthreads();
  }
  if (threadIdx.x < 16) pose[threadIdx.x] = P[threadIdx.x];
}

hipError_t launch_refine_pose(const SceneDev& s, float* poses, int N, int n_refine, float lr_t, float lr_r, float b1,
                              float b2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_pose, dim3(N), dim3(kBlock), fused_lds_bytes(s), st, s, poses, N, n_refine, lr_t,
                     lr_r, b1, b2, eps);
  return hipGetLastError();
}

// One Adam step of one pose spread over row bands: block b scores the image
// rows [b R, (b + 1) R) of the pose's region (render, windows, adjoint) and
// writes its terms to partial[9 b .. 9 b + 9) (logL, d(dt, dw), d sigma,
// d p_out, without the background outside the region, which the pose
// gradient does not involve).
template <int RM>
__global__ __launch_bounds__(kBlock, 4) void k_refine_bands(SceneDev s, const float* __restrict__ pose, int R,
                                                            float* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  render_score_one<true, false, RM>(s, pose, partial + 9 * b, partial + 9 * b + 1, smem, nullptr, b * R,
                                    (b + 1) * R);
}

// The band sums in band order (double), then the Adam update of the pose;
// the moments live in state[0..12) (zero at iter 1).  One thread.
__global__ void k_refine_update(float* __restrict__ pose, const float* __restrict__ partial, int nb,
                                float* __restrict__ state, int iter, float lr_t, float lr_r, float b1, float b2,
                                float eps) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float g[6], m[6], v[6], P[16];
  for (int k = 0; k < 6; ++k) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += (double)partial[9 * b + 1 + k];
    g[k] = (float)t;
    m[k] = iter == 1 ? 0.0f : state[k];
    v[k] = iter == 1 ? 0.0f : state[6 + k];
  }
  for (int k = 0; k < 16; ++k) P[k] = pose[k];
  adam_update(P, g, m, v, iter, lr_t, lr_r, b1, b2, eps);
  for (int k = 0; k < 16; ++k) pose[k] = P[k];
  for (int k = 0; k < 6; ++k) {
    state[k] = m[k];
    state[6 + k] = v[k];
  }
}

hipError_t launch_refine_banded(const SceneDev& s, float* pose, int n_refine, float lr_t, float lr_r, float b1,
                                float b2, float eps, int R, float* partial, float* state, hipStream_t st) {
  const int nb = (s.cam.H + R - 1) / R;
  for (int it = 1; it <= n_refine; ++it) {
    if (s.mesh.has_big)
      hipLaunchKernelGGL(k_refine_bands<kRasterBig>, dim3(nb), dim3(kBlock), fused_lds_bytes(s), st, s, pose, R,
                         partial);
    else
      hipLaunchKernelGGL(k_refine_bands<kRasterSmall>, dim3(nb), dim3(kBlock), fused_lds_bytes(s), st, s, pose, R,
                         partial);
    hipLaunchKernelGGL(k_refine_update, dim3(1), dim3(64), 0, st, pose, partial, nb, state, it, lr_t, lr_r, b1, b2,
                       eps);
  }
  return hipGetLastError();
}

// Window sums under each deviation of a noise grid: S[a] = sum_j
// exp(-D_ij c2[a]) over the rendered points of the window of observed point
// (ox, oy, oz) at pixel (r, c) (as window_sums, with each distance computed
// once).  NA > 0: the grid's number of deviations known at compile time (no
// exponential for the unused ones); NA = 0: any number up to kMaxSigma.
template <int HH, int NA>
__device__ __forceinline__ void window_sums_grid(const unsigned long long* __restrict__ zbuf, const Rect& L, int lw,
                                                 const float* __restrict__ dxt, const float* __restrict__ dyt, int r,
                                                 int c, int h, float ox, float oy, float oz, const NoiseGridDev& g,
                                                 float (&S)[kMaxSigma]) {
#pragma unroll
  for (int a = 0; a < kMaxSigma; ++a) S[a] = 0.0f;
  auto add = [&](float D) {
#pragma unroll
    for (int a = 0; a < (NA > 0 ? NA : kMaxSigma); ++a)
      if (NA > 0 || a < g.A) S[a] += f_exp2(-D * g.c2[a]);
  };
  if (HH > 0) {
    constexpr int n = 2 * HH + 1;
    float dxs[n];
#pragma unroll
    for (int k = 0; k < n; ++k) dxs[k] = dxt[c - HH + k];
    const unsigned long long* zr = zbuf + (r - HH - L.y0) * lw + (c - HH - L.x0);
#pragma unroll 1
    for (int j = 0; j < n; ++j, zr += lw) {
      const float dy = dyt[r - HH + j];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const float z = key_depth(zr[k]);
        const float ex = ox - z * dxs[k], ey = oy - z * dy, ez = oz - z;
        add(ex * ex + ey * ey + ez * ez);
      }
    }
  } else {
    const int r0 = max(r - h, L.y0), r1 = min(r + h, L.y1 - 1);
    const int c0 = max(c - h, L.x0), c1 = min(c + h, L.x1 - 1);
    for (int rj = r0; rj <= r1; ++rj) {
      const float dy = dyt[rj];
      const unsigned long long* zr = zbuf + (rj - L.y0) * lw - L.x0;
      for (int cj = c0; cj <= c1; ++cj) {
        const unsigned long long key = zr[cj];
        if (key == kEmptyKey) continue;
        const float z = key_depth(key);
        const float ex = ox - z * dxt[cj], ey = oy - z * dy, ez = oz - z;
        add(ex * ex + ey * ey + ez * ez);
      }
    }
  }
}

// logL of one hypothesis under every point of the noise grid (grid_out[k],
// k = a * B + b) and their weighted log-sum-exp (*marg_out).  The same
// render and windows as render_score_one; each observed pixel's window
// distances are computed once and exponentiated per deviation.  With
// row0 >= 0 the block instead scores the full-width image rows [row0, row1)
// (their pixels only, no background table) and grid_out[k] receives the
// block's sum for grid point k; marg_out is not written.  Whole block.
__device__ __forceinline__ void render_score_grid_one(const SceneDev& s, const NoiseGridDev& g,
                                                      const float* __restrict__ pose16, float* __restrict__ grid_out,
                                                      float* __restrict__ marg_out, unsigned char* smem, int row0,
                                                      int row1) {
  unsigned long long* zbuf = reinterpret_cast<unsigned long long*>(smem + kRasterLdsBytes);
  float* red = reinterpret_cast<float*>(zbuf + s.zcap);
  float* sbuf = reinterpret_cast<float*>(smem);  // per thread: S[a] normM[a] (raster scratch, free by then)
  const Cam& cam = s.cam;
  const int H = cam.H, W = cam.W, h = s.sc.h;
  float* dxt = red + 64 + 2 * h;
  float* dyt = dxt + W + 4 * h;
  const Pose P = load_pose(pose16);
  for (int i = (int)threadIdx.x - 2 * h; i < W + 2 * h; i += kBlock) dxt[i] = ray_x(cam, i);
  for (int i = (int)threadIdx.x - 2 * h; i < H + 2 * h; i += kBlock) dyt[i] = ray_y(cam, i);
  const bool rows = row0 >= 0;
  Rect all;
  all.x0 = 0;
  all.x1 = W;
  all.y0 = 0;
  all.y1 = H;
  Rect obj = all;
  if (rows) {
    obj.y0 = row0;
    obj.y1 = row1;
  } else {
    obj = object_rect(s.mesh, P, cam);
  }
  Rect region = rows ? obj : grow_clip(obj, h, W, H);
  if (obj.empty()) region.x1 = region.x0;
  const int nk_grid = g.A * g.B;
  float acc[kMaxNoise];
#pragma unroll
  for (int k = 0; k < kMaxNoise; ++k) acc[k] = 0.0f;
  if (!obj.empty()) {
    const Rect lds = grow(obj, 2 * h);
    const int lw = lds.w(), rw = region.w();
    const int band = max(s.zcap / lw - 4 * h, 1);
    for (int a = region.y0; a < region.y1; a += band) {
      const int b = min(a + band, region.y1);
      Rect L = lds;
      L.y0 = a - 2 * h;
      L.y1 = b + 2 * h;
      raster_band<false>(s, P, L, zbuf, smem, red, nullptr);
      const int nw = (b - a) * rw;
      // observed pixel g of the region always goes to thread g mod kBlock;
      // na: the grid's number of deviations as a compile-time constant (0: any)
      const float inv_rw = 1.0f / (float)rw;
      auto pixels = [&](auto na) {
        constexpr int NA = decltype(na)::value;
        for (int k = first_of(threadIdx.x, (a - region.y0) * rw); k < nw; k += kBlock) {
          int r, c;
          row_col(k, rw, inv_rw, r, c);
          r += a;
          c += region.x0;
          const float* q = s.obs + 3 * ((size_t)r * W + c);
          const float ox = q[0], oy = q[1], oz = q[2];
          if (!(oz > 0.0f)) continue;
          float S[kMaxSigma];
          switch (h) {
            case 1:
              window_sums_grid<1, NA>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, g, S);
              break;
            case 2:
              window_sums_grid<2, NA>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, g, S);
              break;
            default:
              window_sums_grid<0, NA>(zbuf, L, lw, dxt, dyt, r, c, h, ox, oy, oz, g, S);
          }
#pragma unroll
          for (int ai = 0; ai < (NA > 0 ? NA : kMaxSigma); ++ai)
            if (NA > 0 || ai < g.A) sbuf[ai * kBlock + threadIdx.x] = S[ai] * g.normM[ai];
#pragma unroll
          for (int kk = 0; kk < kMaxNoise; ++kk)
            if (kk < nk_grid) acc[kk] += f_ln(g.pa[kk] + g.pomp[kk] * sbuf[g.ka[kk] * kBlock + threadIdx.x]);
        }
      };
      switch (g.A) {
        case 1:
          pixels(std::integral_constant<int, 1>{});
          break;
        case 2:
          pixels(std::integral_constant<int, 2>{});
          break;
        case 3:
          pixels(std::integral_constant<int, 3>{});
          break;
        case 4:
          pixels(std::integral_constant<int, 4>{});
          break;
        default:
          pixels(std::integral_constant<int, 0>{});
      }
      __syncthreads();
    }
  }
  block_sum<kMaxNoise>(acc, red);
  if (threadIdx.x == 0) {
    if (rows) {
      for (int k = 0; k < nk_grid; ++k) grid_out[k] = acc[k];
      return;
    }
    double v[kMaxNoise], m = -1e300;
    for (int k = 0; k < nk_grid; ++k) {
      const double* sat = g.sat + g.sat_stride * k;
      v[k] = (double)acc[k] + rect_sum(sat, W, all) - rect_sum(sat, W, region);
      grid_out[k] = (float)v[k];
      m = fmax(m, v[k] + (double)g.logw[k]);
    }
    double t = 0.0;
    for (int k = 0; k < nk_grid; ++k) t += exp(v[k] + (double)g.logw[k] - m);
    *marg_out = (float)(m + log(t));
  }
}

__global__ __launch_bounds__(kBlock, 4) void k_render_score_grid(SceneDev s, NoiseGridDev g,
                                                                 const float* __restrict__ poses, int N,
                                                                 float* __restrict__ logL_grid,
                                                                 float* __restrict__ logL_marg) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = blockIdx.x;
  if (n >= N) return;
  float dummy[kMaxNoise];
  float* gout = logL_grid ? logL_grid + (size_t)g.A * g.B * n : dummy;
  render_score_grid_one(s, g, poses + 16 * (size_t)n, gout, logL_marg + n, smem, -1, -1);
}

hipError_t launch_render_score_grid(const SceneDev& s, const NoiseGridDev& g, const float* poses, int N,
                                    float* logL_grid, float* logL_marg, hipStream_t st) {
  hipLaunchKernelGGL(k_render_score_grid, dim3(N), dim3(kBlock), fused_lds_bytes(s), st, s, g, poses, N, logL_grid,
                     logL_marg);
  return hipGetLastError();
}

// The noise grid of one observation point (sigma, p_out): the constants of
// eq. (1) as the host computes them, in double then rounded.
__device__ NoiseGridDev grid_point(float sigma, float p_out, double inv_V, double M) {
  NoiseGridDev g{};
  const double s = sigma;
  g.A = 1;
  g.B = 1;
  g.c2[0] = (float)(1.0 / (2.0 * s * s) / 0.69314718055994530942);
  g.normM[0] = (float)(pow(2.0 * 3.14159265358979323846 * s * s, -1.5) / M);
  g.ka[0] = 0;
  g.pa[0] = (float)((double)p_out * inv_V);
  g.pomp[0] = (float)(1.0 - (double)p_out);
  g.logw[0] = 0.0f;
  return g;
}

// Block (band b, scene j of the group): full-width rows [b R, (b + 1) R) of
// scene j's image under the group's noise grid, or under the scene's own
// (sigma, p_out) when G.noise[j] is set; per-point sums to
// partial[((G.first + j) n_bands + b) kMaxNoise + k].
__global__ __launch_bounds__(kBlock) void k_score_rows_grid(RowsGroupDev G, int R, int n_bands,
                                                            float* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x, j = blockIdx.y;
  if (j >= G.S) return;
  const SceneDev& s = G.s[j];
  const int row0 = b * R;
  const int row1 = min(s.cam.H, row0 + R);
  float* out = partial + ((size_t)(G.first + j) * n_bands + b) * kMaxNoise;
  if (row0 >= row1) {
    if (threadIdx.x < kMaxNoise) out[threadIdx.x] = 0.0f;
    return;
  }
  if (G.noise[j]) {
    const NoiseGridDev g = grid_point(G.noise[j][0], G.noise[j][1], G.inv_V, G.M_norm);
    render_score_grid_one(s, g, G.pose[j], out, nullptr, smem, row0, row1);
  } else {
    render_score_grid_one(s, G.grid, G.pose[j], out, nullptr, smem, row0, row1);
  }
}

// One thread per (scene, grid point): the band sums in band order, in
// double; then per scene the log-sum-exp with the grid's log weights.
__global__ void k_reduce_rows_grid(const float* __restrict__ partial, int P, int n_bands, int nk,
                                   NoiseGridDev g, float* __restrict__ grid_out, float* __restrict__ marg_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double v[kMaxNoise], m = -1e300;
  for (int k = 0; k < nk; ++k) {
    double t = 0.0;
    for (int b = 0; b < n_bands; ++b) t += (double)partial[((size_t)p * n_bands + b) * kMaxNoise + k];
    v[k] = t;
    grid_out[(size_t)p * nk + k] = (float)t;
    m = fmax(m, t + (double)g.logw[k]);
  }
  if (marg_out) {
    double t = 0.0;
    for (int k = 0; k < nk; ++k) t += exp(v[k] + (double)g.logw[k] - m);
    marg_out[p] = (float)(m + log(t));
  }
}

hipError_t launch_score_rows_grid(const RowsGroupDev& G, int R, int n_bands, float* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_score_rows_grid, dim3(n_bands, G.S), dim3(kBlock), fused_lds_bytes(G.s[0]), st, G, R, n_bands,
                     partial);
  return hipGetLastError();
}

hipError_t launch_reduce_rows_grid(const float* partial, int P, int n_bands, int nk, const NoiseGridDev& g,
                                   float* grid_out, float* marg_out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_rows_grid, dim3((P + 63) / 64), dim3(64), 0, st, partial, P, n_bands, nk, g, grid_out,
                     marg_out);
  return hipGetLastError();
}

// The counting instantiation: same work, plus per-launch totals of the work
// items in work[kCntN] (64-bit, accumulated).
__global__ __launch_bounds__(kBlock) void k_render_score_count(SceneDev s, const float* __restrict__ poses, int N,
                                                               float* __restrict__ logL, float* __restrict__ grad,
                                                               unsigned long long* __restrict__ work) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned cnt[kCntN];
  const int n = blockIdx.x;
  if (n >= N) return;
  if (threadIdx.x < kCntN) cnt[threadIdx.x] = 0u;
  __syncthreads();
  render_score_one<true, true>(s, poses + 16 * (size_t)n, logL + n, grad + 8 * (size_t)n, smem, cnt);
  __syncthreads();
  if (threadIdx.x < kCntN) atomicAdd(&work[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

hipError_t launch_render_score_count(const SceneDev& s, const float* poses, int N, float* logL, float* grad,
                                     unsigned long long* work, hipStream_t st) {
  hipLaunchKernelGGL(k_render_score_count, dim3(N), dim3(kBlock), fused_lds_bytes(s), st, s, poses, N, logL, grad,
                     work);
  return hipGetLastError();
}

hipError_t launch_render_score(const SceneDev& s, const float* poses, int N, float* logL, float* grad,
                               hipStream_t st) {
  const size_t lds = fused_lds_bytes(s);
  const bool big = s.mesh.has_big != 0;
  if (grad && big)
    hipLaunchKernelGGL((k_render_score<true, kRasterBig>), dim3(N), dim3(kBlock), lds, st, s, poses, N, logL, grad);
  else if (grad)
    hipLaunchKernelGGL((k_render_score<true, kRasterSmall>), dim3(N), dim3(kBlock), lds, st, s, poses, N, logL, grad);
  else if (big)
    hipLaunchKernelGGL((k_render_score<false, kRasterBig>), dim3(N), dim3(kBlock), lds, st, s, poses, N, logL, grad);
  else
    hipLaunchKernelGGL((k_render_score<false, kRasterSmall>), dim3(N), dim3(kBlock), lds, st, s, poses, N, logL,
                       grad);
  return hipGetLastError();
}

}  // namespace b3d

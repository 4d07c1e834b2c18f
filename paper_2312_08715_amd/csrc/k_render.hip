// Split-path rendering kernels: batched point-image render (one workgroup
// per hypothesis, LDS depth buffer over the object's pixel rectangle),
// depth-to-point conversion, the frozen-visibility pose adjoint, and the
// global-memory rasteriser used once per scene for static objects.
#include "b3d_launch.hpp"

namespace b3d {

// Write rows [y0, y1) of one hypothesis's outputs: pixels inside `band`
// come from the LDS key buffer, others are empty.
__device__ __forceinline__ void write_rows(const Cam& cam, int y0, int y1, const Rect& band,
                                           const unsigned long long* zbuf, uint32_t id_base, float* __restrict__ xyz,
                                           int* __restrict__ tri) {
  const int W = cam.W;
  const int nf = (y1 - y0) * W * 3;
  float* xo = xyz + (size_t)y0 * W * 3;
  for (int f = threadIdx.x; f < nf; f += kBlock) {
    const int p = f / 3, comp = f - 3 * p;
    const int r = y0 + p / W, c = p - (p / W) * W;
    float v = 0.0f;
    if (r >= band.y0 && r < band.y1 && c >= band.x0 && c < band.x1) {
      const unsigned long long k = zbuf[(r - band.y0) * band.w() + (c - band.x0)];
      if (k != kEmptyKey) {
        const float z = key_depth(k);
        v = comp == 0 ? z * ray_x(cam, c) : (comp == 1 ? z * ray_y(cam, r) : z);
      }
    }
    xo[f] = v;
  }
  if (tri) {
    int* to = tri + (size_t)y0 * W;
    const int np = (y1 - y0) * W;
    for (int p = threadIdx.x; p < np; p += kBlock) {
      const int r = y0 + p / W, c = p - (p / W) * W;
      int id = -1;
      if (r >= band.y0 && r < band.y1 && c >= band.x0 && c < band.x1) {
        const unsigned long long k = zbuf[(r - band.y0) * band.w() + (c - band.x0)];
        if (k != kEmptyKey) id = (int)(key_id(k) - id_base);
      }
      to[p] = id;
    }
  }
}

// write_rows for W a multiple of 4: each thread writes four pixels at a time
// (three 16-byte words of points, one of ids), so every store is a whole
// 16-byte word of a contiguous row span.
__device__ __forceinline__ void write_rows4(const Cam& cam, int y0, int y1, const Rect& band,
                                            const unsigned long long* zbuf, uint32_t id_base, float* __restrict__ xyz,
                                            int* __restrict__ tri) {
  const int W = cam.W, qpr = W / 4;  // pixel quads per row
  const int nq = (y1 - y0) * qpr;
  float4* xo = reinterpret_cast<float4*>(xyz + (size_t)y0 * W * 3);
  int4* to = tri ? reinterpret_cast<int4*>(tri + (size_t)y0 * W) : nullptr;
  const bool rows_in = y0 < band.y1 && y1 > band.y0 && !band.empty();
  for (int q = threadIdx.x; q < nq; q += kBlock) {
    const int dr = q / qpr;
    const int r = y0 + dr, c0 = 4 * (q - dr * qpr);
    float z[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int id[4] = {-1, -1, -1, -1};
    if (rows_in && r >= band.y0 && r < band.y1 && c0 + 4 > band.x0 && c0 < band.x1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + u;
        if (c >= band.x0 && c < band.x1) {
          const unsigned long long k = zbuf[(r - band.y0) * band.w() + (c - band.x0)];
          if (k != kEmptyKey) {
            z[u] = key_depth(k);
            id[u] = (int)(key_id(k) - id_base);
          }
        }
      }
    }
    const float ry = ray_y(cam, r);
    float x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = z[u] * ray_x(cam, c0 + u);
      y[u] = z[u] * ry;
    }
    xo[3 * q + 0] = make_float4(x[0], y[0], z[0], x[1]);
    xo[3 * q + 1] = make_float4(y[1], z[1], x[2], y[2]);
    xo[3 * q + 2] = make_float4(z[2], x[3], y[3], z[3]);
    if (to) to[q] = make_int4(id[0], id[1], id[2], id[3]);
  }
}

__global__ __launch_bounds__(kBlock) void k_render_batch(MeshDev m, Cam cam, const float* __restrict__ poses, int N,
                                                         float* __restrict__ xyz, int* __restrict__ tri, int zcap,
                                                         int vec) {
  extern __shared__ __align__(16) unsigned char smem[];
  const RasterLds rl = carve_raster_lds(smem);
  unsigned long long* zbuf = reinterpret_cast<unsigned long long*>(smem + kRasterLdsBytes);
  const int n = blockIdx.x;
  if (n >= N) return;
  const Pose P = load_pose(poses + 16 * (size_t)n);
  const int H = cam.H, W = cam.W;
#define WRITE_ROWS(...) (vec ? write_rows4(__VA_ARGS__) : write_rows(__VA_ARGS__))
  float* xn = xyz + (size_t)n * H * W * 3;
  int* tn = tri ? tri + (size_t)n * H * W : nullptr;
  const Rect obj = object_rect(m, P, cam);
  Rect none;
  none.x0 = none.x1 = none.y0 = none.y1 = 0;
  if (obj.empty()) {
    WRITE_ROWS(cam, 0, H, none, zbuf, 0, xn, tn);
    return;
  }
  const int band_rows = max(zcap / obj.w(), 1);
  for (int a = obj.y0; a < obj.y1; a += band_rows) {
    Rect band = obj;
    band.y0 = a;
    band.y1 = min(a + band_rows, obj.y1);
    const int nk = band.h() * band.w();
    for (int k = threadIdx.x; k < nk; k += kBlock) zbuf[k] = kEmptyKey;
    __syncthreads();
    raster_mesh_any(m, P, cam, 0u, band, band, zbuf, rl);
    refine_depths(m, P, cam, 0u, band, zbuf);
    WRITE_ROWS(cam, band.y0, band.y1, band, zbuf, 0u, xn, tn);
    __syncthreads();
  }
  // the rows the object does not reach, last: their stores drain while the
  // next workgroup on this CU rasterises (a barrier waits for every store
  // issued before it)
  WRITE_ROWS(cam, 0, obj.y0, none, zbuf, 0, xn, tn);
  WRITE_ROWS(cam, obj.y1, H, none, zbuf, 0, xn, tn);
}
#undef WRITE_ROWS

hipError_t launch_render_batch(const MeshDev& m, const Cam& cam, const float* poses, int N, float* xyz, int* tri,
                               int zcap, hipStream_t st) {
  const size_t lds = kRasterLdsBytes + sizeof(unsigned long long) * (size_t)zcap;
  // quads of pixels as whole 16-byte words: rows of W % 4 == 0 pixels in 16-byte aligned buffers
  const int vec = (cam.W % 4 == 0) && ((uintptr_t)xyz & 15) == 0 && ((uintptr_t)tri & 15) == 0;
  hipLaunchKernelGGL(k_render_batch, dim3(N), dim3(kBlock), lds, st, m, cam, poses, N, xyz, tri, zcap, vec);
  return hipGetLastError();
}

__global__ void k_unproject(const float* __restrict__ depth, int B, Cam cam, float* __restrict__ xyz) {
  const size_t total = (size_t)B * cam.H * cam.W;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < total; p += (size_t)gridDim.x * blockDim.x) {
    const int pix = (int)(p % ((size_t)cam.H * cam.W));
    const int r = pix / cam.W, c = pix - r * cam.W;
    const float z = depth[p] > 0.0f ? depth[p] : 0.0f;
    xyz[3 * p + 0] = z * ray_x(cam, c);
    xyz[3 * p + 1] = z * ray_y(cam, r);
    xyz[3 * p + 2] = z;
  }
}

hipError_t launch_unproject(const float* depth, int B, const Cam& cam, float* xyz, hipStream_t st) {
  const size_t total = (size_t)B * cam.H * cam.W;
  const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_unproject, dim3(blocks), dim3(256), 0, st, depth, B, cam, xyz);
  return hipGetLastError();
}

// d_pose[n] = sum_j g_j (n/(n.d), n x (t - q)/(n.d)), g_j = d_rend_j . d_j,
// with the depth of pixel j taken on the plane of its triangle.
__global__ __launch_bounds__(kBlock) void k_render_backward(MeshDev m, Cam cam, const float* __restrict__ poses,
                                                            int N, const int* __restrict__ tri,
                                                            const float* __restrict__ d_rend,
                                                            float* __restrict__ d_pose) {
  __shared__ float red[kWaves * 6];
  const int n = blockIdx.x;
  if (n >= N) return;
  const Pose P = load_pose(poses + 16 * (size_t)n);
  const int HW = cam.H * cam.W;
  const int* tn = tri + (size_t)n * HW;
  const float* dn = d_rend + (size_t)n * HW * 3;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < HW; p += kBlock) {
    const int id = tn[p];
    if (id < 0 || id >= m.T) continue;
    const int r = p / cam.W, c = p - r * cam.W;
    const float dx = ray_x(cam, c), dy = ray_y(cam, r);
    const float g = dn[3 * p] * dx + dn[3 * p + 1] * dy + dn[3 * p + 2];
    if (g == 0.0f) continue;
    const float4 no = m.normals[id];
    const float3 nn = rotate(P, no.x, no.y, no.z);
    const float nd = nn.x * dx + nn.y * dy + nn.z;
    const float z = plane_depth(m, P, cam, (uint32_t)id, r, c);
    const float tx = P.t[0] - z * dx, ty = P.t[1] - z * dy, tz = P.t[2] - z;
    const float s = g / nd;
    acc[0] += s * nn.x;
    acc[1] += s * nn.y;
    acc[2] += s * nn.z;
    acc[3] += s * (nn.y * tz - nn.z * ty);
    acc[4] += s * (nn.z * tx - nn.x * tz);
    acc[5] += s * (nn.x * ty - nn.y * tx);
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 6; ++k) d_pose[6 * (size_t)n + k] = acc[k];
}

hipError_t launch_render_backward(const MeshDev& m, const Cam& cam, const float* poses, int N, const int* tri,
                                  const float* d_rend, float* d_pose, hipStream_t st) {
  hipLaunchKernelGGL(k_render_backward, dim3(N), dim3(kBlock), 0, st, m, cam, poses, N, tri, d_rend, d_pose);
  return hipGetLastError();
}

__global__ void k_fill_keys(unsigned long long* keys, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    keys[i] = kEmptyKey;
}

hipError_t launch_fill_keys(unsigned long long* keys, size_t n, hipStream_t st) {
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_keys, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, keys, n);
  return hipGetLastError();
}

// One thread per (triangle, slice of its rows), whole image, global 64-bit
// atomicMin: used per scene to draw the static objects.  Slicing the rows
// keeps a triangle that spans the image (a table top) from serialising on
// one thread; the minimum does not depend on the order.
constexpr int kRasterSlices = 32;

__global__ void k_raster_global(MeshDev m, Cam cam, Pose P, uint32_t id_base, unsigned long long* keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int slice = blockIdx.y;
  if (i >= m.T) return;
  const int4 tr = m.tris[i];
  float4 pv[3];
  const int vi[3] = {tr.x, tr.y, tr.z};
  for (int k = 0; k < 3; ++k) {
    const float4 o = m.verts[vi[k]];
    const float3 p = xform(P, o.x, o.y, o.z);
    const float iz = 1.0f / p.z;
    pv[k] = make_float4(cam.fx * p.x * iz + cam.cx, cam.fy * p.y * iz + cam.cy, p.z, iz);
  }
  const float4 p0 = pv[0], p1 = pv[1], p2 = pv[2];
  if (p0.z <= cam.znear || p1.z <= cam.znear || p2.z <= cam.znear) return;
  const float area = (p1.x - p0.x) * (p2.y - p0.y) - (p2.x - p0.x) * (p1.y - p0.y);
  if (!(area < 0.0f)) return;
  const float umin = fminf(p0.x, fminf(p1.x, p2.x)), umax = fmaxf(p0.x, fmaxf(p1.x, p2.x));
  const float vmin = fminf(p0.y, fminf(p1.y, p2.y)), vmax = fmaxf(p0.y, fmaxf(p1.y, p2.y));
  const float fc0 = ceilf(fmaxf(umin - 0.5f, 0.0f)), fc1 = floorf(fminf(umax - 0.5f, (float)(cam.W - 1)));
  const float fr0 = ceilf(fmaxf(vmin - 0.5f, 0.0f)), fr1 = floorf(fminf(vmax - 0.5f, (float)(cam.H - 1)));
  if (!(fc0 <= fc1) || !(fr0 <= fr1)) return;
  const float inv_area = 1.0f / area;
  const float e0x = p2.x - p1.x, e0y = p2.y - p1.y;
  const float e1x = p0.x - p2.x, e1y = p0.y - p2.y;
  const float e2x = p1.x - p0.x, e2y = p1.y - p0.y;
  for (int r = (int)fr0 + slice; r <= (int)fr1; r += kRasterSlices) {
    const float py = (float)r + 0.5f;
    for (int c = (int)fc0; c <= (int)fc1; ++c) {
      const float px = (float)c + 0.5f;
      const float w0 = e0x * (py - p1.y) - e0y * (px - p1.x);
      const float w1 = e1x * (py - p2.y) - e1y * (px - p2.x);
      const float w2 = e2x * (py - p0.y) - e2y * (px - p0.x);
      if (w0 > 0.0f || w1 > 0.0f || w2 > 0.0f) continue;
      const float invz = (w0 * p0.w + w1 * p1.w + w2 * p2.w) * inv_area;
      const float z = __builtin_amdgcn_rcpf(invz);
      if (!(z > 0.0f)) continue;
      atomicMin(&keys[(size_t)r * cam.W + c], pack_key(z, id_base + (uint32_t)i));
    }
  }
}

// Exact plane depth for every pixel of a full-image key buffer drawn by this
// mesh (see plane_depth); the pose comes from `pose16_dev` when not null.
__global__ void k_refine_global(MeshDev m, Cam cam, Pose P, const float* __restrict__ pose16_dev, uint32_t id_base,
                                unsigned long long* keys) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= cam.H * cam.W) return;
  const unsigned long long key = keys[p];
  if (key == kEmptyKey) return;
  const uint32_t id = key_id(key) - id_base;
  if (id >= (uint32_t)m.T) return;
  const Pose Q = pose16_dev ? load_pose(pose16_dev) : P;
  const int r = p / cam.W, c = p - r * cam.W;
  keys[p] = pack_key(plane_depth(m, Q, cam, id, r, c), key_id(key));
}

hipError_t launch_raster_global(const MeshDev& m, const Cam& cam, const float* pose16, uint32_t id_base,
                                unsigned long long* keys, hipStream_t st) {
  Pose P;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P.r[3 * i + j] = pose16[4 * i + j];
    P.t[i] = pose16[4 * i + 3];
  }
  hipLaunchKernelGGL(k_raster_global, dim3((m.T + 255) / 256, kRasterSlices), dim3(256), 0, st, m, cam, P, id_base,
                     keys);
  return hipGetLastError();
}

hipError_t launch_refine_global(const MeshDev& m, const Cam& cam, const float* pose16_host, const float* pose16_dev,
                                uint32_t id_base, unsigned long long* keys, hipStream_t st) {
  Pose P = {};
  if (pose16_host)
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) P.r[3 * i + j] = pose16_host[4 * i + j];
      P.t[i] = pose16_host[4 * i + 3];
    }
  hipLaunchKernelGGL(k_refine_global, dim3((cam.H * cam.W + 255) / 256), dim3(256), 0, st, m, cam, P, pose16_dev,
                     id_base, keys);
  return hipGetLastError();
}

}  // namespace b3d

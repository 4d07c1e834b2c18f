// Pose refinement and tracking helpers: Adam ascent on the pose tangent,
// best-hypothesis selection, and drawing static objects whose poses live in
// device memory (so that a captured frame graph sees the latest estimates).
#include "b3d_launch.hpp"

namespace b3d {

// Adam step for each pose n; state [N][12] = (m, v).
__global__ void k_adam_pose(float* __restrict__ poses, const float* __restrict__ grad, int gstride,
                            float* __restrict__ state, int N, int iter, float lr_t, float lr_r, float b1, float b2,
                            float eps) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float* m = state + 12 * (size_t)n;
  adam_update(poses + 16 * (size_t)n, grad + (size_t)gstride * n, m, m + 6, iter, lr_t, lr_r, b1, b2, eps);
}

hipError_t launch_adam_pose(float* poses, const float* grad, int gstride, float* state, int N, int iter, float lr_t,
                            float lr_r, float b1, float b2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(k_adam_pose, dim3((N + 63) / 64), dim3(64), 0, st, poses, grad, gstride, state, N, iter, lr_t,
                     lr_r, b1, b2, eps);
  return hipGetLastError();
}

// Rotation exp([w]x) as a row-major 3x3 (Rodrigues), and the coefficients
// a = (1 - cos th)/th^2, b = (th - sin th)/th^3 of the left Jacobian
// J(w) = I + a [w]x + b [w]x^2 (series below th = 1e-2).
__device__ void so3_exp(float wx, float wy, float wz, float* E, float* a, float* b) {
  const float t2 = wx * wx + wy * wy + wz * wz, th = sqrtf(t2);
  float s_t, c_t2;  // sin(th)/th, (1 - cos th)/th^2
  if (th < 1e-2f) {
    s_t = 1.0f - t2 / 6.0f;
    c_t2 = 0.5f - t2 / 24.0f;
    *b = 1.0f / 6.0f - t2 / 120.0f;
  } else {
    s_t = sinf(th) / th;
    c_t2 = (1.0f - cosf(th)) / t2;
    *b = (th - sinf(th)) / (t2 * th);
  }
  *a = c_t2;
  E[0] = 1.0f - c_t2 * (wy * wy + wz * wz);
  E[1] = -s_t * wz + c_t2 * wx * wy;
  E[2] = s_t * wy + c_t2 * wx * wz;
  E[3] = s_t * wz + c_t2 * wx * wy;
  E[4] = 1.0f - c_t2 * (wx * wx + wz * wz);
  E[5] = -s_t * wx + c_t2 * wy * wz;
  E[6] = -s_t * wy + c_t2 * wx * wz;
  E[7] = s_t * wx + c_t2 * wy * wz;
  E[8] = 1.0f - c_t2 * (wx * wx + wy * wy);
}

// out[n] = (exp([w_n]x) R_b, t_b + dt_n) with xi_n = (dt, w) and base pose b =
// n (n_base = N) or 0 (n_base = 1).
__global__ void k_pose_retract(const float* __restrict__ base, int n_base, const float* __restrict__ xi, int N,
                               float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const float* B = base + 16 * (size_t)(n_base == 1 ? 0 : n);
  const float* x = xi + 6 * (size_t)n;
  float E[9], a, b;
  so3_exp(x[3], x[4], x[5], E, &a, &b);
  float* P = out + 16 * (size_t)n;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P[4 * i + j] = E[3 * i] * B[j] + E[3 * i + 1] * B[4 + j] + E[3 * i + 2] * B[8 + j];
    P[4 * i + 3] = B[4 * i + 3] + x[i];
  }
  P[12] = B[12];
  P[13] = B[13];
  P[14] = B[14];
  P[15] = B[15];
}

// Chain rule through the retraction: with g = (d/d dt, d/d dw) at the
// retracted pose (tangent perturbation exp([d]x) R), d/d xi_t = u g_t and
// d/d xi_w = u J(w)^T g_w, u = dlogL[n] (1 when dlogL is NULL).  One block
// also forms the fixed-order sums over n of u g[6] and u g[7] (sigma and p_out
// shared by every hypothesis) into dsp[2] when dsp is not NULL.
__global__ __launch_bounds__(kBlock) void k_pose_retract_backward(const float* __restrict__ xi,
                                                                  const float* __restrict__ grad,
                                                                  const float* __restrict__ dlogL, int N,
                                                                  float* __restrict__ dxi, float* __restrict__ dsp) {
  __shared__ float red[2 * kWaves];
  float acc[2] = {0.0f, 0.0f};
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const float* x = xi + 6 * (size_t)n;
    const float* g = grad + 8 * (size_t)n;
    const float u = dlogL ? dlogL[n] : 1.0f;
    const float wx = x[3], wy = x[4], wz = x[5];
    float E[9], a, b;
    so3_exp(wx, wy, wz, E, &a, &b);
    // J^T v = v - a (w x v) + b w x (w x v)
    const float vx = g[3], vy = g[4], vz = g[5];
    const float cx = wy * vz - wz * vy, cy = wz * vx - wx * vz, cz = wx * vy - wy * vx;
    const float ccx = wy * cz - wz * cy, ccy = wz * cx - wx * cz, ccz = wx * cy - wy * cx;
    float* d = dxi + 6 * (size_t)n;
    d[0] = u * g[0];
    d[1] = u * g[1];
    d[2] = u * g[2];
    d[3] = u * (vx - a * cx + b * ccx);
    d[4] = u * (vy - a * cy + b * ccy);
    d[5] = u * (vz - a * cz + b * ccz);
    acc[0] += u * g[6];
    acc[1] += u * g[7];
  }
  if (!dsp) return;
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    dsp[0] = acc[0];
    dsp[1] = acc[1];
  }
}

hipError_t launch_pose_retract(const float* base, int n_base, const float* xi, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_retract, dim3((N + 63) / 64), dim3(64), 0, st, base, n_base, xi, N, out);
  return hipGetLastError();
}

hipError_t launch_pose_retract_backward(const float* xi, const float* grad, const float* dlogL, int N, float* dxi,
                                        float* dsp, hipStream_t st) {
  hipLaunchKernelGGL(k_pose_retract_backward, dim3(1), dim3(kBlock), 0, st, xi, grad, dlogL, N, dxi, dsp);
  return hipGetLastError();
}

__global__ void k_fill_f32(float* __restrict__ p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st) {
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

__global__ void k_copy_f32(const float* __restrict__ src, int n, float* __restrict__ dst) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

hipError_t launch_copy_f32(const float* src, int n, float* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3((n + 255) / 256), dim3(256), 0, st, src, n, dst);
  return hipGetLastError();
}

// The tracker's occlusion decision for one object; one block.  Seen pixels:
// those the object (drawn alone into objkeys) covers, whose key is below the
// other objects' key (nearer; the object's ids, numbered first, win equal
// depths, as in the fused kernel's composite), that have a valid observed
// point within distance sqrt(tol2) of the object's point among the
// (2h + 1)^2 pixels centred on them.  seen = seen pixels / covered pixels (0
// when none).  At or above min_visible the update stands and its motion is
// kept: rotation R_pose R_prev^T, translation t_pose - t_prev.  Below it the
// pose becomes prev moved by the kept motion (R <- dR R_prev,
// t <- t_prev + dt).  gate = (seen, dropped updates in a row, stage 0's
// translation scale for the next frame, 0).
__global__ __launch_bounds__(kBlock) void k_track_gate(const unsigned long long* __restrict__ objkeys,
                                                       const unsigned long long* __restrict__ bg,
                                                       const float* __restrict__ obs, Cam cam, int h, float tol2,
                                                       float min_visible, float widen, const float* __restrict__ prev,
                                                       float* __restrict__ pose, float* __restrict__ motion,
                                                       float* __restrict__ gate) {
  __shared__ unsigned sd[kWaves], sv[kWaves];
  unsigned drawn = 0, seen = 0;
  const int HW = cam.H * cam.W;
  // some valid observed point in the window of pixel (r, c) within the
  // tolerance of the point at depth z on that pixel's ray
  auto confirmed = [&](int r, int c, float z) {
    const float qx = z * ray_x(cam, c), qy = z * ray_y(cam, r);
    for (int dy = -h; dy <= h; ++dy) {
      const int ri = r + dy;
      if (ri < 0 || ri >= cam.H) continue;
      for (int dx = -h; dx <= h; ++dx) {
        const int ci = c + dx;
        if (ci < 0 || ci >= cam.W) continue;
        const float* o = obs + 3 * ((size_t)ri * cam.W + ci);
        const float ex = o[0] - qx, ey = o[1] - qy, ez = o[2] - z;
        if (o[2] > 0.0f && ex * ex + ey * ey + ez * ez <= tol2) return true;
      }
    }
    return false;
  };
  for (int p = threadIdx.x; p < HW; p += kBlock) {
    const unsigned long long k = objkeys[p];
    if (k == kEmptyKey) continue;
    ++drawn;
    if (bg && !(k < bg[p])) continue;  // behind the others
    const int r = p / cam.W, c = p - r * cam.W;
    if (confirmed(r, c, key_depth(k))) ++seen;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    drawn += __shfl_xor(drawn, o, 64);
    seen += __shfl_xor(seen, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sd[wave] = drawn;
    sv[wave] = seen;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  drawn = 0;
  seen = 0;
  for (int w = 0; w < kWaves; ++w) {
    drawn += sd[w];
    seen += sv[w];
  }
  const float frac = drawn ? (float)seen / (float)drawn : 0.0f;
  gate[0] = frac;
  if (frac >= min_visible) {
    // keep the update; its motion: dR = R R_prev^T, dt = t - t_prev
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b)
        motion[3 * a + b] = pose[4 * a + 0] * prev[4 * b + 0] + pose[4 * a + 1] * prev[4 * b + 1] +
                            pose[4 * a + 2] * prev[4 * b + 2];
      motion[9 + a] = pose[4 * a + 3] - prev[4 * a + 3];
    }
    gate[1] = 0.0f;
    gate[2] = 1.0f;
  } else {
    // drop it: prev moved by the kept motion
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b)
        pose[4 * a + b] = motion[3 * a + 0] * prev[b] + motion[3 * a + 1] * prev[4 + b] + motion[3 * a + 2] * prev[8 + b];
      pose[4 * a + 3] = prev[4 * a + 3] + motion[9 + a];
    }
    for (int k = 12; k < 16; ++k) pose[k] = prev[k];
    gate[1] += 1.0f;
    gate[2] = widen;
  }
  gate[3] = 0.0f;
}

hipError_t launch_track_gate(const unsigned long long* objkeys, const unsigned long long* bg, const float* obs,
                             const Cam& cam, int h, float tol, float min_visible, float widen, const float* prev,
                             float* pose, float* motion, float* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_track_gate, dim3(1), dim3(kBlock), 0, st, objkeys, bg, obs, cam, h, tol * tol, min_visible,
                     widen, prev, pose, motion, gate);
  return hipGetLastError();
}

// out = poses[argmax logL] (ties to the lowest index); one block.
__global__ __launch_bounds__(kBlock) void k_argmax_pose(const float* __restrict__ logL, const float* __restrict__ poses,
                                                        int N, float* __restrict__ out) {
  __shared__ float rv[kWaves];
  __shared__ int ri[kWaves];
  __shared__ int best;
  float bv = -INFINITY;
  int bi = -1;
  for (int n = threadIdx.x; n < N; n += kBlock)
    if (bi < 0 || logL[n] > bv) {
      bv = logL[n];
      bi = n;
    }
  for (int o = 32; o >= 1; o >>= 1) {
    const float ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (oi >= 0 && (bi < 0 || ov > bv || (ov == bv && oi < bi))) {
      bv = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    best = bi < 0 ? 0 : bi;
  }
  __syncthreads();
  if (threadIdx.x < 16) out[threadIdx.x] = poses[16 * (size_t)best + threadIdx.x];
}

hipError_t launch_argmax_pose(const float* logL, const float* poses, int N, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_argmax_pose, dim3(1), dim3(kBlock), 0, st, logL, poses, N, out);
  return hipGetLastError();
}

// As k_raster_global, with the pose read from device memory.
__global__ void k_raster_global_dev(MeshDev m, Cam cam, const float* __restrict__ pose16, uint32_t id_base,
                                    unsigned long long* keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.T) return;
  const Pose P = load_pose(pose16);
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
  for (int r = (int)fr0; r <= (int)fr1; ++r) {
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

hipError_t launch_raster_global_dev(const MeshDev& m, const Cam& cam, const float* pose16_dev, uint32_t id_base,
                                    unsigned long long* keys, hipStream_t st) {
  hipLaunchKernelGGL(k_raster_global_dev, dim3((m.T + 255) / 256), dim3(256), 0, st, m, cam, pose16_dev, id_base,
                     keys);
  return hipGetLastError();
}

}  // namespace b3d

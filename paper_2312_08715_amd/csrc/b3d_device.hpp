// Device-side building blocks shared by the gfx950 kernels: camera and pose
// helpers, packed depth/id keys, the cluster-based triangle rasteriser that
// fills an LDS depth buffer, and fixed-order block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace b3d {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kClusterPrims = 64;    // max primitives (triangles or quads) per cluster, one per lane of a wave
constexpr uint32_t kNoTri = 0xFFFFFFFFu;  // second id of a primitive that is a single triangle
// The key of a pixel with no surface: depth 1e15 m (bits 0x58635FA9), id all
// ones.  It compares above every surface nearer than that, and its depth is
// finite, so a window term against an empty slot evaluates to exactly 0
// (exp of minus a huge distance) without a test, provided rays stay within
// |x/z|, |y/z| <= 1e3 (checked when a scene is created).
constexpr unsigned long long kEmptyKey = (0x58635FA9ull << 32) | 0xFFFFFFFFull;

// Pinhole camera and image size.
struct Cam {
  float fx, fy, cx, cy, znear;
  int H, W;
};

// Row-major rotation and translation of an object-to-camera pose.
struct Pose {
  float r[9];
  float t[3];
};

// A group of up to kClusterPrims primitives of one orientation class that
// are close in space: primitives [pfirst, pfirst + np).  A primitive is the
// triangle (a, b, c) and, when its second id is not kNoTri, the triangle
// (a, c, d) sharing the edge a-c (a convex planar quad).  sphere = centre and
// radius of a ball holding them; cone = unit axis and half-angle (radians) of
// a cone holding their face normals (half-angle > pi/2 means "no bound").
struct ClusterDev {
  int pfirst, np, pad0, pad1;
  float4 sphere;
  float4 cone;
};

// Device view of an uploaded mesh.
struct MeshDev {
  const ClusterDev* clusters;  // [0, n_visible) drawn; [n_visible, n_clusters) only near the near plane
  const float4* pverts;        // [primitives][4] object-frame corners a, b, c, d (d = c for a triangle)
  const uint2* pids;           // [primitives] caller's ids of triangles (a, b, c) and (a, c, d) or kNoTri
  const float4* verts;         // caller's vertices
  const int4* tris;            // caller's triangles (w unused)
  const float4* normals;       // object-frame (v1 - v0) x (v2 - v0)
  int n_clusters, n_visible;
  int has_big;                 // some primitive spans over 1/8 of the bounds' diagonal (table tops, walls)
  int T;                       // triangles
  float sphere[4];             // bounding sphere centre and radius
  float lo[3], hi[3];          // axis-aligned bounds
};

__device__ __forceinline__ Pose load_pose(const float* __restrict__ p) {
  Pose P;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    P.r[3 * i + 0] = p[4 * i + 0];
    P.r[3 * i + 1] = p[4 * i + 1];
    P.r[3 * i + 2] = p[4 * i + 2];
    P.t[i] = p[4 * i + 3];
  }
  return P;
}

__device__ __forceinline__ float3 xform(const Pose& P, float x, float y, float z) {
  return make_float3(P.r[0] * x + P.r[1] * y + P.r[2] * z + P.t[0], P.r[3] * x + P.r[4] * y + P.r[5] * z + P.t[1],
                     P.r[6] * x + P.r[7] * y + P.r[8] * z + P.t[2]);
}

__device__ __forceinline__ float3 rotate(const Pose& P, float x, float y, float z) {
  return make_float3(P.r[0] * x + P.r[1] * y + P.r[2] * z, P.r[3] * x + P.r[4] * y + P.r[5] * z,
                     P.r[6] * x + P.r[7] * y + P.r[8] * z);
}

// Ray direction components of pixel column c / row r (the z component is 1).
// Correctly rounded division, so every kernel gets bit-identical rays.
__device__ __forceinline__ float ray_x(const Cam& cam, int c) { return ((float)c + 0.5f - cam.cx) / cam.fx; }
__device__ __forceinline__ float ray_y(const Cam& cam, int r) { return ((float)r + 0.5f - cam.cy) / cam.fy; }

// Packed depth/id key: positive float bits are monotone, so the smallest key
// is the nearest surface and, at equal depth, the smallest triangle id.
__device__ __forceinline__ unsigned long long pack_key(float z, uint32_t id) {
  return ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)id;
}
__device__ __forceinline__ float key_depth(unsigned long long k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_id(unsigned long long k) { return (uint32_t)(k & 0xffffffffull); }

// Integer rectangle [x0, x1) x [y0, y1).
struct Rect {
  int x0, x1, y0, y1;
  __device__ __forceinline__ int w() const { return x1 - x0; }
  __device__ __forceinline__ int h() const { return y1 - y0; }
  __device__ __forceinline__ bool empty() const { return x1 <= x0 || y1 <= y0; }
};

__device__ __forceinline__ Rect grow(const Rect& r, int m) {
  Rect o;
  o.x0 = r.x0 - m;
  o.x1 = r.x1 + m;
  o.y0 = r.y0 - m;
  o.y1 = r.y1 + m;
  return o;
}

__device__ __forceinline__ Rect grow_clip(const Rect& r, int m, int W, int H) {
  Rect o;
  o.x0 = max(r.x0 - m, 0);
  o.x1 = min(r.x1 + m, W);
  o.y0 = max(r.y0 - m, 0);
  o.y1 = min(r.y1 + m, H);
  return o;
}

// Bounds of the projections of the 8 corners of the box [lo, hi] (camera
// frame after pose P when `posed`, else already camera-frame corners).
// Returns false when a corner is not in front of the near plane.
__device__ __forceinline__ bool project_box(const Pose& P, const float* lo, const float* hi, bool posed, const Cam& cam,
                                            float* b) {
  bool ok = true;
  b[0] = 3.0e38f;
  b[1] = -3.0e38f;
  b[2] = 3.0e38f;
  b[3] = -3.0e38f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float x = (k & 1) ? hi[0] : lo[0];
    const float y = (k & 2) ? hi[1] : lo[1];
    const float z = (k & 4) ? hi[2] : lo[2];
    const float3 c = posed ? xform(P, x, y, z) : make_float3(x, y, z);
    ok = ok && (c.z > cam.znear);
    const float iz = 1.0f / c.z;
    const float u = cam.fx * c.x * iz + cam.cx, v = cam.fy * c.y * iz + cam.cy;
    b[0] = fminf(b[0], u);
    b[1] = fmaxf(b[1], u);
    b[2] = fminf(b[2], v);
    b[3] = fmaxf(b[3], v);
  }
  return ok;
}

// Range of x/z over a sphere (centre c, radius r) in front of the camera:
// the planes x = k z through the camera that touch the sphere have
// (c_x - k c_z)^2 = r^2 (1 + k^2), i.e.
// k = (c_x c_z -+ r sqrt(c_x^2 + c_z^2 - r^2)) / (c_z^2 - r^2).
__device__ __forceinline__ void sphere_slopes(float cx, float cz, float r, float& k0, float& k1) {
  const float den = cz * cz - r * r;
  const float root = r * sqrtf(fmaxf(cx * cx + cz * cz - r * r, 0.0f));
  k0 = (cx * cz - root) / den;
  k1 = (cx * cz + root) / den;
}

// Conservative pixel rectangle of the object under pose P: the projection of
// the mesh's posed bounding box intersected with the exact projection bounds
// of its bounding sphere (slightly enlarged against rounding), widened by one
// pixel, clipped to the image.  The whole image when neither bound applies
// (the box reaches the near plane and the sphere reaches the camera plane).
__device__ __forceinline__ Rect object_rect(const MeshDev& m, const Pose& P, const Cam& cam) {
  float a[4], b[4];
  const bool aok = project_box(P, m.lo, m.hi, true, cam, a);
  const float3 c = xform(P, m.sphere[0], m.sphere[1], m.sphere[2]);
  const float rad = m.sphere[3] * 1.0001f + 1e-6f;
  const bool sok = c.z - rad > cam.znear;
  Rect r;
  if (!aok && !sok) {
    r.x0 = 0;
    r.x1 = cam.W;
    r.y0 = 0;
    r.y1 = cam.H;
    return r;
  }
  if (sok) {
    float k0, k1;
    sphere_slopes(c.x, c.z, rad, k0, k1);
    b[0] = cam.fx * k0 + cam.cx - 0.01f;
    b[1] = cam.fx * k1 + cam.cx + 0.01f;
    sphere_slopes(c.y, c.z, rad, k0, k1);
    b[2] = cam.fy * k0 + cam.cy - 0.01f;
    b[3] = cam.fy * k1 + cam.cy + 0.01f;
    if (aok) {
      b[0] = fmaxf(a[0], b[0]);
      b[1] = fminf(a[1], b[1]);
      b[2] = fmaxf(a[2], b[2]);
      b[3] = fminf(a[3], b[3]);
    }
  } else {
    for (int k = 0; k < 4; ++k) b[k] = a[k];
  }
  // pixel centres c + 1/2 in [umin, umax], widened by one pixel each side
  const float fx0 = fmaxf(ceilf(b[0] - 0.5f) - 1.0f, 0.0f);
  const float fx1 = fminf(floorf(b[1] - 0.5f) + 2.0f, (float)cam.W);
  const float fy0 = fmaxf(ceilf(b[2] - 0.5f) - 1.0f, 0.0f);
  const float fy1 = fminf(floorf(b[3] - 0.5f) + 2.0f, (float)cam.H);
  r.x0 = (int)fminf(fx0, (float)cam.W);
  r.x1 = (int)fmaxf(fx1, fx0);
  r.y0 = (int)fminf(fy0, (float)cam.H);
  r.y1 = (int)fmaxf(fy1, fy0);
  if (r.x1 > cam.W) r.x1 = cam.W;
  if (r.y1 > cam.H) r.y1 = cam.H;
  return r;
}

// Depth of pixel (r, c) on the plane of triangle `id` under pose P: the ray
// z d meets the plane n.(x - c0) = 0 at z = (n.c0)/(n.d), with
// c_k = R v_k + t and n = (c1 - c0) x (c2 - c0), all in double precision.
// The rasteriser's interpolated 1/z decides visibility; this value is the
// depth reported and scored.  (For a triangle seen nearly edge-on the depth
// is ill-conditioned in the vertex coordinates, and single precision would
// put errors of several micrometres into the point and its gradient.)
__device__ __forceinline__ float plane_depth(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id, int r,
                                             int c) {
  const int4 tr = m.tris[id];
  const float4 v[3] = {m.verts[tr.x], m.verts[tr.y], m.verts[tr.z]};
  double q[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      q[k][i] = (double)P.r[3 * i] * v[k].x + (double)P.r[3 * i + 1] * v[k].y + (double)P.r[3 * i + 2] * v[k].z +
                (double)P.t[i];
  const double e1[3] = {q[1][0] - q[0][0], q[1][1] - q[0][1], q[1][2] - q[0][2]};
  const double e2[3] = {q[2][0] - q[0][0], q[2][1] - q[0][1], q[2][2] - q[0][2]};
  const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double dx = ((double)c + 0.5 - (double)cam.cx) / (double)cam.fx;
  const double dy = ((double)r + 0.5 - (double)cam.cy) / (double)cam.fy;
  return (float)((n[0] * q[0][0] + n[1] * q[0][1] + n[2] * q[0][2]) / (n[0] * dx + n[1] * dy + n[2]));
}

// Replace the depth of every band pixel drawn by this mesh (id - id_base in
// [0, T)) by plane_depth, keeping its id.  Whole block; ends with a barrier.
__device__ __forceinline__ void refine_depths(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id_base,
                                              const Rect& band, unsigned long long* zbuf) {
  const int pitch = band.w();
  const int np = band.h() * pitch;
  for (int k = threadIdx.x; k < np; k += kBlock) {
    const unsigned long long key = zbuf[k];
    if (key == kEmptyKey) continue;
    const uint32_t id = key_id(key) - id_base;
    if (id >= (uint32_t)m.T) continue;
    const int r = band.y0 + k / pitch, c = band.x0 + (k - (k / pitch) * pitch);
    zbuf[k] = pack_key(plane_depth(m, P, cam, id, r, c), key_id(key));
  }
  __syncthreads();
}

// Whether a cluster can draw into `band` under pose P: false when its
// sphere lies behind the near plane, when every normal of its cone faces away
// from every point of its sphere (the angle between the cone axis and the
// direction to the sphere centre, plus the cone's and the sphere's angular
// radii, stays below a right angle by a margin), or when the sphere's screen
// box misses the band.  Uniform across the block.
// When it may draw and its sphere lies in front of the near plane, box[4]
// receives the sphere's screen box (umin, umax, vmin, vmax) and *zmin the
// depth of its nearest point; otherwise *zmin = 0.
__device__ __forceinline__ bool cluster_may_draw(const ClusterDev& c, const Pose& P, const Cam& cam,
                                                 const Rect& band, float* box, float* zmin) {
  const float3 s = xform(P, c.sphere.x, c.sphere.y, c.sphere.z);
  const float r = c.sphere.w;
  *zmin = 0.0f;
  if (s.z + r <= cam.znear) return false;
  const float d2 = s.x * s.x + s.y * s.y + s.z * s.z;
  if (c.cone.w < 1.5f && d2 > r * r) {
    const float3 a = rotate(P, c.cone.x, c.cone.y, c.cone.z);
    const float d = sqrtf(d2);
    const float ct = fminf(1.0f, fmaxf(-1.0f, (a.x * s.x + a.y * s.y + a.z * s.z) / d));
    if (acosf(ct) + c.cone.w + asinf(fminf(1.0f, r / d)) < 1.5707963f - 2e-3f) return false;
  }
  if (s.z - r > cam.znear) {
    const float lo[3] = {s.x - r, s.y - r, s.z - r}, hi[3] = {s.x + r, s.y + r, s.z + r};
    project_box(P, lo, hi, false, cam, box);
    if (box[1] < (float)band.x0 - 1.0f || box[0] > (float)band.x1 + 1.0f || box[3] < (float)band.y0 - 1.0f ||
        box[2] > (float)band.y1 + 1.0f)
      return false;
    *zmin = s.z - r;
  }
  return true;
}


// Coverage of pixel (r, c) by triangle `id` decided in double precision with
// exactly the operations, in the same order, of the plain definition
// (transform, near-plane drop, back-face test on ((c1-c0)x(c2-c0)).c0,
// projection, edge functions at the pixel centre, inclusive).  Used only for
// pixel centres that single precision cannot place on one side of an edge.
__device__ __forceinline__ bool covered_exact(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id,
                                                        int r, int col) {
#pragma clang fp contract(off)
  const int4 tr = m.tris[id];
  const float4 v[3] = {m.verts[tr.x], m.verts[tr.y], m.verts[tr.z]};
  double c[3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i)
      c[k][i] = (double)P.r[3 * i] * (double)v[k].x + (double)P.r[3 * i + 1] * (double)v[k].y +
                (double)P.r[3 * i + 2] * (double)v[k].z + (double)P.t[i];
  const double zn = (double)cam.znear;
  if (c[0][2] <= zn || c[1][2] <= zn || c[2][2] <= zn) return false;
  const double e1[3] = {c[1][0] - c[0][0], c[1][1] - c[0][1], c[1][2] - c[0][2]};
  const double e2[3] = {c[2][0] - c[0][0], c[2][1] - c[0][1], c[2][2] - c[0][2]};
  const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
  const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
  const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
  const double nc0 = n0 * c[0][0] + n1 * c[0][1] + n2 * c[0][2];
  if (!(nc0 < 0.0)) return false;
  const double fx = cam.fx, fy = cam.fy, cx = cam.cx, cy = cam.cy;
  const double u0 = fx * c[0][0] / c[0][2] + cx, v0 = fy * c[0][1] / c[0][2] + cy;
  const double u1 = fx * c[1][0] / c[1][2] + cx, v1 = fy * c[1][1] / c[1][2] + cy;
  const double u2 = fx * c[2][0] / c[2][2] + cx, v2 = fy * c[2][1] / c[2][2] + cy;
  const double px = col + 0.5, py = r + 0.5;
  const double w0 = (u2 - u1) * (py - v1) - (v2 - v1) * (px - u1);
  const double w1 = (u0 - u2) * (py - v2) - (v0 - v2) * (px - u2);
  const double w2 = (u1 - u0) * (py - v0) - (v1 - v0) * (px - u0);
  return !(w0 > 0.0 || w1 > 0.0 || w2 > 0.0);
}

// LDS scratch of the rasteriser (free again once raster_mesh returns; the
// fused kernel then reuses it for the window weights, which sets its size).
struct RasterLds {
  uint2* queue;  // (band pixel, triangle id) pairs left for the exact test
  int* list;     // drawable clusters of the current group of kBlock
  int* counts;   // [0] queue fill, [1..kWaves] per-wave drawable counts, [kWaves + 1] next list entry
  int qcap;
};

constexpr int kQueueCap = 1536;
constexpr size_t kRasterLdsBytes = sizeof(uint2) * kQueueCap + sizeof(int) * kBlock + sizeof(int) * 16;

constexpr int kBigCentres = 64;  // a box of more centres than this is walked by the whole wave
constexpr int kBigSlots = 2;     // such boxes a wave takes together per cluster
constexpr int kStageWords = 36;  // words of one staged box
// the staged boxes take the queue's last entries
constexpr int kStageQueueEntries = (int)((sizeof(float) * kWaves * kBigSlots * kStageWords + 7) / 8);
static_assert(kStageQueueEntries < kQueueCap / 4, "staging area too large for the exact-test queue");

__device__ __forceinline__ RasterLds carve_raster_lds(unsigned char* p) {
  RasterLds r;
  r.queue = reinterpret_cast<uint2*>(p);
  r.list = reinterpret_cast<int*>(r.queue + kQueueCap);
  r.counts = r.list + kBlock;
  r.qcap = kQueueCap;
  return r;
}

// Staging slots of the large-box walk (only meshes with large primitives use
// them, with the queue shortened to kQueueCap - kStageQueueEntries).
__device__ __forceinline__ float* raster_stage(const RasterLds& r) {
  return reinterpret_cast<float*>(r.queue + (kQueueCap - kStageQueueEntries));
}

// Work counters of the counting instantiation (indices into a per-block
// array): vertices transformed, triangles tested, triangles set up, covered
// pixel centres, window pairs, observed pixels that saw a point, object pixels
// of the adjoint, centres decided by the exact test.
enum { kCntVert = 0, kCntTri, kCntSetup, kCntFrag, kCntPair, kCntObs, kCntAdj, kCntExact, kCntN };

// Pixel position, depth and 1/depth of an object-frame point under pose P.
__device__ __forceinline__ float4 project_corner(const Pose& P, const Cam& cam, const float4 o) {
  const float3 p = xform(P, o.x, o.y, o.z);
  // hardware reciprocal (1 ulp): far inside the rasteriser's edge margin
  const float iz = __builtin_amdgcn_rcpf(p.z);
  return make_float4(cam.fx * p.x * iz + cam.cx, cam.fy * p.y * iz + cam.cy, p.z, iz);
}

// A centre of one triangle: queued for the exact test when within the
// margin of an edge (or the triangle is nearly edge-on), else written.
// (x0, x1, x2) are its edge functions, (m0, m1, m2) their margins, (i0, i1,
// i2) the corners' 1/z and ia 1/area.
template <bool COUNT>
__device__ __forceinline__ void emit_centre(int pix, bool eon, float x0, float x1, float x2, float m0, float m1,
                                            float m2, float i0, float i1, float i2, float ia, uint32_t tid,
                                            uint32_t id_base, unsigned long long* zbuf, const RasterLds& lds,
                                            unsigned& c_frag) {
  if (eon || x0 >= -m0 || x1 >= -m1 || x2 >= -m2) {
    const int slot = atomicAdd(&lds.counts[0], 1);
    if (slot < lds.qcap) {
      lds.queue[slot] = make_uint2((uint32_t)pix, tid);
      return;
    }
    if (eon || x0 > 0.0f || x1 > 0.0f || x2 > 0.0f) return;  // queue full: single precision
  }
  // 1/z is affine in screen space: interpolate with barycentrics x_k/area
  const float z = __builtin_amdgcn_rcpf((x0 * i0 + x1 * i1 + x2 * i2) * ia);
  if (!(z > 0.0f)) return;
  if (COUNT) ++c_frag;
  atomicMin(&zbuf[pix], pack_key(z, id_base + tid));
}

// Word layout of a staged box: edge vectors e0, e1, e2, f0, f1 (x, y), edge
// margins t0, t1, t2, s0, s1, 1/area of both triangles, the edge functions at
// the box's first centre, the corners' 1/z, then (as ints) the box, the two
// triangle ids and the flags act1 | act2 << 1 | eon1 << 2 | eon2 << 3.
enum { kStE = 0, kStT = 10, kStIa = 15, kStW = 17, kStIz = 22, kStBox = 26, kStIds = 30, kStFlags = 32 };

// The whole wave walks a staged box, lane l taking centres l, l + 64, ...;
// each centre gets the coverage tests of the single-lane walk from the same
// values (which walk a box takes depends only on the mesh and the pose).
template <bool COUNT>
__device__ __forceinline__ void walk_staged(const float* __restrict__ st, int lane, const Rect& buf, int pitch,
                                            uint32_t id_base, unsigned long long* zbuf, const RasterLds& lds,
                                            unsigned& c_frag) {
  const int* si = reinterpret_cast<const int*>(st);
  const int c0 = si[kStBox], c1 = si[kStBox + 1], r0 = si[kStBox + 2], r1 = si[kStBox + 3];
  const uint32_t id1 = (uint32_t)si[kStIds], id2 = (uint32_t)si[kStIds + 1];
  const int flags = si[kStFlags];
  const bool act1 = flags & 1, act2 = flags & 2, eon1 = flags & 4, eon2 = flags & 8;
  const float e0x = st[kStE], e0y = st[kStE + 1], e1x = st[kStE + 2], e1y = st[kStE + 3];
  const float e2x = st[kStE + 4], e2y = st[kStE + 5], f0x = st[kStE + 6], f0y = st[kStE + 7];
  const float f1x = st[kStE + 8], f1y = st[kStE + 9];
  const float t0 = st[kStT], t1 = st[kStT + 1], t2 = st[kStT + 2], s0 = st[kStT + 3], s1 = st[kStT + 4];
  const float ia1 = st[kStIa], ia2 = st[kStIa + 1];
  const float w0b = st[kStW], w1b = st[kStW + 1], w2b = st[kStW + 2], v0b = st[kStW + 3], v1b = st[kStW + 4];
  const float izA = st[kStIz], izB = st[kStIz + 1], izC = st[kStIz + 2], izD = st[kStIz + 3];
  const int wc = c1 - c0 + 1, n_cent = wc * (r1 - r0 + 1);
  for (int k = lane; k < n_cent; k += 64) {
    const int dri = k / wc;
    const int r = r0 + dri, col = c0 + (k - dri * wc);
    const float dr = (float)dri, dc = (float)(col - c0);
    const float w0 = __builtin_fmaf(-e0y, dc, __builtin_fmaf(e0x, dr, w0b));
    const float w1 = __builtin_fmaf(-e1y, dc, __builtin_fmaf(e1x, dr, w1b));
    const float w2 = __builtin_fmaf(-e2y, dc, __builtin_fmaf(e2x, dr, w2b));
    const float v0 = __builtin_fmaf(-f0y, dc, __builtin_fmaf(f0x, dr, v0b));
    const float v1 = __builtin_fmaf(-f1y, dc, __builtin_fmaf(f1x, dr, v1b));
    const bool out1 = !act1 || w0 > t0 || w1 > t1 || w2 > t2;
    const bool out2 = !act2 || v0 > s0 || v1 > s1 || -w1 > t1;
    if (out1 && out2) continue;
    const int pix = (r - buf.y0) * pitch + (col - buf.x0);
    if (!out1) emit_centre<COUNT>(pix, eon1, w0, w1, w2, t0, t1, t2, izA, izB, izC, ia1, id1, id_base, zbuf, lds, c_frag);
    if (!out2) emit_centre<COUNT>(pix, eon2, v0, v1, -w1, s0, s1, t1, izA, izC, izD, ia2, id2, id_base, zbuf, lds, c_frag);
  }
}

// Rasterise the mesh under pose P into the pixels of the image rectangle
// `band` of an LDS key buffer that covers the rectangle `buf` (row pitch
// buf.w(); band inside buf).  Triangle ids written are
// id_base + the caller's triangle index.  Clusters are tested for drawing,
// kBlock at a time, and the drawable ones compacted into a list; the four
// waves then take clusters from the list independently: a wave transforms
// its cluster's vertices into its own LDS buffer and each lane takes one
// primitive (a quad or a triangle), walking the pixel centres of its screen
// box; with BIG, up to kBigSlots boxes of more than kBigCentres centres per
// wave and cluster are walked by the whole wave instead (with the same
// coverage tests from the same values).  A centre that single
// precision places clearly inside all three edges is written at once (64-bit
// atomicMin of the packed depth/id key); one that lies within a rounding
// margin of an edge, or any centre of a triangle seen nearly edge-on, is
// queued and decided afterwards by covered_exact.  Must be called by the whole
// block; ends after a barrier with the buffer complete.
template <bool COUNT, bool BIG>
__device__ __forceinline__ void raster_mesh(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id_base,
                                            const Rect& band, const Rect& buf, unsigned long long* zbuf,
                                            const RasterLds& lds, unsigned* cnt = nullptr) {
  unsigned c_vert = 0, c_tri = 0, c_setup = 0, c_frag = 0, c_exact = 0;
  const int pitch = buf.w();
  const float bx0 = (float)band.x0, bx1 = (float)(band.x1 - 1);
  const float by0 = (float)band.y0, by1 = (float)(band.y1 - 1);
  if (threadIdx.x == 0) lds.counts[0] = 0;
  // the hidden-pair clusters matter only when the object reaches the near plane
  bool straddle = false;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float3 c = xform(P, (k & 1) ? m.hi[0] : m.lo[0], (k & 2) ? m.hi[1] : m.lo[1], (k & 4) ? m.hi[2] : m.lo[2]);
    straddle = straddle || !(c.z > cam.znear);
  }
  const int n_clusters = straddle ? m.n_clusters : m.n_visible;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = 0; base < n_clusters; base += kBlock) {
    // each thread tests one cluster; the drawable ones are compacted into `list`
    const int mine = base + threadIdx.x;
    float box[4], zmin;
    const bool draw = mine < n_clusters && cluster_may_draw(m.clusters[mine], P, cam, band, box, &zmin);
    const unsigned long long mask = __ballot(draw);
    __syncthreads();  // the previous group's list is no longer read
    if (lane == 0) lds.counts[1 + wave] = __popcll(mask);
    if (threadIdx.x == 0) lds.counts[1 + kWaves] = 0;
    __syncthreads();
    int off = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
      off += (w < wave) ? lds.counts[1 + w] : 0;
      total += lds.counts[1 + w];
    }
    if (draw) lds.list[off + __popcll(mask & ((1ull << lane) - 1ull))] = mine;
    __syncthreads();
    for (;;) {
      int q = 0;
      if (lane == 0) q = atomicAdd(&lds.counts[1 + kWaves], 1);
      q = __shfl(q, 0, 64);
      if (q >= total) break;
      const ClusterDev cl = m.clusters[lds.list[q]];
      bool staged = false;
      if (lane < cl.np) {
        const size_t pi = (size_t)cl.pfirst + lane;
        const uint2 ids = m.pids[pi];
        const bool quad = ids.y != kNoTri;
        // corners as (u, v, z, 1/z); triangle 1 = (a, b, c), triangle 2 = (a, c, d)
        const float4* pv = m.pverts + 4 * pi;
        const float4 A = project_corner(P, cam, pv[0]), B = project_corner(P, cam, pv[1]);
        const float4 C = project_corner(P, cam, pv[2]), D = project_corner(P, cam, pv[3]);
        if (COUNT) {
          c_vert += 4;
          c_tri += quad ? 2 : 1;
        }
        const float zn = cam.znear;
        const bool near1 = A.z <= zn || B.z <= zn || C.z <= zn;
        const bool near2 = A.z <= zn || C.z <= zn || D.z <= zn;
        // edges of triangle 1 (e_k opposite corner k) and of triangle 2 (f_k); the
        // diagonal a-c is e1 (c -> a) for triangle 1 and -e1 for triangle 2
        const float e0x = C.x - B.x, e0y = C.y - B.y;
        const float e1x = A.x - C.x, e1y = A.y - C.y;
        const float e2x = B.x - A.x, e2y = B.y - A.y;
        const float f0x = D.x - C.x, f0y = D.y - C.y;
        const float f1x = A.x - D.x, f1y = A.y - D.y;
        // rounding margin (pixels) from the magnitudes of the corners in use
        float mag = fmaxf(fmaxf(fabsf(A.x), fabsf(A.y)), fmaxf(fabsf(C.x), fabsf(C.y)));
        const float area1 = e2x * (C.y - A.y) - (C.x - A.x) * e2y;
        const float area2 = -e1x * (D.y - A.y) + (D.x - A.x) * e1y;
        // preliminary activity (near plane) decides which corners set the margin
        const bool use1 = !near1, use2 = quad && !near2;
        mag = fmaxf(mag, use1 ? fmaxf(fabsf(B.x), fabsf(B.y)) : 0.0f);
        mag = fmaxf(mag, use2 ? fmaxf(fabsf(D.x), fabsf(D.y)) : 0.0f);
        const float tau = 2e-6f * fmaxf(mag, 256.0f);
        const float amb1 = 2.0f * tau * (fabsf(e1x) + fabsf(e1y) + fabsf(e2x) + fabsf(e2y));
        const float amb2 = 2.0f * tau * (fabsf(f1x) + fabsf(f1y) + fabsf(e1x) + fabsf(e1y));
        // drawn unless behind the near plane or facing away
        const bool act1 = use1 && !(area1 > amb1);
        const bool act2 = use2 && !(area2 > amb2);
        // box of the active triangles' corners (a and c belong to both)
        const float bxu = act1 ? B.x : A.x, bxv = act1 ? B.y : A.y;
        const float dxu = act2 ? D.x : A.x, dxv = act2 ? D.y : A.y;
        const float umin = fminf(fminf(A.x, C.x), fminf(bxu, dxu)), umax = fmaxf(fmaxf(A.x, C.x), fmaxf(bxu, dxu));
        const float vmin = fminf(fminf(A.y, C.y), fminf(bxv, dxv)), vmax = fmaxf(fmaxf(A.y, C.y), fmaxf(bxv, dxv));
        const float fc0 = ceilf(fmaxf(umin - 0.5f - tau, bx0)), fc1 = floorf(fminf(umax - 0.5f + tau, bx1));
        const float fr0 = ceilf(fmaxf(vmin - 0.5f - tau, by0)), fr1 = floorf(fminf(vmax - 0.5f + tau, by1));
        if ((act1 || act2) && fc0 <= fc1 && fr0 <= fr1) {
          const int c0 = (int)fc0, c1 = (int)fc1, r0 = (int)fr0, r1 = (int)fr1;
          if (COUNT) c_setup += (act1 ? 1u : 0u) + (act2 ? 1u : 0u);
          const bool eon1 = area1 >= -amb1, eon2 = area2 >= -amb2;
          const float ia1 = __builtin_amdgcn_rcpf(area1), ia2 = __builtin_amdgcn_rcpf(area2);
          const float t0 = tau * (fabsf(e0x) + fabsf(e0y)), t1 = tau * (fabsf(e1x) + fabsf(e1y)),
                      t2 = tau * (fabsf(e2x) + fabsf(e2y));
          const float s0 = tau * (fabsf(f0x) + fabsf(f0y)), s1 = tau * (fabsf(f1x) + fabsf(f1y));
          // a centre of triangle k: queued for the exact test when within the
          // margin of an edge (or the triangle is nearly edge-on), else written
          // edge functions (each the negative area at the opposite corner) at the
          // box's first centre; at a centre dr rows and dc columns further they
          // are w + e_x dr - e_y dc with exact small integers dr, dc: two FMAs
          // each, and the rounding stays far below the margin for any box size
          const float py0 = (float)r0 + 0.5f, px0 = (float)c0 + 0.5f;
          const float w0b = e0x * (py0 - B.y) - e0y * (px0 - B.x);
          const float w1b = e1x * (py0 - C.y) - e1y * (px0 - C.x);
          const float w2b = e2x * (py0 - A.y) - e2y * (px0 - A.x);
          const float v0b = f0x * (py0 - C.y) - f0y * (px0 - C.x);
          const float v1b = f1x * (py0 - D.y) - f1y * (px0 - D.x);
          // one flat walk over the box's centres: a wave then iterates max(rows x cols)
          // times over its lanes, not max(rows) x max(cols)
          int n_cent = (c1 - c0 + 1) * (r1 - r0 + 1);
          // a large box (a table top, a wall) would keep this lane walking long
          // after the others are done: the first kBigSlots of them are staged in
          // the wave's LDS slots and walked by the whole wave below
          const unsigned long long bigm = BIG ? __ballot(n_cent > kBigCentres) : 0ull;
          if (BIG && bigm != 0ull && n_cent > kBigCentres && __popcll(bigm & ((1ull << lane) - 1ull)) < kBigSlots) {
            const int rank = __popcll(bigm & ((1ull << lane) - 1ull));
            float* st = raster_stage(lds) + (wave * kBigSlots + rank) * kStageWords;
            int* si = reinterpret_cast<int*>(st);
            const float vals[26] = {e0x, e0y, e1x, e1y, e2x, e2y, f0x, f0y, f1x, f1y, t0,  t1,  t2,
                                    s0,  s1,  ia1, ia2, w0b, w1b, w2b, v0b, v1b, A.w, B.w, C.w, D.w};
#pragma unroll
            for (int k = 0; k < 26; ++k) st[k] = vals[k];
            si[kStBox] = c0;
            si[kStBox + 1] = c1;
            si[kStBox + 2] = r0;
            si[kStBox + 3] = r1;
            si[kStIds] = (int)ids.x;
            si[kStIds + 1] = (int)ids.y;
            si[kStFlags] = (act1 ? 1 : 0) | (act2 ? 2 : 0) | (eon1 ? 4 : 0) | (eon2 ? 8 : 0);
            staged = true;
            n_cent = 0;
          }
          // the offsets from the box's first centre as exact small floats,
          // stepped along the row and wrapped to the next one
          const float dcmax = (float)(c1 - c0), drmax = n_cent > 0 ? (float)(r1 - r0) : -1.0f;
          float dr = 0.0f, dc = 0.0f;
          while (dr <= drmax) {
            const float drn = dc < dcmax ? dr : dr + 1.0f;
            const float dcn = dc < dcmax ? dc + 1.0f : 0.0f;
            const float w0 = __builtin_fmaf(-e0y, dc, __builtin_fmaf(e0x, dr, w0b));
            const float w1 = __builtin_fmaf(-e1y, dc, __builtin_fmaf(e1x, dr, w1b));
            const float w2 = __builtin_fmaf(-e2y, dc, __builtin_fmaf(e2x, dr, w2b));
            const float v0 = __builtin_fmaf(-f0y, dc, __builtin_fmaf(f0x, dr, v0b));
            const float v1 = __builtin_fmaf(-f1y, dc, __builtin_fmaf(f1x, dr, v1b));
            const bool out1 = !act1 || w0 > t0 || w1 > t1 || w2 > t2;
            const bool out2 = !act2 || v0 > s0 || v1 > s1 || -w1 > t1;
            const float drc = dr, dcc = dc;
            dr = drn;
            dc = dcn;
            if (out1 && out2) continue;  // clearly outside both
            const int r = r0 + (int)drc, col = c0 + (int)dcc;
            const int pix = (r - buf.y0) * pitch + (col - buf.x0);
            if (!out1)
              emit_centre<COUNT>(pix, eon1, w0, w1, w2, t0, t1, t2, A.w, B.w, C.w, ia1, ids.x, id_base, zbuf, lds,
                                 c_frag);
            if (!out2)
              emit_centre<COUNT>(pix, eon2, v0, v1, -w1, s0, s1, t1, A.w, C.w, D.w, ia2, ids.y, id_base, zbuf, lds,
                                 c_frag);
          }
        }
      }
      if constexpr (BIG) {
        __builtin_amdgcn_wave_barrier();
        const unsigned long long sm = __ballot(staged);
        if (sm != 0ull) {
          const int n_staged = __popcll(sm);
          for (int j = 0; j < n_staged; ++j)
            walk_staged<COUNT>(raster_stage(lds) + (wave * kBigSlots + j) * kStageWords, lane, buf, pitch, id_base,
                               zbuf, lds, c_frag);
        }
      }
    }
  }
  __syncthreads();
  // centres near an edge: the exact test, then the plane depth
  const int nq = min(lds.counts[0], lds.qcap);
  for (int k = threadIdx.x; k < nq; k += kBlock) {
    const uint2 e = lds.queue[k];
    const int r = buf.y0 + (int)e.x / pitch, col = buf.x0 + (int)e.x % pitch;
    if (COUNT) ++c_exact;
    if (!covered_exact(m, P, cam, e.y, r, col)) continue;
    const float z = plane_depth(m, P, cam, e.y, r, col);
    if (!(z > 0.0f)) continue;
    if (COUNT) ++c_frag;
    atomicMin(&zbuf[e.x], pack_key(z, id_base + e.y));
  }
  if (COUNT) {
    atomicAdd(&cnt[kCntVert], c_vert);
    atomicAdd(&cnt[kCntTri], c_tri);
    atomicAdd(&cnt[kCntSetup], c_setup);
    atomicAdd(&cnt[kCntFrag], c_frag);
    atomicAdd(&cnt[kCntExact], c_exact);
  }
  __syncthreads();
}

// Which rasteriser a kernel holds: the plain one, the one with the wave walk
// of large boxes, or both behind a test of the mesh's has_big (the large-box
// walk costs meshes without large primitives a few per cent).
enum RasterMode { kRasterSmall = 0, kRasterBig = 1, kRasterAny = 2 };

template <bool COUNT, int MODE>
__device__ __forceinline__ void raster_mesh_mode(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id_base,
                                                 const Rect& band, const Rect& buf, unsigned long long* zbuf,
                                                 const RasterLds& lds, unsigned* cnt = nullptr) {
  if (MODE == kRasterBig || (MODE == kRasterAny && m.has_big)) {
    RasterLds shorter = lds;
    shorter.qcap = kQueueCap - kStageQueueEntries;
    raster_mesh<COUNT, true>(m, P, cam, id_base, band, buf, zbuf, shorter, cnt);
  } else {
    raster_mesh<COUNT, false>(m, P, cam, id_base, band, buf, zbuf, lds, cnt);
  }
}

template <bool COUNT = false>
__device__ __forceinline__ void raster_mesh_any(const MeshDev& m, const Pose& P, const Cam& cam, uint32_t id_base,
                                                const Rect& band, const Rect& buf, unsigned long long* zbuf,
                                                const RasterLds& lds, unsigned* cnt = nullptr) {
  raster_mesh_mode<COUNT, kRasterAny>(m, P, cam, id_base, band, buf, zbuf, lds, cnt);
}

// One Adam ascent step on logL for pose P (row-major 4x4), on the tangent
// (dt, dw): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// s = lr * mhat / (sqrt(vhat) + eps), then t <- t + s[0:3], R <- exp([s[3:6]]x) R.
__device__ __forceinline__ void adam_update(float* P, const float* g, float* m, float* v, int iter, float lr_t,
                                            float lr_r, float b1, float b2, float eps) {
  const float c1 = 1.0f - powf(b1, (float)iter), c2 = 1.0f - powf(b2, (float)iter);
  float s[6];
  for (int k = 0; k < 6; ++k) {
    m[k] = b1 * m[k] + (1.0f - b1) * g[k];
    v[k] = b2 * v[k] + (1.0f - b2) * g[k] * g[k];
    const float mh = m[k] / c1, vh = v[k] / c2;
    s[k] = (k < 3 ? lr_t : lr_r) * mh / (sqrtf(vh) + eps);
  }
  for (int k = 0; k < 3; ++k) P[4 * k + 3] += s[k];
  const float wx = s[3], wy = s[4], wz = s[5];
  const float th = sqrtf(wx * wx + wy * wy + wz * wz);
  if (th > 0.0f) {
    const float kx = wx / th, ky = wy / th, kz = wz / th;
    const float sn = sinf(th), cs = 1.0f - cosf(th);
    const float E[9] = {1.0f + cs * (kx * kx - 1.0f), -sn * kz + cs * kx * ky,       sn * ky + cs * kx * kz,
                        sn * kz + cs * kx * ky,       1.0f + cs * (ky * ky - 1.0f), -sn * kx + cs * ky * kz,
                        -sn * ky + cs * kx * kz,      sn * kx + cs * ky * kz,       1.0f + cs * (kz * kz - 1.0f)};
    float R[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) R[3 * i + j] = E[3 * i] * P[j] + E[3 * i + 1] * P[4 + j] + E[3 * i + 2] * P[8 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P[4 * i + j] = R[3 * i + j];
  }
}

// Fixed-order sum over the 64 lanes of a wave (butterfly), result in all lanes.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block sum of NV floats; the result is valid in thread 0.
// `red` must hold kWaves * NV floats of LDS.
template <int NV>
__device__ __forceinline__ void block_sum(float (&v)[NV], float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      float s = red[k];
      for (int w = 1; w < kWaves; ++w) s += red[w * NV + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

}  // namespace b3d

// C ABI of the b3d library: argument validation, error reporting, device
// mesh layout, scenes, and the host side of the coarse-to-fine stage loop.
// Nothing here computes on the host beyond set-up (mesh clustering, bounds,
// constants); every step of the hot path runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "api_internal.hpp"
#include "b3d_mesh_layout.hpp"

using namespace b3d;

namespace b3d_api {

thread_local std::string g_err;

b3d_status fail(b3d_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

b3d_status hip_fail(hipError_t e, const char* where) {
  return fail(B3D_EHIP, "%s: %s", where, hipGetErrorString(e));
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

b3d_status check_intrinsics(const b3d_intrinsics* K) {
  if (!K) return fail(B3D_EINVAL, "intrinsics pointer is NULL");
  if (!(K->fx > 0) || !(K->fy > 0) || !std::isfinite(K->fx) || !std::isfinite(K->fy) || !std::isfinite(K->cx) ||
      !std::isfinite(K->cy))
    return fail(B3D_EINVAL, "intrinsics: fx, fy must be > 0 and all values finite");
  if (!(K->z_near > 0) || !std::isfinite(K->z_near)) return fail(B3D_EINVAL, "intrinsics: z_near must be > 0");
  if (K->H < 1 || K->W < 1 || K->H > kMaxImage || K->W > kMaxImage)
    return fail(B3D_ESHAPE, "image size %dx%d outside 1..%d", K->H, K->W, kMaxImage);
  return B3D_OK;
}

Cam make_cam(const b3d_intrinsics* K) {
  Cam c;
  c.fx = K->fx;
  c.fy = K->fy;
  c.cx = K->cx;
  c.cy = K->cy;
  c.znear = K->z_near;
  c.H = K->H;
  c.W = K->W;
  return c;
}

b3d_status make_consts(const b3d_score_params* p, int H, int W, ScoreConsts* sc) {
  if (!p) return fail(B3D_EINVAL, "score params pointer is NULL");
  if (!(p->sigma > 0) || !std::isfinite(p->sigma)) return fail(B3D_EINVAL, "sigma must be > 0 (got %g)", p->sigma);
  if (!(p->p_out > 0) || !(p->p_out <= 1)) return fail(B3D_EINVAL, "p_out must be in (0, 1] (got %g)", p->p_out);
  if (!(p->outlier_volume > 0) || !std::isfinite(p->outlier_volume))
    return fail(B3D_EINVAL, "outlier_volume must be > 0");
  if (p->window < 1 || p->window > 15 || (p->window % 2) == 0)
    return fail(B3D_EINVAL, "window must be odd and in 1..15 (got %d)", p->window);
  if (!std::isfinite(p->norm_M)) return fail(B3D_EINVAL, "norm_M must be finite");
  const double M = p->norm_M > 0 ? (double)p->norm_M : (double)H * (double)W;
  const double s = p->sigma, V = p->outlier_volume, po = p->p_out;
  const double norm = std::pow(2.0 * M_PI * s * s, -1.5);
  sc->da = po / V;
  sc->dbn = (1.0 - po) / M * norm;
  sc->dc = 1.0 / (2.0 * s * s);
  sc->dinv_s = 1.0 / s;
  sc->dinv_s3 = 1.0 / (s * s * s);
  sc->dinvV = 1.0 / V;
  sc->dnormM = norm / M;
  sc->a = (float)sc->da;
  sc->bn = (float)sc->dbn;
  sc->c2 = (float)(sc->dc / std::log(2.0));
  sc->inv_s = (float)sc->dinv_s;
  sc->inv_s2 = (float)(1.0 / (s * s));
  sc->inv_s3 = (float)sc->dinv_s3;
  sc->invV = (float)sc->dinvV;
  sc->normM = (float)sc->dnormM;
  sc->h = (p->window - 1) / 2;
  return B3D_OK;
}

int default_zcap(const SceneDev& d, int blocks_per_cu) {
  SceneDev t = d;
  t.zcap = 0;
  const size_t share = (160 * 1024) / (size_t)blocks_per_cu;
  const size_t rest = fused_lds_bytes(t);
  return (int)((share > rest ? share - rest : 0) / kFusedBytesPerKey);
}

// two rows of the widest depth buffer (image width plus 2h each side)
int min_zcap(const SceneDev& d) { return (4 * d.sc.h + 2) * (d.cam.W + 4 * d.sc.h); }

int max_zcap(const SceneDev& d) {
  SceneDev t = d;
  t.zcap = 0;
  const size_t rest = fused_lds_bytes(t);
  // also bounded by the drawn-slot list, which lives in the raster scratch
  return (int)std::min<size_t>((kLdsMax > rest ? kLdsMax - rest : 0) / kFusedBytesPerKey, kRasterLdsBytes / 2);
}

b3d_status make_noise_grid(const b3d_score_params& base, int H, int W, const float* sigma, int A, const float* p_out,
                           int B, const float* log_w, NoiseGridDev* g, std::vector<b3d_score_params>* per_point) {
  if (A < 1 || A > kMaxSigma || B < 1 || A * B > kMaxNoise)
    return fail(B3D_ESHAPE, "noise grid: need 1 <= A <= %d, B >= 1, A*B <= %d", kMaxSigma, kMaxNoise);
  *g = NoiseGridDev{};
  g->A = A;
  g->B = B;
  per_point->clear();
  for (int ia = 0; ia < A; ++ia)
    for (int ib = 0; ib < B; ++ib) {
      b3d_score_params p = base;
      p.sigma = sigma[ia];
      p.p_out = p_out[ib];
      ScoreConsts sc;
      if (b3d_status s = make_consts(&p, H, W, &sc)) return s;
      const int k = ia * B + ib;
      g->c2[ia] = sc.c2;
      g->normM[ia] = sc.normM;
      g->ka[k] = ia;
      g->pa[k] = sc.a;
      g->pomp[k] = (float)(1.0 - (double)p.p_out);
      const float lw = log_w ? log_w[k] : (float)(-std::log((double)A * B));
      if (!std::isfinite(lw)) return fail(B3D_EINVAL, "noise grid: non-finite log weight %d", k);
      g->logw[k] = lw;
      per_point->push_back(p);
    }
  return B3D_OK;
}

}  // namespace b3d_api

using namespace b3d_api;

struct b3d_batch {
  BatchPlan plan;
  // a second stream for every other launch, forked from and joined back into
  // the caller's stream on each run (default priority, non-blocking)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct b3d_tracker;


// Background-only per-pixel terms of every noise-grid point, as summed-area
// tables (stream-ordered; the scene's own terms buffer is reused).
static b3d_status grid_background(b3d_scene* S, hipStream_t st) {
  const size_t SP = (size_t)(S->K.H + 1) * (S->K.W + 1);
  for (size_t k = 0; k < S->grid_params.size(); ++k) {
    SceneDev t = S->dev;
    if (b3d_status s = make_consts(&S->grid_params[k], S->K.H, S->K.W, &t.sc)) return s;
    t.sat = S->grid_sat + 3 * SP * k;
    B3D_CHECK_HIP(launch_background_terms(t, S->terms, st), "noise grid");
  }
  return B3D_OK;
}

extern "C" {

const char* b3d_last_error(void) { return g_err.c_str(); }

const char* b3d_version(void) { return "b3d 0.1.0 (gfx950)"; }

b3d_status b3d_mesh_create(const float* verts, int32_t V, const int32_t* tris, int32_t T, b3d_mesh** out) {
  if (!verts || !tris || !out) return fail(B3D_EINVAL, "mesh_create: NULL pointer");
  if (V < 1 || T < 1 || T > (1 << 24)) return fail(B3D_ESHAPE, "mesh_create: need V >= 1 and 1 <= T <= 2^24");
  if (!finite_all(verts, (size_t)V * 3)) return fail(B3D_EINVAL, "mesh_create: non-finite vertex");
  for (int64_t i = 0; i < (int64_t)T * 3; ++i)
    if (tris[i] < 0 || tris[i] >= V) return fail(B3D_EINVAL, "mesh_create: triangle index out of range");

  MeshLayout lay = build_mesh_layout(verts, V, tris, T);
  if (lay.clusters.empty()) {  // every triangle has a repeated vertex: nothing is ever drawn
    lay.clusters.push_back(ClusterDev{});
    lay.clusters.back().cone = make_float4(0.0f, 0.0f, 1.0f, 4.0f);
    lay.n_visible = 0;
  }
  if (lay.pverts.empty()) lay.pverts.assign(4, make_float4(0, 0, 0, 0));
  if (lay.pids.empty()) lay.pids.push_back(make_uint2(0, kNoTri));
  std::vector<float4> v4((size_t)V), nrm((size_t)T);
  std::vector<int4> t4((size_t)T);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int i = 0; i < V; ++i) {
    v4[i] = make_float4(verts[3 * i], verts[3 * i + 1], verts[3 * i + 2], 0.0f);
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], (double)verts[3 * i + k]);
      hi[k] = std::max(hi[k], (double)verts[3 * i + k]);
    }
  }
  for (int t = 0; t < T; ++t) {
    const int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    t4[t] = make_int4(a, b, c, 0);
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = (double)verts[3 * b + k] - verts[3 * a + k];
      e2[k] = (double)verts[3 * c + k] - verts[3 * a + k];
    }
    nrm[t] = make_float4((float)(e1[1] * e2[2] - e1[2] * e2[1]), (float)(e1[2] * e2[0] - e1[0] * e2[2]),
                         (float)(e1[0] * e2[1] - e1[1] * e2[0]), 0.0f);
  }
  double ctr[3], rad = 0.0;
  for (int k = 0; k < 3; ++k) ctr[k] = 0.5 * (lo[k] + hi[k]);
  for (int i = 0; i < V; ++i) {
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) d2 += (verts[3 * i + k] - ctr[k]) * (verts[3 * i + k] - ctr[k]);
    rad = std::max(rad, std::sqrt(d2));
  }

  b3d_mesh* m = new b3d_mesh();
  m->V = V;
  for (int k = 0; k < 3; ++k) {
    m->box_lo[k] = (float)lo[k];
    m->box_hi[k] = (float)hi[k];
  }
  m->T = T;
  m->n_clusters = lay.n_visible == 0 && lay.n_hidden == 0 ? 0 : (int)lay.clusters.size();
  auto upload = [&](const void* src, size_t bytes, void** dst) -> bool {
    if (hipMalloc(dst, bytes) != hipSuccess) return false;
    m->allocs.push_back(*dst);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  void *d_cl, *d_cv, *d_ct, *d_v, *d_t, *d_n;
  bool ok = upload(lay.clusters.data(), std::max<size_t>(1, lay.clusters.size()) * sizeof(ClusterDev), &d_cl) &&
            upload(lay.pverts.data(), lay.pverts.size() * sizeof(float4), &d_cv) &&
            upload(lay.pids.data(), lay.pids.size() * sizeof(uint2), &d_ct) &&
            upload(v4.data(), v4.size() * sizeof(float4), &d_v) && upload(t4.data(), t4.size() * sizeof(int4), &d_t) &&
            upload(nrm.data(), nrm.size() * sizeof(float4), &d_n);
  if (!ok) {
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
    return fail(B3D_ENOMEM, "mesh_create: device allocation or copy failed");
  }
  MeshDev& d = m->dev;
  d.clusters = (const ClusterDev*)d_cl;
  d.pverts = (const float4*)d_cv;
  d.pids = (const uint2*)d_ct;
  d.n_visible = lay.n_visible;
  d.verts = (const float4*)d_v;
  d.tris = (const int4*)d_t;
  d.normals = (const float4*)d_n;
  d.n_clusters = m->n_clusters;
  m->n_drawn = lay.n_drawn;
  m->n_hidden = lay.n_hidden;
  m->n_dropped = lay.n_dropped;
  d.T = T;
  for (int k = 0; k < 3; ++k) {
    // widen by a relative epsilon so that float rounding keeps the bounds conservative
    const double pad = 1e-6 * (std::fabs(lo[k]) + std::fabs(hi[k]) + rad) + 1e-7;
    d.lo[k] = (float)(lo[k] - pad);
    d.hi[k] = (float)(hi[k] + pad);
    d.sphere[k] = (float)ctr[k];
  }
  d.sphere[3] = (float)(rad * (1.0 + 1e-6) + 1e-7);
  // large primitives (relative to the whole mesh) select the rasteriser's
  // wave walk of large screen boxes; results are the same either way
  double diag2 = 0.0;
  for (int k = 0; k < 3; ++k) diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  d.has_big = 0;
  for (size_t q = 0; q + 3 < lay.pverts.size() && !d.has_big; q += 4) {
    for (int a = 0; a < 4 && !d.has_big; ++a)
      for (int b = a + 1; b < 4; ++b) {
        const float4 u = lay.pverts[q + a], w = lay.pverts[q + b];
        const double dx = (double)u.x - w.x, dy = (double)u.y - w.y, dz = (double)u.z - w.z;
        if (64.0 * (dx * dx + dy * dy + dz * dz) > diag2) d.has_big = 1;
      }
  }
  *out = m;
  return B3D_OK;
}

b3d_status b3d_mesh_destroy(b3d_mesh* m) {
  if (!m) return B3D_OK;
  (void)hipDeviceSynchronize();
  for (void* p : m->allocs) (void)hipFree(p);
  delete m;
  return B3D_OK;
}

b3d_status b3d_mesh_layout_info(const float* verts, int32_t V, const int32_t* tris, int32_t T, int32_t* info) {
  if (!verts || !tris || !info) return fail(B3D_EINVAL, "mesh_layout_info: NULL pointer");
  if (V < 1 || T < 1 || T > (1 << 24)) return fail(B3D_ESHAPE, "mesh_layout_info: need V >= 1 and 1 <= T <= 2^24");
  for (int64_t i = 0; i < (int64_t)T * 3; ++i)
    if (tris[i] < 0 || tris[i] >= V) return fail(B3D_EINVAL, "mesh_layout_info: triangle index out of range");
  const MeshLayout lay = build_mesh_layout(verts, V, tris, T);
  info[0] = (int32_t)lay.clusters.size();
  info[1] = lay.n_visible;
  info[2] = lay.n_drawn;
  info[3] = lay.n_hidden;
  info[4] = lay.n_dropped;
  info[5] = lay.n_quads;
  return B3D_OK;
}

b3d_status b3d_mesh_info(const b3d_mesh* m, int32_t* V, int32_t* T, int32_t* n_clusters) {
  if (!m) return fail(B3D_EINVAL, "mesh_info: NULL mesh");
  if (V) *V = m->V;
  if (T) *T = m->T;
  if (n_clusters) *n_clusters = m->n_clusters;
  return B3D_OK;
}

b3d_status b3d_unproject(const float* depth, int32_t B, const b3d_intrinsics* K, float* xyz, void* stream) {
  if (b3d_status s = check_intrinsics(K)) return s;
  if (B < 0) return fail(B3D_ESHAPE, "unproject: B < 0");
  if (B == 0) return B3D_OK;
  if (!depth || !xyz) return fail(B3D_EINVAL, "unproject: NULL pointer");
  B3D_CHECK_HIP(launch_unproject(depth, B, make_cam(K), xyz, (hipStream_t)stream), "unproject");
  return B3D_OK;
}

b3d_status b3d_render_batch(const b3d_mesh* mesh, const float* poses, int32_t N, const b3d_intrinsics* K,
                            float* xyz_out, int32_t* tri_out, void* stream) {
  if (!mesh) return fail(B3D_EINVAL, "render_batch: NULL mesh");
  if (b3d_status s = check_intrinsics(K)) return s;
  if (N < 0) return fail(B3D_ESHAPE, "render_batch: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !xyz_out) return fail(B3D_EINVAL, "render_batch: NULL pointer");
  // a depth buffer of 2048 keys (or one image row) leaves room for five workgroups per CU
  const int zcap = std::max(2048, K->W);
  if (kRasterLdsBytes + 8 * (size_t)zcap > kLdsMax)
    return fail(B3D_ESHAPE, "render_batch: image too wide for the LDS depth buffer");
  B3D_CHECK_HIP(launch_render_batch(mesh->dev, make_cam(K), poses, N, xyz_out, tri_out, zcap, (hipStream_t)stream),
                "render_batch");
  return B3D_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

static int score_cap(int W, int h, int planes, int halo_rows, int want) {
  // floats of LDS for staged rows: at least one output row plus halo
  const int need = planes * W * (1 + halo_rows * h);
  if (need > 16384 - 64) return -1;
  return std::max(need, want);
}

b3d_status b3d_score_workspace_size(int32_t H, int32_t W, size_t* bytes) {
  if (!bytes) return fail(B3D_EINVAL, "score_workspace_size: NULL output");
  if (H < 1 || W < 1 || H > kMaxImage || W > kMaxImage) return fail(B3D_ESHAPE, "score_workspace_size: bad H or W");
  *bytes = score_workspace_bytes(H, W);
  return B3D_OK;
}

b3d_status b3d_score(const float* observed, const float* rendered, int32_t N, int32_t H, int32_t W,
                     const b3d_score_params* p, float* logL_out, void* workspace, size_t ws_bytes, void* stream) {
  if (N < 0 || H < 1 || W < 1 || H > kMaxImage || W > kMaxImage) return fail(B3D_ESHAPE, "score: bad N, H or W");
  ScoreConsts sc;
  if (b3d_status s = make_consts(p, H, W, &sc)) return s;
  if (N == 0) return B3D_OK;
  if (!observed || !rendered || !logL_out) return fail(B3D_EINVAL, "score: NULL pointer");
  if (workspace && ws_bytes < score_workspace_bytes(H, W))
    return fail(B3D_ESHAPE, "score: workspace of %zu bytes < %zu", ws_bytes, score_workspace_bytes(H, W));
  const int R = score_ring_rows(H, W, sc.h);
  if (workspace && R > 0 && aligned16(rendered) && aligned16(workspace)) {
    B3D_CHECK_HIP(launch_score_ring(observed, rendered, N, H, W, sc, R, workspace, logL_out, (hipStream_t)stream),
                  "score");
    return B3D_OK;
  }
  const int cap = score_cap(W, sc.h, 3, 2, 10240 - 64);  // four workgroups per CU
  if (cap < 0) return fail(B3D_ESHAPE, "score: image too wide for the LDS row buffer");
  B3D_CHECK_HIP(launch_score(observed, rendered, N, H, W, sc, logL_out, cap, (hipStream_t)stream), "score");
  return B3D_OK;
}

b3d_status b3d_score_backward(const float* observed, const float* rendered, int32_t N, int32_t H, int32_t W,
                              const b3d_score_params* p, const float* dlogL, float* d_rendered, float* d_sigma,
                              float* d_pout, void* workspace, size_t ws_bytes, void* stream) {
  if (N < 0 || H < 1 || W < 1 || H > kMaxImage || W > kMaxImage)
    return fail(B3D_ESHAPE, "score_backward: bad N, H or W");
  ScoreConsts sc;
  if (b3d_status s = make_consts(p, H, W, &sc)) return s;
  if (N == 0) return B3D_OK;
  if (!observed || !rendered) return fail(B3D_EINVAL, "score_backward: NULL pointer");
  if (!d_rendered && !d_sigma && !d_pout) return B3D_OK;
  if (workspace && ws_bytes < score_workspace_bytes(H, W))
    return fail(B3D_ESHAPE, "score_backward: workspace of %zu bytes < %zu", ws_bytes, score_workspace_bytes(H, W));
  const int R = score_backward_ring_rows(H, W, sc.h);
  if (workspace && R > 0 && aligned16(rendered) && aligned16(d_rendered) && aligned16(workspace)) {
    B3D_CHECK_HIP(launch_score_backward_ring(observed, rendered, N, H, W, sc, R, workspace, dlogL, d_rendered, d_sigma,
                                             d_pout, (hipStream_t)stream),
                  "score_backward");
    return B3D_OK;
  }
  const int cap = score_cap(W, sc.h, 4, 4, 16384 - 64);
  if (cap < 0) return fail(B3D_ESHAPE, "score_backward: image too wide for the LDS row buffer");
  B3D_CHECK_HIP(launch_score_backward(observed, rendered, N, H, W, sc, dlogL, d_rendered, d_sigma, d_pout, cap,
                                      (hipStream_t)stream),
                "score_backward");
  return B3D_OK;
}

b3d_status b3d_render_backward(const b3d_mesh* mesh, const float* poses, int32_t N, const b3d_intrinsics* K,
                               const int32_t* tri, const float* d_rendered, float* d_pose, void* stream) {
  if (!mesh) return fail(B3D_EINVAL, "render_backward: NULL mesh");
  if (b3d_status s = check_intrinsics(K)) return s;
  if (N < 0) return fail(B3D_ESHAPE, "render_backward: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !tri || !d_rendered || !d_pose) return fail(B3D_EINVAL, "render_backward: NULL pointer");
  B3D_CHECK_HIP(launch_render_backward(mesh->dev, make_cam(K), poses, N, tri, d_rendered, d_pose, (hipStream_t)stream),
                "render_backward");
  return B3D_OK;
}

b3d_status b3d_scene_create(const b3d_mesh* mesh, const b3d_intrinsics* K, const b3d_score_params* p,
                            b3d_scene** out) {
  if (!mesh || !out) return fail(B3D_EINVAL, "scene_create: NULL pointer");
  if (b3d_status s = check_intrinsics(K)) return s;
  ScoreConsts sc;
  if (b3d_status s = make_consts(p, K->H, K->W, &sc)) return s;
  b3d_scene* S = new b3d_scene();
  S->mesh = mesh;
  S->K = *K;
  S->params = *p;
  S->dev.mesh = mesh->dev;
  S->dev.cam = make_cam(K);
  S->dev.sc = sc;
  const int h = sc.h, W = K->W;
  {
    // the fused kernel's empty depth slots rely on rays with |x/z|, |y/z| <= 1e3
    // over the image and 2h pixels beyond it
    const double rx = std::max(std::fabs((-2.0 * h + 0.5 - K->cx) / K->fx), std::fabs((W + 2.0 * h - 0.5 - K->cx) / K->fx));
    const double ry =
        std::max(std::fabs((-2.0 * h + 0.5 - K->cy) / K->fy), std::fabs((K->H + 2.0 * h - 0.5 - K->cy) / K->fy));
    if (!(rx <= 1e3 && ry <= 1e3)) {
      delete S;
      return fail(B3D_ESHAPE, "scene_create: field of view too wide (|x/z| or |y/z| above 1e3 at the image edge)");
    }
  }
  // window weights live in the rasteriser's scratch once the depth buffer is done
  S->dev.wcap = (int)(kRasterLdsBytes / sizeof(float));
  // depth keys: as many as leave room for four workgroups per CU (160 KB of LDS)
  S->dev.zcap = std::max(default_zcap(S->dev, 4), min_zcap(S->dev));
  // one band row of window weights must leave a round of the drawn-pixel list
  if ((2 * h + 1) * W > S->dev.wcap || 4 * (size_t)(2 * h + 1) * W + 2 * kBlock > kRasterLdsBytes ||
      S->dev.zcap > max_zcap(S->dev) || fused_lds_bytes(S->dev) > kLdsMax) {
    delete S;
    return fail(B3D_ESHAPE, "scene_create: image width %d too large for the fused kernel's LDS budget", W);
  }
  const size_t HW = (size_t)K->H * K->W, SP = (size_t)(K->H + 1) * (K->W + 1);
  if (hipMalloc((void**)&S->terms, 3 * HW * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&S->sat, 3 * SP * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&S->bg, HW * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipFree(S->terms);
    (void)hipFree(S->sat);
    (void)hipFree(S->bg);
    delete S;
    return fail(B3D_ENOMEM, "scene_create: device allocation failed");
  }
  S->dev.sat = S->sat;
  S->dev.bg = nullptr;
  *out = S;
  return B3D_OK;
}

b3d_status b3d_scene_destroy(b3d_scene* S) {
  if (!S) return B3D_OK;
  (void)hipDeviceSynchronize();
  (void)hipFree(S->terms);
  (void)hipFree(S->sat);
  (void)hipFree(S->bg);
  (void)hipFree(S->grid_sat);
  delete S;
  return B3D_OK;
}

b3d_status b3d_scene_set_background(b3d_scene* S, const b3d_mesh* const* meshes, const float* poses, int32_t n,
                                    void* stream) {
  if (!S) return fail(B3D_EINVAL, "scene_set_background: NULL scene");
  if (n < 0) return fail(B3D_ESHAPE, "scene_set_background: n < 0");
  S->observed = false;
  if (n == 0) {
    S->has_bg = false;
    S->dev.bg = nullptr;
    return B3D_OK;
  }
  if (!meshes || !poses) return fail(B3D_EINVAL, "scene_set_background: NULL pointer");
  if (!finite_all(poses, (size_t)n * 16)) return fail(B3D_EINVAL, "scene_set_background: non-finite pose");
  for (int i = 0; i < n; ++i)
    if (!meshes[i]) return fail(B3D_EINVAL, "scene_set_background: NULL mesh %d", i);
  hipStream_t st = (hipStream_t)stream;
  const size_t HW = (size_t)S->K.H * S->K.W;
  B3D_CHECK_HIP(launch_fill_keys(S->bg, HW, st), "scene_set_background");
  uint64_t base = (uint64_t)S->mesh->T;
  for (int i = 0; i < n; ++i) {
    if (base + (uint64_t)meshes[i]->T >= 0xffffffffull)
      return fail(B3D_ESHAPE, "scene_set_background: too many triangles for 32-bit ids");
    B3D_CHECK_HIP(launch_raster_global(meshes[i]->dev, S->dev.cam, poses + 16 * (size_t)i, (uint32_t)base, S->bg, st),
                  "scene_set_background");
    base += (uint64_t)meshes[i]->T;
  }
  base = (uint64_t)S->mesh->T;
  for (int i = 0; i < n; ++i) {
    B3D_CHECK_HIP(launch_refine_global(meshes[i]->dev, S->dev.cam, poses + 16 * (size_t)i, nullptr, (uint32_t)base,
                                       S->bg, st),
                  "scene_set_background");
    base += (uint64_t)meshes[i]->T;
  }
  S->has_bg = true;
  S->dev.bg = S->bg;
  return B3D_OK;
}

b3d_status b3d_scene_set_observed(b3d_scene* S, const float* observed, void* stream) {
  if (!S || !observed) return fail(B3D_EINVAL, "scene_set_observed: NULL pointer");
  S->dev.obs = observed;
  B3D_CHECK_HIP(launch_background_terms(S->dev, S->terms, (hipStream_t)stream), "scene_set_observed");
  if (b3d_status s = grid_background(S, (hipStream_t)stream)) return s;
  S->observed = true;
  return B3D_OK;
}

b3d_status b3d_scene_set_params(b3d_scene* S, const b3d_score_params* p, void* stream) {
  if (!S || !p) return fail(B3D_EINVAL, "scene_set_params: NULL pointer");
  ScoreConsts sc;
  if (b3d_status s = make_consts(p, S->K.H, S->K.W, &sc)) return s;
  if (sc.h != S->dev.sc.h) return fail(B3D_ESHAPE, "scene_set_params: the window size cannot change");
  S->params = *p;
  S->dev.sc = sc;
  if (S->observed)
    B3D_CHECK_HIP(launch_background_terms(S->dev, S->terms, (hipStream_t)stream), "scene_set_params");
  return B3D_OK;
}

b3d_status b3d_pose_retract(const float* base, int32_t n_base, const float* xi, int32_t N, float* out, void* stream) {
  if (N < 0) return fail(B3D_ESHAPE, "pose_retract: N < 0");
  if (N == 0) return B3D_OK;
  if (!base || !xi || !out) return fail(B3D_EINVAL, "pose_retract: NULL pointer");
  if (n_base != 1 && n_base != N) return fail(B3D_ESHAPE, "pose_retract: n_base must be 1 or N");
  if (out == base) return fail(B3D_EINVAL, "pose_retract: out aliases base");
  B3D_CHECK_HIP(launch_pose_retract(base, n_base, xi, N, out, (hipStream_t)stream), "pose_retract");
  return B3D_OK;
}

b3d_status b3d_pose_retract_backward(const float* xi, const float* grad, const float* dlogL, int32_t N, float* dxi,
                                     float* dsp, void* stream) {
  if (N < 0) return fail(B3D_ESHAPE, "pose_retract_backward: N < 0");
  if (N == 0) return B3D_OK;
  if (!xi || !grad || !dxi) return fail(B3D_EINVAL, "pose_retract_backward: NULL pointer");
  B3D_CHECK_HIP(launch_pose_retract_backward(xi, grad, dlogL, N, dxi, dsp, (hipStream_t)stream),
                "pose_retract_backward");
  return B3D_OK;
}

b3d_status b3d_refine_poses(const b3d_scene* S, float* poses, int32_t N, int32_t n_refine, float lr_t, float lr_r,
                            float beta1, float beta2, float eps, void* stream) {
  if (!S) return fail(B3D_EINVAL, "refine_poses: NULL scene");
  if (!S->observed) return fail(B3D_EINVAL, "refine_poses: call b3d_scene_set_observed first");
  if (N < 0 || n_refine < 0 || n_refine > 100000) return fail(B3D_ESHAPE, "refine_poses: N >= 0, n_refine in 0..1e5");
  if (N == 0 || n_refine == 0) return B3D_OK;
  if (!poses) return fail(B3D_EINVAL, "refine_poses: NULL pointer");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(B3D_EINVAL, "refine_poses: bad Adam parameters");
  B3D_CHECK_HIP(launch_refine_pose(S->dev, poses, N, n_refine, lr_t, lr_r, beta1, beta2, eps, (hipStream_t)stream),
                "refine_poses");
  return B3D_OK;
}

b3d_status b3d_noise_midpoints(double sigma_max, int32_t A, int32_t B, float* sigma_out, float* p_out_out) {
  if (!sigma_out || !p_out_out) return fail(B3D_EINVAL, "noise_midpoints: NULL output");
  if (A < 1 || B < 1) return fail(B3D_ESHAPE, "noise_midpoints: need A, B >= 1");
  if (!(sigma_max > 0) || !std::isfinite(sigma_max)) return fail(B3D_EINVAL, "noise_midpoints: sigma_max must be > 0");
  for (int a = 0; a < A; ++a) sigma_out[a] = (float)(sigma_max * (a + 0.5) / A);
  for (int b = 0; b < B; ++b) p_out_out[b] = (float)((b + 0.5) / B);
  return B3D_OK;
}

b3d_status b3d_scene_set_noise_grid(b3d_scene* S, const float* sigma, int32_t A, const float* p_out, int32_t B,
                                    const float* log_w, void* stream) {
  if (!S || !sigma || !p_out) return fail(B3D_EINVAL, "scene_set_noise_grid: NULL pointer");
  NoiseGridDev g{};
  std::vector<b3d_score_params> ps;
  if (b3d_status s = make_noise_grid(S->params, S->K.H, S->K.W, sigma, A, p_out, B, log_w, &g, &ps)) return s;
  const size_t SP = (size_t)(S->K.H + 1) * (S->K.W + 1);
  double* sat = nullptr;
  if (hipMalloc((void**)&sat, sizeof(double) * 3 * SP * ps.size()) != hipSuccess)
    return fail(B3D_ENOMEM, "scene_set_noise_grid: device allocation failed");
  if (S->grid_sat) {
    (void)hipDeviceSynchronize();  // launches in flight may still read the old tables
    (void)hipFree(S->grid_sat);    // freed after the new allocation, so a failure keeps the old grid
  }
  S->grid_sat = sat;
  g.sat = sat;
  g.sat_stride = (long long)(3 * SP);
  S->grid = g;
  S->grid_params = ps;
  if (S->observed)
    if (b3d_status s = grid_background(S, (hipStream_t)stream)) return s;
  return B3D_OK;
}

b3d_status b3d_render_score_marginal(const b3d_scene* S, const float* poses, int32_t N, float* logL_grid,
                                     float* logL_marg, void* stream) {
  if (!S) return fail(B3D_EINVAL, "render_score_marginal: NULL scene");
  if (S->grid_params.empty()) return fail(B3D_EINVAL, "render_score_marginal: call b3d_scene_set_noise_grid first");
  if (!S->observed) return fail(B3D_EINVAL, "render_score_marginal: call b3d_scene_set_observed first");
  if (N < 0) return fail(B3D_ESHAPE, "render_score_marginal: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !logL_marg) return fail(B3D_EINVAL, "render_score_marginal: NULL pointer");
  B3D_CHECK_HIP(launch_render_score_grid(S->dev, S->grid, poses, N, logL_grid, logL_marg, (hipStream_t)stream),
                "render_score_marginal");
  return B3D_OK;
}

b3d_status b3d_render_score(const b3d_scene* S, const float* poses, int32_t N, float* logL_out, float* grad_out,
                            void* stream) {
  if (!S) return fail(B3D_EINVAL, "render_score: NULL scene");
  if (!S->observed) return fail(B3D_EINVAL, "render_score: call b3d_scene_set_observed first");
  if (N < 0) return fail(B3D_ESHAPE, "render_score: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !logL_out) return fail(B3D_EINVAL, "render_score: NULL pointer");
  B3D_CHECK_HIP(launch_render_score(S->dev, poses, N, logL_out, grad_out, (hipStream_t)stream), "render_score");
  return B3D_OK;
}

}  // extern "C"

namespace b3d_api {

b3d_status plan_batch(const std::vector<BatchItemDev>& items_in, bool grad, BatchPlan* plan, bool cap_tiles) {
  // One launch shares one LDS size, the largest of its scenes', which sets
  // how many blocks fit a CU for all of them: with cap_tiles each scene's
  // depth-buffer tile is capped at the default one (four blocks per CU), or
  // at the smallest the scene allows when that is larger.  No result depends
  // on the tile.
  std::vector<BatchItemDev> items = items_in;
  if (cap_tiles)
    for (BatchItemDev& it : items) it.s.zcap = std::max(min_zcap(it.s), std::min(it.s.zcap, default_zcap(it.s, 4)));
  const int S = (int)items.size();
  std::vector<int> order((size_t)S);
  std::vector<double> cost((size_t)S);
  size_t lds = 0;
  for (int i = 0; i < S; ++i) {
    order[i] = i;
    const SceneDev& d = items[i].s;
    cost[i] = (double)d.mesh.T + 0.25 * (double)d.cam.H * d.cam.W;
    lds = std::max(lds, fused_lds_bytes(d));
  }
  if (lds > kLdsMax) return fail(B3D_ESHAPE, "batch: LDS budget exceeded");
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  plan->grad = grad;
  plan->lds = lds;
  plan->groups.clear();
  for (int k0 = 0; k0 < S; k0 += kBatchGroup) {
    BatchGroupDev g{};
    g.S = std::min(kBatchGroup, S - k0);
    long long first = 0;
    for (int j = 0; j < g.S; ++j) {
      const BatchItemDev& it = items[order[k0 + j]];
      g.s[j] = it.s;
      g.poses[j] = it.poses;
      g.logL[j] = it.logL;
      g.grad[j] = it.grad;
      g.first[j] = first;
      first += it.N;
    }
    g.first[g.S] = first;
    if (first == 0) continue;
    if (first > 0x7fffffffLL) return fail(B3D_ESHAPE, "batch: more than 2^31 - 1 hypotheses in one launch");
    plan->groups.push_back(g);
  }
  return B3D_OK;
}

b3d_status run_batch(const BatchPlan& plan, hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
  const bool two = side && plan.groups.size() > 1;
  if (two) {
    B3D_CHECK_HIP(hipEventRecord(fork, st), "batch");
    B3D_CHECK_HIP(hipStreamWaitEvent(side, fork, 0), "batch");
  }
  for (size_t k = 0; k < plan.groups.size(); ++k)
    B3D_CHECK_HIP(launch_batch(plan.groups[k], plan.grad, plan.lds, two && k % 2 ? side : st), "batch");
  if (two) {
    B3D_CHECK_HIP(hipEventRecord(join, side), "batch");
    B3D_CHECK_HIP(hipStreamWaitEvent(st, join, 0), "batch");
  }
  return B3D_OK;
}

b3d_status run_batch_queue(const BatchPlan& plan, unsigned long long* counters, hipStream_t st) {
  if (plan.groups.empty()) return B3D_OK;
  int dev = 0, cus = 0, occ = 0;
  B3D_CHECK_HIP(hipGetDevice(&dev), "batch");
  B3D_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "batch");
  B3D_CHECK_HIP(batch_queue_occupancy(plan.grad, plan.lds, &occ), "batch");
  for (size_t k = 0; k < plan.groups.size(); ++k) {
    const BatchGroupDev& g = plan.groups[k];
    const int blocks = (int)std::max<long long>(1, std::min<long long>((long long)cus * std::max(occ, 1), g.first[g.S]));
    B3D_CHECK_HIP(launch_batch_queue(g, counters + 32 * k, plan.grad, plan.lds, blocks, st), "batch");
  }
  return B3D_OK;
}

}  // namespace b3d_api

extern "C" {

b3d_status b3d_batch_create(const b3d_batch_item* items, int32_t S, b3d_batch** out) {
  if (!items || !out) return fail(B3D_EINVAL, "batch_create: NULL pointer");
  if (S < 1) return fail(B3D_ESHAPE, "batch_create: need at least one item");
  const bool grad = items[0].grad_out != nullptr;
  std::vector<BatchItemDev> its((size_t)S);
  for (int i = 0; i < S; ++i) {
    const b3d_batch_item& it = items[i];
    if (!it.scene) return fail(B3D_EINVAL, "batch_create: item %d has no scene", i);
    if (!it.scene->observed) return fail(B3D_EINVAL, "batch_create: item %d: scene has no observed image", i);
    if (it.N < 0) return fail(B3D_ESHAPE, "batch_create: item %d: N < 0", i);
    if (it.N > 0 && (!it.poses || !it.logL_out)) return fail(B3D_EINVAL, "batch_create: item %d: NULL buffer", i);
    if ((it.grad_out != nullptr) != grad)
      return fail(B3D_ENOTSUP, "batch_create: grad_out must be given for all items or for none");
    its[i] = BatchItemDev{it.scene->dev, it.poses, it.N, it.logL_out, it.grad_out};
  }
  b3d_batch* b = new b3d_batch();
  if (b3d_status s = plan_batch(its, grad, &b->plan, true)) {
    delete b;
    return s;
  }
  if (b->plan.groups.size() > 1 &&
      (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)) {
    b3d_batch_destroy(b);
    return fail(B3D_EHIP, "batch_create: stream or event creation failed");
  }
  *out = b;
  return B3D_OK;
}

b3d_status b3d_batch_run(const b3d_batch* b, void* stream) {
  if (!b) return fail(B3D_EINVAL, "batch_run: NULL batch");
  return run_batch(b->plan, (hipStream_t)stream, b->side, b->fork, b->join);
}

b3d_status b3d_batch_destroy(b3d_batch* b) {
  if (!b) return B3D_OK;
  (void)hipDeviceSynchronize();
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->side) (void)hipStreamDestroy(b->side);
  delete b;
  return B3D_OK;
}

b3d_status b3d_scene_tile_limits(const b3d_scene* S, int32_t* min_keys, int32_t* max_keys, int32_t* current) {
  if (!S) return fail(B3D_EINVAL, "scene_tile_limits: NULL scene");
  if (min_keys) *min_keys = min_zcap(S->dev);
  if (max_keys) *max_keys = max_zcap(S->dev);
  if (current) *current = S->dev.zcap;
  return B3D_OK;
}

b3d_status b3d_scene_set_tile(b3d_scene* S, int32_t zcap) {
  if (!S) return fail(B3D_EINVAL, "scene_set_tile: NULL scene");
  SceneDev t = S->dev;
  t.zcap = zcap <= 0 ? std::max(default_zcap(S->dev, 4), min_zcap(S->dev)) : zcap;
  if (t.zcap < min_zcap(S->dev) || t.zcap > max_zcap(S->dev) || fused_lds_bytes(t) > kLdsMax)
    return fail(B3D_ESHAPE, "scene_set_tile: %d keys outside [%d, LDS limit]", zcap, min_zcap(S->dev));
  S->dev.zcap = t.zcap;
  return B3D_OK;
}

b3d_status b3d_scene_autotune(b3d_scene* S, const float* poses, int32_t N, int32_t grad, int32_t* zcap_out,
                              void* stream) {
  if (!S || !poses) return fail(B3D_EINVAL, "scene_autotune: NULL pointer");
  if (!S->observed) return fail(B3D_EINVAL, "scene_autotune: call b3d_scene_set_observed first");
  if (N < 1) return fail(B3D_ESHAPE, "scene_autotune: need N >= 1");
  hipStream_t st = (hipStream_t)stream;
  float* out = nullptr;
  if (hipMalloc((void**)&out, sizeof(float) * 9 * (size_t)N) != hipSuccess)
    return fail(B3D_ENOMEM, "scene_autotune: scratch allocation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int keep = S->dev.zcap;
  int best = keep;
  float best_ms = 3.0e38f;
  std::vector<int> cands;
  for (int b = 2; b <= 6; ++b) {
    const int z = std::min(default_zcap(S->dev, b), max_zcap(S->dev));
    if (cands.empty() || cands.back() != z) cands.push_back(z);
  }
  if (cands.back() != min_zcap(S->dev)) cands.push_back(min_zcap(S->dev));
  b3d_status status = B3D_OK;
  for (int z : cands) {
    SceneDev t = S->dev;
    t.zcap = z;
    if (z < min_zcap(S->dev) || fused_lds_bytes(t) > kLdsMax) continue;
    float ms = 0.0f;
    for (int rep = 0; rep < 3 && status == B3D_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess ||
          launch_render_score(t, poses, N, out, grad ? out + N : nullptr, st) != hipSuccess ||
          hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        status = fail(B3D_EHIP, "scene_autotune: timing launch failed");
    }
    if (status != B3D_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = z;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (status != B3D_OK) return status;
  S->dev.zcap = best;
  if (zcap_out) *zcap_out = best;
  return B3D_OK;
}

b3d_status b3d_render_score_work(const b3d_scene* S, const float* poses, int32_t N, float* logL_out, float* grad_out,
                                 unsigned long long* work, void* stream) {
  if (!S) return fail(B3D_EINVAL, "render_score_work: NULL scene");
  if (!S->observed) return fail(B3D_EINVAL, "render_score_work: call b3d_scene_set_observed first");
  if (N < 0) return fail(B3D_ESHAPE, "render_score_work: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !logL_out || !grad_out || !work) return fail(B3D_EINVAL, "render_score_work: NULL pointer");
  B3D_CHECK_HIP(launch_render_score_count(S->dev, poses, N, logL_out, grad_out, work, (hipStream_t)stream),
                "render_score_work");
  return B3D_OK;
}

static b3d_status make_grid(const b3d_grid* g, GridDev* d, int64_t* N) {
  if (!g) return fail(B3D_EINVAL, "grid pointer is NULL");
  for (int k = 0; k < 3; ++k) {
    if (g->count[k] < 1) return fail(B3D_EINVAL, "grid: count[%d] must be >= 1", k);
    if (!(g->half_extent[k] >= 0) || !std::isfinite(g->half_extent[k]))
      return fail(B3D_EINVAL, "grid: half_extent[%d] must be >= 0", k);
  }
  if (g->n_rot < 1) return fail(B3D_EINVAL, "grid: n_rot must be >= 1");
  if (!std::isfinite(g->rot_max_angle) || g->rot_max_angle < 0) return fail(B3D_EINVAL, "grid: bad rot_max_angle");
  if (!finite_all(g->center, 16)) return fail(B3D_EINVAL, "grid: non-finite centre pose");
  const int64_t n = (int64_t)g->count[0] * g->count[1] * g->count[2] * g->n_rot;
  if (n > (1ll << 28)) return fail(B3D_ESHAPE, "grid: too many hypotheses");
  std::memcpy(d->center, g->center, sizeof(d->center));
  for (int k = 0; k < 3; ++k) {
    d->half[k] = g->half_extent[k];
    d->count[k] = g->count[k];
  }
  d->cell_centres = g->cell_centres ? 1 : 0;
  d->n_rot = g->n_rot;
  d->max_angle = g->rot_max_angle;
  d->rots = g->rotations;
  *N = n;
  return B3D_OK;
}

int64_t b3d_grid_size(const b3d_grid* g) {
  GridDev d;
  int64_t n = 0;
  std::string keep = g_err;
  if (make_grid(g, &d, &n) != B3D_OK) {
    g_err = keep;
    return 0;
  }
  return n;
}

b3d_status b3d_enumerate(const b3d_grid* g, uint64_t seed, int32_t stage, float* poses_out, void* stream) {
  GridDev d;
  int64_t N;
  if (b3d_status s = make_grid(g, &d, &N)) return s;
  if (!poses_out) return fail(B3D_EINVAL, "enumerate: NULL output");
  if (stage < 0) return fail(B3D_EINVAL, "enumerate: stage < 0");
  B3D_CHECK_HIP(launch_enumerate(d, nullptr, 1, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)stage, poses_out,
                                 (hipStream_t)stream),
                "enumerate");
  return B3D_OK;
}

b3d_status b3d_sample(const float* logL, int32_t P, int32_t N, int32_t K, uint64_t seed, uint32_t stage, uint32_t k0,
                      float* weights_out, int32_t* idx_out, float* logw_out, void* stream) {
  if (P < 0 || N < 0) return fail(B3D_ESHAPE, "sample: P, N must be >= 0");
  if (K < 1 || K > 4096) return fail(B3D_EINVAL, "sample: K must be in 1..4096");
  if (P == 0) return B3D_OK;
  if (N == 0) return fail(B3D_ESHAPE, "sample: cannot draw from an empty segment");
  if ((int64_t)P * K > (1ll << 30)) return fail(B3D_ESHAPE, "sample: too many draws");
  if (!logL || !idx_out) return fail(B3D_EINVAL, "sample: NULL pointer");
  B3D_CHECK_HIP(launch_sample(logL, P, N, K, (uint32_t)seed, (uint32_t)(seed >> 32), stage, k0, weights_out, idx_out,
                              logw_out, (hipStream_t)stream),
                "sample");
  return B3D_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct C2FLayout {
  size_t poses, logL, idx, logw, total;
  int64_t max_hyp;
};

static b3d_status c2f_layout(const b3d_schedule* s, int32_t K, C2FLayout* L) {
  if (!s) return fail(B3D_EINVAL, "schedule pointer is NULL");
  if (s->n_stages < 1 || s->n_stages > B3D_MAX_STAGES)
    return fail(B3D_EINVAL, "schedule: n_stages must be in 1..%d", B3D_MAX_STAGES);
  if (K < 1 || K > 4096) return fail(B3D_EINVAL, "c2f: K must be in 1..4096");
  int64_t mx = 0;
  for (int t = 0; t < s->n_stages; ++t) {
    GridDev d;
    int64_t n;
    if (b3d_status st = make_grid(&s->stages[t], &d, &n)) return st;
    mx = std::max(mx, t == 0 ? n : n * K);
  }
  if (mx > (1ll << 31) - 1) return fail(B3D_ESHAPE, "c2f: too many hypotheses in one stage");
  L->max_hyp = mx;
  size_t off = 0;
  L->poses = off;
  off = align256(off + sizeof(float) * 16 * (size_t)mx);
  L->logL = off;
  off = align256(off + sizeof(float) * (size_t)mx);
  L->idx = off;
  off = align256(off + sizeof(int) * (size_t)K);
  L->logw = off;
  off = align256(off + sizeof(float) * (size_t)K);
  L->total = off;
  return B3D_OK;
}

b3d_status b3d_c2f_workspace_size(const b3d_schedule* s, int32_t K, size_t* bytes) {
  if (!bytes) return fail(B3D_EINVAL, "c2f_workspace_size: NULL output");
  C2FLayout L;
  if (b3d_status st = c2f_layout(s, K, &L)) return st;
  *bytes = L.total;
  return B3D_OK;
}

b3d_status b3d_c2f_weights_count(const b3d_schedule* s, int32_t K, int64_t* count) {
  if (!count) return fail(B3D_EINVAL, "c2f_weights_count: NULL output");
  C2FLayout L;
  if (b3d_status st = c2f_layout(s, K, &L)) return st;
  int64_t total = 0;
  for (int t = 0; t < s->n_stages; ++t) {
    GridDev d;
    int64_t n;
    (void)make_grid(&s->stages[t], &d, &n);
    total += t == 0 ? n : n * K;
  }
  *count = total;
  return B3D_OK;
}

b3d_status b3d_c2f_step(const b3d_scene* S, const float* center, const b3d_schedule* s, int32_t K, uint64_t seed,
                        void* workspace, size_t ws_bytes, float* weights_out, float* poses_out, float* logq_out,
                        int32_t* idx_out, void* stream) {
  if (!S || !center || !poses_out || !logq_out || !workspace) return fail(B3D_EINVAL, "c2f_step: NULL pointer");
  if (!S->observed) return fail(B3D_EINVAL, "c2f_step: call b3d_scene_set_observed first");
  if (!finite_all(center, 16)) return fail(B3D_EINVAL, "c2f_step: non-finite centre pose");
  C2FLayout L;
  if (b3d_status st = c2f_layout(s, K, &L)) return st;
  if (ws_bytes < L.total) return fail(B3D_ESHAPE, "c2f_step: workspace of %zu bytes < %zu", ws_bytes, L.total);
  char* ws = (char*)workspace;
  float* poses = (float*)(ws + L.poses);
  float* logL = (float*)(ws + L.logL);
  int* idx = (int*)(ws + L.idx);
  float* logw = (float*)(ws + L.logw);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  size_t woff = 0;  // stage t's weights: segment p of stage t at woff + p n
  for (int t = 0; t < s->n_stages; ++t) {
    GridDev d;
    int64_t n;
    (void)make_grid(&s->stages[t], &d, &n);
    const int P = (t == 0) ? 1 : K;
    if (t == 0) std::memcpy(d.center, center, sizeof(d.center));
    B3D_CHECK_HIP(launch_enumerate(d, t == 0 ? nullptr : poses_out, P, k0, k1, (uint32_t)t, poses, st), "c2f_step");
    B3D_CHECK_HIP(launch_render_score(S->dev, poses, (int)(n * P), logL, nullptr, st), "c2f_step");
    B3D_CHECK_HIP(launch_sample(logL, P, (int)n, t == 0 ? K : 1, k0, k1, (uint32_t)t, 0u,
                                weights_out ? weights_out + woff : nullptr, idx, logw, st),
                  "c2f_step");
    woff += (size_t)n * P;
    B3D_CHECK_HIP(launch_c2f_update(poses, P, (int)n, idx, logw, K, t > 0, poses_out, logq_out,
                                    idx_out ? idx_out + (size_t)t * K : nullptr, st),
                  "c2f_step");
  }
  return B3D_OK;
}

b3d_status b3d_adam_pose_step(float* poses, const float* grad, int32_t gstride, float* state, int32_t N, int32_t iter,
                              float lr_t, float lr_r, float beta1, float beta2, float eps, void* stream) {
  if (N < 0) return fail(B3D_ESHAPE, "adam_pose_step: N < 0");
  if (N == 0) return B3D_OK;
  if (!poses || !grad || !state) return fail(B3D_EINVAL, "adam_pose_step: NULL pointer");
  if (gstride < 6) return fail(B3D_EINVAL, "adam_pose_step: gstride must be >= 6");
  if (iter < 1) return fail(B3D_EINVAL, "adam_pose_step: iter must be >= 1");
  if (!(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || !std::isfinite(lr_t) ||
      !std::isfinite(lr_r))
    return fail(B3D_EINVAL, "adam_pose_step: need 0 <= beta < 1, eps > 0, finite rates");
  B3D_CHECK_HIP(launch_adam_pose(poses, grad, gstride, state, N, iter, lr_t, lr_r, beta1, beta2, eps,
                                 (hipStream_t)stream),
                "adam_pose_step");
  return B3D_OK;
}

}  // extern "C"

// ---- tracker -------------------------------------------------------------

// Image rows per block of the tracker's refinement steps.
constexpr int kRefineRows = 8;

struct b3d_tracker {
  int M = 0;
  int64_t N = 0;
  b3d_track_params tp{};
  std::vector<const b3d_mesh*> meshes;
  std::vector<b3d_scene*> scenes;
  float* obs = nullptr;      // [H][W][3] frame buffer read by the graph
  // per-object state, one allocation: poses [M][16] (current estimates),
  // prev [M][16] (estimates before the frame's update), motion [M][12] (last
  // accepted frame-to-frame rotation and translation), gate [M][4]
  // (visibility, dropped updates in a row, stage 0's translation scale, 0)
  float* poses = nullptr;
  float* prev = nullptr;
  float* motion = nullptr;
  float* gate = nullptr;
  unsigned long long* objkeys = nullptr;  // [H][W] the updated object drawn alone
  float* hyp = nullptr;      // [N][16]
  float* logL = nullptr;     // [N]
  float* partial = nullptr;  // [ceil(H / kRefineRows)][9] band sums of a refinement step
  float* adam = nullptr;     // [M][12] Adam moments of the refinement
  size_t obs_bytes = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Object o's scene for the frame in T->obs: the other objects at their
// current estimates drawn as its static background, then the background's
// likelihood terms.
static b3d_status tracker_background(b3d_tracker* T, int o, hipStream_t st) {
  b3d_scene* S = T->scenes[o];
  const size_t HW = (size_t)S->K.H * S->K.W;
  if (T->M > 1) {
    B3D_CHECK_HIP(launch_fill_keys(S->bg, HW, st), "tracker");
    uint32_t base = (uint32_t)S->mesh->T;
    for (int k = 0; k < T->M; ++k) {
      if (k == o) continue;
      B3D_CHECK_HIP(launch_raster_global_dev(T->meshes[k]->dev, S->dev.cam, T->poses + 16 * k, base, S->bg, st),
                    "tracker");
      B3D_CHECK_HIP(launch_refine_global(T->meshes[k]->dev, S->dev.cam, nullptr, T->poses + 16 * k, base, S->bg, st),
                    "tracker");
      base += (uint32_t)T->meshes[k]->T;
    }
  }
  B3D_CHECK_HIP(launch_background_terms(S->dev, S->terms, st), "tracker");
  return B3D_OK;
}

// Floats of per-object state in the tracker's state allocation.
constexpr int kTrackStateFloats = 16 + 16 + 12 + 4;

static b3d_status tracker_record(b3d_tracker* T, hipStream_t st) {
  const b3d_track_params& tp = T->tp;
  const bool gating = tp.min_visible > 0.0f;
  GridDev g[B3D_MAX_STAGES];
  int64_t ns[B3D_MAX_STAGES];
  for (int s = 0; s < tp.n_stages; ++s) (void)make_grid(&tp.stages[s], &g[s], &ns[s]);
  for (int o = 0; o < T->M; ++o) {
    b3d_scene* S = T->scenes[o];
    if (b3d_status s = tracker_background(T, o, st)) return s;
    if (gating) B3D_CHECK_HIP(launch_copy_f32(T->poses + 16 * o, 16, T->prev + 16 * o, st), "tracker");
    for (int s = 0; s < tp.n_stages; ++s) {
      // stage 0's translations scaled after a dropped update
      const float* hscale = gating && s == 0 ? T->gate + 4 * o + 2 : nullptr;
      B3D_CHECK_HIP(launch_enumerate(g[s], T->poses + 16 * o, 1, 0u, 0u, (uint32_t)s, T->hyp, st, hscale), "tracker");
      B3D_CHECK_HIP(launch_render_score(S->dev, T->hyp, (int)ns[s], T->logL, nullptr, st), "tracker");
      B3D_CHECK_HIP(launch_argmax_pose(T->logL, T->hyp, (int)ns[s], T->poses + 16 * o, st), "tracker");
    }
    if (tp.n_refine > 0)
      B3D_CHECK_HIP(launch_refine_banded(S->dev, T->poses + 16 * o, tp.n_refine, tp.lr_t, tp.lr_r, tp.beta1, tp.beta2,
                                         tp.eps, kRefineRows, T->partial, T->adam + 12 * o, st),
                    "tracker");
    if (gating) {
      // the object alone at its new pose, then how much of it is in front of
      // the others and confirmed by the observation, and the decision
      const SceneDev& d = S->dev;
      const size_t HW = (size_t)d.cam.H * d.cam.W;
      B3D_CHECK_HIP(launch_fill_keys(T->objkeys, HW, st), "tracker");
      B3D_CHECK_HIP(launch_raster_global_dev(d.mesh, d.cam, T->poses + 16 * o, 0u, T->objkeys, st), "tracker");
      B3D_CHECK_HIP(launch_refine_global(d.mesh, d.cam, nullptr, T->poses + 16 * o, 0u, T->objkeys, st), "tracker");
      B3D_CHECK_HIP(launch_track_gate(T->objkeys, T->M > 1 ? S->bg : nullptr, T->obs, d.cam, d.sc.h,
                                      3.0f * S->params.sigma, tp.min_visible, tp.widen, T->prev + 16 * o,
                                      T->poses + 16 * o, T->motion + 12 * o, T->gate + 4 * o, st),
                    "tracker");
    }
  }
  return B3D_OK;
}

// Chooses the fused kernel's depth-buffer tile (the same for every object's
// scene) by timing whole frames on the frame in T->obs, restoring the
// estimates after each; no result depends on the tile.  Synchronises `st`.
static b3d_status tracker_tune(b3d_tracker* T, hipStream_t st) {
  const SceneDev& d0 = T->scenes[0]->dev;
  std::vector<int> cands;
  for (int b = 2; b <= 6; ++b) {
    const int z = std::min(default_zcap(d0, b), max_zcap(d0));
    SceneDev t = d0;
    t.zcap = z;
    if (z >= min_zcap(d0) && fused_lds_bytes(t) <= kLdsMax && (cands.empty() || cands.back() != z))
      cands.push_back(z);
  }
  if (cands.size() < 2) return B3D_OK;
  const size_t pose_bytes = sizeof(float) * kTrackStateFloats * (size_t)T->M;  // estimates and occlusion state
  float* saved = nullptr;
  if (hipMalloc((void**)&saved, pose_bytes) != hipSuccess)
    return fail(B3D_ENOMEM, "tracker_frame: tuning scratch allocation failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  b3d_status status = B3D_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemcpyAsync(saved, T->poses, pose_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
    status = fail(B3D_EHIP, "tracker_frame: tuning set-up failed");
  const int keep = d0.zcap;
  int best = keep;
  float best_ms = 3.0e38f;
  for (size_t c = 0; c < cands.size() && status == B3D_OK; ++c) {
    for (b3d_scene* S : T->scenes) S->dev.zcap = cands[c];
    float ms = 3.0e38f;
    for (int rep = 0; rep < 3 && status == B3D_OK; ++rep) {  // the first run warms up
      float t = 0.0f;
      if (hipEventRecord(e0, st) != hipSuccess) status = fail(B3D_EHIP, "tracker_frame: tuning event failed");
      if (status == B3D_OK) status = tracker_record(T, st);
      if (status == B3D_OK &&
          (hipEventRecord(e1, st) != hipSuccess ||
           hipMemcpyAsync(T->poses, saved, pose_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
           hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        status = fail(B3D_EHIP, "tracker_frame: tuning run failed");
      if (rep > 0) ms = std::min(ms, t);
    }
    if (status == B3D_OK && ms < best_ms) {
      best_ms = ms;
      best = cands[c];
    }
  }
  for (b3d_scene* S : T->scenes) S->dev.zcap = status == B3D_OK ? best : keep;
  if (hipStreamSynchronize(st) != hipSuccess && status == B3D_OK) status = fail(B3D_EHIP, "tracker_frame: tuning");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(saved);
  return status;
}

extern "C" {

b3d_status b3d_tracker_create(const b3d_mesh* const* meshes, int32_t M, const b3d_intrinsics* K,
                              const b3d_score_params* p, const b3d_track_params* tp, const float* init_poses,
                              b3d_tracker** out) {
  if (!meshes || !tp || !init_poses || !out) return fail(B3D_EINVAL, "tracker_create: NULL pointer");
  if (M < 1 || M > 16) return fail(B3D_ESHAPE, "tracker_create: M must be in 1..16");
  if (b3d_status s = check_intrinsics(K)) return s;
  ScoreConsts sc;
  if (b3d_status s = make_consts(p, K->H, K->W, &sc)) return s;
  if (tp->n_stages < 1 || tp->n_stages > B3D_MAX_STAGES)
    return fail(B3D_ESHAPE, "tracker_create: n_stages must be in 1..%d", B3D_MAX_STAGES);
  int64_t n = 0;
  for (int s = 0; s < tp->n_stages; ++s) {
    GridDev g;
    int64_t ns;
    if (b3d_status st = make_grid(&tp->stages[s], &g, &ns)) return st;
    if (ns > (1 << 24)) return fail(B3D_ESHAPE, "tracker_create: grid of stage %d too large", s);
    n = std::max(n, ns);
  }
  if (tp->n_refine < 0 || tp->n_refine > 1000) return fail(B3D_EINVAL, "tracker_create: n_refine in 0..1000");
  if (!(tp->min_visible >= 0.0f && tp->min_visible <= 1.0f))
    return fail(B3D_EINVAL, "tracker_create: min_visible must be in [0, 1]");
  if (tp->min_visible > 0.0f && !(tp->widen >= 1.0f && tp->widen <= 100.0f))
    return fail(B3D_EINVAL, "tracker_create: widen must be in [1, 100]");
  if (!(tp->beta1 >= 0 && tp->beta1 < 1) || !(tp->beta2 >= 0 && tp->beta2 < 1) || !(tp->eps > 0))
    return fail(B3D_EINVAL, "tracker_create: bad Adam parameters");
  if (!finite_all(init_poses, (size_t)M * 16)) return fail(B3D_EINVAL, "tracker_create: non-finite pose");
  for (int i = 0; i < M; ++i)
    if (!meshes[i]) return fail(B3D_EINVAL, "tracker_create: NULL mesh %d", i);
  b3d_tracker* T = new b3d_tracker();
  T->M = M;
  T->N = n;
  T->tp = *tp;
  T->meshes.assign(meshes, meshes + M);
  T->obs_bytes = sizeof(float) * 3 * (size_t)K->H * K->W;
  auto cleanup = [&](b3d_status s, const char* msg) {
    for (b3d_scene* S : T->scenes) b3d_scene_destroy(S);
    (void)hipFree(T->obs);
    (void)hipFree(T->poses);
    (void)hipFree(T->hyp);
    (void)hipFree(T->logL);
    (void)hipFree(T->partial);
    (void)hipFree(T->adam);
    (void)hipFree(T->objkeys);
    if (T->cap) (void)hipStreamDestroy(T->cap);
    delete T;
    return fail(s, "%s", msg);
  };
  if (hipMalloc((void**)&T->obs, T->obs_bytes) != hipSuccess ||
      hipMalloc((void**)&T->poses, sizeof(float) * kTrackStateFloats * M) != hipSuccess ||
      hipMalloc((void**)&T->objkeys, sizeof(unsigned long long) * (size_t)K->H * K->W) != hipSuccess ||
      hipMalloc((void**)&T->hyp, sizeof(float) * 16 * (size_t)n) != hipSuccess ||
      hipMalloc((void**)&T->logL, sizeof(float) * (size_t)n) != hipSuccess ||
      hipMalloc((void**)&T->partial, sizeof(float) * 9 * (size_t)((K->H + kRefineRows - 1) / kRefineRows)) != hipSuccess ||
      hipMalloc((void**)&T->adam, sizeof(float) * 12 * (size_t)M) != hipSuccess)
    return cleanup(B3D_ENOMEM, "tracker_create: device allocation failed");
  T->prev = T->poses + 16 * M;
  T->motion = T->prev + 16 * M;
  T->gate = T->motion + 12 * M;
  std::vector<float> state((size_t)kTrackStateFloats * M, 0.0f);
  for (int o = 0; o < M; ++o) {
    for (int k = 0; k < 16; ++k) state[16 * o + k] = state[16 * (M + o) + k] = init_poses[16 * o + k];
    float* mo = state.data() + 32 * M + 12 * o;  // no motion: identity rotation, zero translation
    mo[0] = mo[4] = mo[8] = 1.0f;
    state[44 * M + 4 * o + 2] = 1.0f;  // stage 0 at its own extents
  }
  if (hipMemcpy(T->poses, state.data(), sizeof(float) * state.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(T->obs, 0, T->obs_bytes) != hipSuccess)
    return cleanup(B3D_EHIP, "tracker_create: initial copy failed");
  for (int o = 0; o < M; ++o) {
    b3d_scene* S = nullptr;
    if (b3d_scene_create(meshes[o], K, p, &S) != B3D_OK) return cleanup(B3D_ENOMEM, g_err.c_str());
    T->scenes.push_back(S);
    S->dev.obs = T->obs;
    S->observed = true;
    if (M > 1) {
      S->has_bg = true;
      S->dev.bg = S->bg;
    }
  }
  if (hipStreamCreateWithFlags(&T->cap, hipStreamNonBlocking) != hipSuccess)
    return cleanup(B3D_EHIP, "tracker_create: stream creation failed");
  *out = T;
  return B3D_OK;
}

b3d_status b3d_tracker_frame(b3d_tracker* T, const float* observed, void* stream) {
  if (!T || !observed) return fail(B3D_EINVAL, "tracker_frame: NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  if (!T->exec) {
    B3D_CHECK_HIP(hipMemcpyAsync(T->obs, observed, T->obs_bytes, hipMemcpyDeviceToDevice, st), "tracker_frame: copy");
    if (b3d_status s = tracker_tune(T, st)) return s;
    B3D_CHECK_HIP(hipStreamBeginCapture(T->cap, hipStreamCaptureModeThreadLocal), "tracker_frame: capture");
    b3d_status s = tracker_record(T, T->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(T->cap, &g);
    if (s != B3D_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "tracker_frame: end capture");
    T->graph = g;
    B3D_CHECK_HIP(hipGraphInstantiate(&T->exec, T->graph, nullptr, nullptr, 0), "tracker_frame: instantiate");
  }
  B3D_CHECK_HIP(hipMemcpyAsync(T->obs, observed, T->obs_bytes, hipMemcpyDeviceToDevice, st), "tracker_frame: copy");
  B3D_CHECK_HIP(hipGraphLaunch(T->exec, st), "tracker_frame: launch");
  return B3D_OK;
}

b3d_status b3d_tracker_frame_eager(b3d_tracker* T, const float* observed, void* stream) {
  if (!T || !observed) return fail(B3D_EINVAL, "tracker_frame_eager: NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  B3D_CHECK_HIP(hipMemcpyAsync(T->obs, observed, T->obs_bytes, hipMemcpyDeviceToDevice, st), "tracker_frame: copy");
  return tracker_record(T, st);
}

b3d_status b3d_tracker_state(const b3d_tracker* T, float* state_out, void* stream) {
  if (!T || !state_out) return fail(B3D_EINVAL, "tracker_state: NULL pointer");
  B3D_CHECK_HIP(hipMemcpy2DAsync(state_out, sizeof(float) * 3, T->gate, sizeof(float) * 4, sizeof(float) * 3, T->M,
                                 hipMemcpyDeviceToDevice, (hipStream_t)stream),
                "tracker_state");
  return B3D_OK;
}

b3d_status b3d_tracker_poses(const b3d_tracker* T, float* poses_out, void* stream) {
  if (!T || !poses_out) return fail(B3D_EINVAL, "tracker_poses: NULL pointer");
  B3D_CHECK_HIP(hipMemcpyAsync(poses_out, T->poses, sizeof(float) * 16 * T->M, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream),
                "tracker_poses");
  return B3D_OK;
}

b3d_status b3d_tracker_destroy(b3d_tracker* T) {
  if (!T) return B3D_OK;
  (void)hipDeviceSynchronize();
  if (T->exec) (void)hipGraphExecDestroy(T->exec);
  if (T->graph) (void)hipGraphDestroy(T->graph);
  for (b3d_scene* S : T->scenes) b3d_scene_destroy(S);
  (void)hipFree(T->obs);
  (void)hipFree(T->poses);
  (void)hipFree(T->hyp);
  (void)hipFree(T->logL);
  (void)hipFree(T->partial);
  (void)hipFree(T->adam);
  (void)hipFree(T->objkeys);
  if (T->cap) (void)hipStreamDestroy(T->cap);
  delete T;
  return B3D_OK;
}

}  // extern "C"

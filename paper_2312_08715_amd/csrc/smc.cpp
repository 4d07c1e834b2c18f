// Host side of the table-contact placement and of the SMC sampler over the
// objects of a table scene (Sec. III-A (i), Sec. III-B, eq. (2)-(3)): set-up
// of the resting frames and placement boxes, and the per-stage sequence of
// launches.  Every per-hypothesis and per-particle step runs in the kernels;
// the host reads back only the particles' noise, chosen types and earlier
// objects to set up each stage's scenes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "api_internal.hpp"

using namespace b3d;
using namespace b3d_api;

namespace {

// Resting frame of face c: a rotation taking the face's outward normal
// (-x, +x, -y, +y, -z, +z for c = 0..5) to -z.
constexpr float kFaceRot[6][9] = {
    {0, 0, -1, 0, 1, 0, 1, 0, 0},  {0, 0, 1, 0, 1, 0, -1, 0, 0}, {1, 0, 0, 0, 0, -1, 0, 1, 0},
    {1, 0, 0, 0, 0, 1, 0, -1, 0},  {1, 0, 0, 0, 1, 0, 0, 0, 1},  {1, 0, 0, 0, -1, 0, 0, 0, -1},
};

// Faces of a mesh's object-frame bounding box, with their log prior
// densities on a table (zero footprint margin gives B3D_ESHAPE).
b3d_status make_faces(const b3d_mesh* m, int n_types, const b3d_table* t, FaceDev* out) {
  for (int c = 0; c < 6; ++c) {
    FaceDev& f = out[c];
    std::memcpy(f.R, kFaceRot[c], sizeof(f.R));
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < 8; ++i) {
      const double p[3] = {(i & 4) ? m->box_hi[0] : m->box_lo[0], (i & 2) ? m->box_hi[1] : m->box_lo[1],
                           (i & 1) ? m->box_hi[2] : m->box_lo[2]};
      for (int r = 0; r < 3; ++r) {
        const double q = f.R[3 * r] * p[0] + f.R[3 * r + 1] * p[1] + f.R[3 * r + 2] * p[2];
        mn[r] = std::min(mn[r], q);
        mx[r] = std::max(mx[r], q);
      }
    }
    f.d[0] = (float)(-0.5 * (mn[0] + mx[0]));
    f.d[1] = (float)(-0.5 * (mn[1] + mx[1]));
    f.d[2] = (float)(-mn[2]);
    f.w = (float)(mx[0] - mn[0]);
    f.h = (float)(mx[1] - mn[1]);
    const double ax = (double)t->width - f.w, ay = (double)t->height - f.h;
    if (!(ax > 0) || !(ay > 0)) return fail(B3D_ESHAPE, "face %d of a type does not fit on the table", c);
    f.lprior = -(std::log((double)n_types) + std::log(6.0) + std::log(ax) + std::log(ay) + std::log(2.0 * M_PI));
  }
  return B3D_OK;
}

b3d_status make_contact(const b3d_mesh* const* types, int n_types, const b3d_table* t, std::vector<FaceDev>* faces) {
  if (!types || !t) return fail(B3D_EINVAL, "NULL pointer");
  if (n_types < 1 || n_types > B3D_MAX_TYPES) return fail(B3D_ESHAPE, "need 1 <= n_types <= %d", B3D_MAX_TYPES);
  if (!finite_all(t->pose, 16) || !(t->width > 0) || !(t->height > 0) || !std::isfinite(t->width) ||
      !std::isfinite(t->height))
    return fail(B3D_EINVAL, "table: non-finite pose or non-positive extent");
  faces->assign((size_t)n_types * 6, FaceDev{});
  for (int o = 0; o < n_types; ++o) {
    if (!types[o]) return fail(B3D_EINVAL, "NULL mesh for type %d", o);
    if (b3d_status s = make_faces(types[o], n_types, t, faces->data() + 6 * o)) return s;
  }
  return B3D_OK;
}

template <class T>
b3d_status dev_alloc(std::vector<void*>& owned, T** p, size_t n) {
  if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
    return fail(B3D_ENOMEM, "smc: device allocation failed");
  owned.push_back((void*)*p);
  return B3D_OK;
}

}  // namespace

struct b3d_contact {
  ContactDev C{};  // table pose and the device copy of every type's six resting faces
};

struct b3d_smc {
  b3d_smc_params p{};
  b3d_table table{};
  b3d_intrinsics K{};
  std::vector<const b3d_mesh*> types, fixed;
  std::vector<float> fixed_poses;
  int n_stage0 = 0;  // hypotheses per particle at stage 0
  int max_split = 0;
  std::vector<b3d_scene*> scenes;  // one per particle
  ContactDev C{};
  CellDev* roots = nullptr;  // [n_types * 6]
  float* stage0_poses = nullptr;
  PartDev st[2]{};
  int cur = 0;
  int placed = 0;
  const float* observed = nullptr;
  NoiseGridDev noise_mid{};
  // stage buffers
  CellDev* cells = nullptr;
  double *clogq = nullptr, *logq = nullptr, *logp_new = nullptr, *lprior_new = nullptr, *logW_pre = nullptr;
  double* ess = nullptr;
  int *choice = nullptr, *idx = nullptr, *nidx = nullptr, *drawn = nullptr, *anc = nullptr;
  float *hyp = nullptr, *logL_h = nullptr, *logw = nullptr, *nlogw = nullptr, *lw_shift = nullptr;
  float *dphi_new = nullptr, *pose_new = nullptr, *noise_new = nullptr, *logL_new = nullptr, *noise_grid = nullptr;
  float* marg = nullptr;
  float* type_post = nullptr;  // [M][n_types]
  float* partial = nullptr;  // [M][n_bands][kMaxNoise] band sums of the whole-image scores
  int rows_R = 0, n_bands = 0;
  long long scored = 0;  // hypotheses rendered and scored since the last reset
  int zcap = 0;          // depth-buffer tile of the particles' scenes, tuned on the first step
  // one work counter per launch of a step's scoring (persistent grids: the
  // sampler's launches are few, long and of long items)
  unsigned long long* counters = nullptr;
  int max_groups = 0;
  std::vector<void*> owned;
};

// Whole-image logL of each particle's scene with its proposed object at
// pose_new: under the noise cells' midpoints (into noise_grid) or, with
// own_noise, under the particle's proposed noise (into logL_new).
static b3d_status whole_image_scores(b3d_smc* S, hipStream_t st, const std::vector<int>& type_of,
                                     const std::vector<int>& rep, bool own_noise) {
  const b3d_smc_params& p = S->p;
  const int M = p.n_particles;
  for (int g0 = 0; g0 < M; g0 += kBatchGroup) {
    RowsGroupDev G{};
    G.S = std::min(kBatchGroup, M - g0);
    G.first = g0;
    G.grid = S->noise_mid;
    G.inv_V = 1.0 / (double)p.outlier_volume;
    G.M_norm = p.norm_M > 0 ? (double)p.norm_M : (double)S->K.H * S->K.W;
    for (int j = 0; j < G.S; ++j) {
      const int m = g0 + j;
      SceneDev d = S->scenes[rep[m]]->dev;
      d.mesh = S->types[type_of[m]]->dev;
      d.zcap = max_zcap(d);
      G.s[j] = d;
      G.pose[j] = S->pose_new + 16 * (size_t)m;
      G.noise[j] = own_noise ? S->noise_new + 2 * (size_t)m : nullptr;
    }
    B3D_CHECK_HIP(launch_score_rows_grid(G, S->rows_R, S->n_bands, S->partial, st), "smc_step");
  }
  NoiseGridDev one{};
  if (own_noise) {
    one.A = one.B = 1;
    one.logw[0] = 0.0f;
  }
  const NoiseGridDev& g = own_noise ? one : S->noise_mid;
  B3D_CHECK_HIP(launch_reduce_rows_grid(S->partial, M, S->n_bands, g.A * g.B, g, own_noise ? S->logL_new : S->noise_grid,
                                        nullptr, st),
                "smc_step");
  return B3D_OK;
}

extern "C" {

b3d_status b3d_contact_create(const b3d_mesh* const* types, int32_t n_types, const b3d_table* table,
                              b3d_contact** out) {
  if (!out) return fail(B3D_EINVAL, "contact_create: NULL output");
  *out = nullptr;
  std::vector<FaceDev> faces;
  if (b3d_status s = make_contact(types, n_types, table, &faces)) return s;
  FaceDev* fd = nullptr;
  if (hipMalloc((void**)&fd, sizeof(FaceDev) * faces.size()) != hipSuccess)
    return fail(B3D_ENOMEM, "contact_create: device allocation failed");
  if (hipMemcpy(fd, faces.data(), sizeof(FaceDev) * faces.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(fd);
    return fail(B3D_EHIP, "contact_create: upload failed");
  }
  b3d_contact* c = new b3d_contact();
  std::memcpy(c->C.T, table->pose, sizeof(c->C.T));
  c->C.faces = fd;
  c->C.n_types = n_types;
  *out = c;
  return B3D_OK;
}

b3d_status b3d_contact_destroy(b3d_contact* c) {
  if (!c) return B3D_OK;
  (void)hipFree((void*)c->C.faces);
  delete c;
  return B3D_OK;
}

b3d_status b3d_contact_poses(const b3d_contact* c, const int32_t* place, const float* dphi, int32_t N,
                             float* poses_out, void* stream) {
  if (!c) return fail(B3D_EINVAL, "contact_poses: NULL contact set");
  if (N < 0) return fail(B3D_ESHAPE, "contact_poses: N < 0");
  if (N == 0) return B3D_OK;
  if (!place || !dphi || !poses_out) return fail(B3D_EINVAL, "contact_poses: NULL buffer");
  B3D_CHECK_HIP(launch_contact_poses(c->C, place, dphi, N, poses_out, (hipStream_t)stream), "contact_poses");
  return B3D_OK;
}

b3d_status b3d_smc_create(const b3d_mesh* const* types, int32_t n_types, const b3d_mesh* const* fixed,
                          const float* fixed_poses, int32_t n_fixed, const b3d_table* table, const b3d_intrinsics* K,
                          const b3d_smc_params* p, b3d_smc** out) {
  if (!out || !p) return fail(B3D_EINVAL, "smc_create: NULL pointer");
  std::vector<FaceDev> faces;
  if (b3d_status s = make_contact(types, n_types, table, &faces)) return s;
  if (b3d_status s = check_intrinsics(K)) return s;
  const int M = p->n_particles;
  if (M < 1 || M > 1024) return fail(B3D_ESHAPE, "smc_create: need 1 <= n_particles <= 1024");
  if (p->n_objects < 1 || p->n_objects > B3D_MAX_SMC_OBJECTS)
    return fail(B3D_ESHAPE, "smc_create: need 1 <= n_objects <= %d", B3D_MAX_SMC_OBJECTS);
  if (p->n_stages < 1 || p->n_stages > B3D_MAX_STAGES)
    return fail(B3D_ESHAPE, "smc_create: need 1 <= n_stages <= %d", B3D_MAX_STAGES);
  int max_split = 0;
  for (int t = 0; t < p->n_stages; ++t) {
    long long n = 1;
    for (int k = 0; k < 3; ++k) {
      if (p->counts[t][k] < 1 || p->counts[t][k] > 4096) return fail(B3D_ESHAPE, "smc_create: counts out of range");
      n *= p->counts[t][k];
    }
    if (n > (1 << 20)) return fail(B3D_ESHAPE, "smc_create: stage %d splits into too many cells", t);
    if (t > 0) max_split = std::max(max_split, (int)n);
  }
  const long long n0 = (long long)p->counts[0][0] * p->counts[0][1] * p->counts[0][2];
  const long long N0 = n0 * 6 * n_types;
  if ((long long)M * N0 > (1ll << 26) || (long long)M * max_split > (1ll << 26))
    return fail(B3D_ESHAPE, "smc_create: too many hypotheses per stage");
  if (!(p->sigma_max > 0) || !std::isfinite(p->sigma_max)) return fail(B3D_EINVAL, "smc_create: sigma_max <= 0");
  if (!(p->sigma0 > 0) || !(p->p_out0 > 0) || !(p->p_out0 <= 1) || !std::isfinite(p->sigma0))
    return fail(B3D_EINVAL, "smc_create: bad initial noise");
  if (!(p->ess_threshold >= 0) || !std::isfinite(p->ess_threshold))
    return fail(B3D_EINVAL, "smc_create: bad ess_threshold");
  for (int t = 0; t < p->n_stages; ++t)
    if (!(p->stage_sigma[t] >= 0) || !std::isfinite(p->stage_sigma[t]) ||
        (p->stage_sigma[t] > 0 && !(p->stage_p_out[t] > 0 && p->stage_p_out[t] <= 1)))
      return fail(B3D_EINVAL, "smc_create: bad noise for stage %d", t);
  if (n_fixed < 0 || n_fixed > 16 || (n_fixed > 0 && (!fixed || !fixed_poses)))
    return fail(B3D_EINVAL, "smc_create: bad fixed content");
  if (n_fixed > 0 && !finite_all(fixed_poses, 16 * (size_t)n_fixed))
    return fail(B3D_EINVAL, "smc_create: non-finite fixed pose");
  // moving-mesh triangle ids are numbered below every background id: the
  // scenes are made with the largest type and the others swapped in
  int big = 0;
  uint64_t tris = 0;
  for (int o = 0; o < n_types; ++o)
    if (types[o]->T > types[big]->T) big = o;
  tris = (uint64_t)types[big]->T * (1 + p->n_objects);
  for (int f = 0; f < n_fixed; ++f) {
    if (!fixed[f]) return fail(B3D_EINVAL, "smc_create: NULL fixed mesh %d", f);
    tris += (uint64_t)fixed[f]->T;
  }
  if (tris >= 0xffffffffull) return fail(B3D_ESHAPE, "smc_create: too many triangles for 32-bit ids");
  b3d_score_params sp{p->sigma0, p->p_out0, p->outlier_volume, p->norm_M, p->window};
  {
    ScoreConsts sc;
    if (b3d_status s = make_consts(&sp, K->H, K->W, &sc)) return s;
  }
  // the noise proposal's cell midpoints
  const int A = p->noise_A, B = p->noise_B;
  if (A < 1 || B < 1 || A > kMaxSigma || A * B > kMaxNoise)
    return fail(B3D_ESHAPE, "smc_create: need 1 <= noise_A <= %d, noise_A * noise_B <= %d", kMaxSigma, kMaxNoise);
  std::vector<float> sig(A), po(B);
  if (b3d_status s = b3d_noise_midpoints(p->sigma_max, A, B, sig.data(), po.data())) return s;
  NoiseGridDev mid{};
  std::vector<b3d_score_params> per;
  if (b3d_status s = make_noise_grid(sp, K->H, K->W, sig.data(), A, po.data(), B, nullptr, &mid, &per)) return s;

  b3d_smc* S = new b3d_smc();
  auto bail = [&](b3d_status s) {
    b3d_smc_destroy(S);
    return s;
  };
  S->p = *p;
  S->table = *table;
  S->K = *K;
  S->types.assign(types, types + n_types);
  if (n_fixed > 0) {
    S->fixed.assign(fixed, fixed + n_fixed);
    S->fixed_poses.assign(fixed_poses, fixed_poses + 16 * (size_t)n_fixed);
  }
  S->n_stage0 = (int)N0;
  S->max_split = max_split;
  S->noise_mid = mid;
  for (int m = 0; m < M; ++m) {
    b3d_scene* sc = nullptr;
    if (b3d_status s = b3d_scene_create(types[big], K, &sp, &sc)) return bail(s);
    S->scenes.push_back(sc);
  }
  // device state
  const int n = p->n_objects, T = p->n_stages;
  FaceDev* fd = nullptr;
  b3d_status s = B3D_OK;
  if ((s = dev_alloc(S->owned, &fd, faces.size()))) return bail(s);
  std::memcpy(S->C.T, table->pose, sizeof(S->C.T));
  S->C.faces = fd;
  S->C.n_types = n_types;
  for (int b = 0; b < 2; ++b) {
    PartDev& d = S->st[b];
    if ((s = dev_alloc(S->owned, &d.place, (size_t)M * n * 2)) || (s = dev_alloc(S->owned, &d.dphi, (size_t)M * n * 3)) ||
        (s = dev_alloc(S->owned, &d.poses, (size_t)M * n * 16)) || (s = dev_alloc(S->owned, &d.noise, (size_t)M * 2)) ||
        (s = dev_alloc(S->owned, &d.logL, (size_t)M)) || (s = dev_alloc(S->owned, &d.logp, (size_t)M)) ||
        (s = dev_alloc(S->owned, &d.lprior, (size_t)M)) || (s = dev_alloc(S->owned, &d.logW, (size_t)M)))
      return bail(s);
  }
  const size_t hyp = std::max<size_t>((size_t)N0, (size_t)M * max_split);
  if ((s = dev_alloc(S->owned, &S->roots, (size_t)n_types * 6)) ||
      (s = dev_alloc(S->owned, &S->stage0_poses, (size_t)N0 * 16)) || (s = dev_alloc(S->owned, &S->hyp, hyp * 16)) ||
      (s = dev_alloc(S->owned, &S->logL_h, std::max<size_t>((size_t)M * N0, (size_t)M * max_split))) ||
      (s = dev_alloc(S->owned, &S->cells, (size_t)M)) || (s = dev_alloc(S->owned, &S->clogq, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->logq, (size_t)M)) || (s = dev_alloc(S->owned, &S->logp_new, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->lprior_new, (size_t)M)) || (s = dev_alloc(S->owned, &S->logW_pre, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->ess, 1)) || (s = dev_alloc(S->owned, &S->choice, (size_t)T * M)) ||
      (s = dev_alloc(S->owned, &S->idx, (size_t)M)) || (s = dev_alloc(S->owned, &S->nidx, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->drawn, (size_t)M)) || (s = dev_alloc(S->owned, &S->anc, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->logw, (size_t)M)) || (s = dev_alloc(S->owned, &S->nlogw, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->lw_shift, (size_t)M)) || (s = dev_alloc(S->owned, &S->dphi_new, (size_t)M * 3)) ||
      (s = dev_alloc(S->owned, &S->pose_new, (size_t)M * 16)) || (s = dev_alloc(S->owned, &S->noise_new, (size_t)M * 2)) ||
      (s = dev_alloc(S->owned, &S->logL_new, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->noise_grid, (size_t)M * A * B)) || (s = dev_alloc(S->owned, &S->marg, (size_t)M)) ||
      (s = dev_alloc(S->owned, &S->type_post, (size_t)M * n_types)))
    return bail(s);
  {
    // whole-image scores in bands of full-width rows, the largest that fit
    SceneDev d = S->scenes[0]->dev;
    d.zcap = max_zcap(d);
    const int h = d.sc.h;
    S->rows_R = d.zcap / (K->W + 4 * h) - 4 * h;
    if (S->rows_R < 1) return bail(fail(B3D_ESHAPE, "smc_create: image too wide for whole-image scoring"));
    S->n_bands = (K->H + S->rows_R - 1) / S->rows_R;
    if ((s = dev_alloc(S->owned, &S->partial, (size_t)M * S->n_bands * kMaxNoise))) return bail(s);
  }
  S->max_groups = (M * n_types + kBatchGroup - 1) / kBatchGroup;
  if ((s = dev_alloc(S->owned, &S->counters, 32 * (size_t)S->max_groups))) return bail(s);
  // the root cells (every type and face: dx, dy over the table less the
  // footprint, dth over a full turn) and the stage-0 hypotheses, the same
  // for every particle
  std::vector<CellDev> roots((size_t)n_types * 6);
  for (int o = 0; o < n_types; ++o)
    for (int c = 0; c < 6; ++c) {
      const FaceDev& f = faces[6 * o + c];
      CellDev& r = roots[6 * o + c];
      r.type = o;
      r.face = c;
      r.lo[0] = -0.5f * (table->width - f.w);
      r.hi[0] = 0.5f * (table->width - f.w);
      r.lo[1] = -0.5f * (table->height - f.h);
      r.hi[1] = 0.5f * (table->height - f.h);
      r.lo[2] = 0.0f;
      r.hi[2] = (float)(2.0 * M_PI);
    }
  if (hipMemcpy(fd, faces.data(), sizeof(FaceDev) * faces.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->roots, roots.data(), sizeof(CellDev) * roots.size(), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(B3D_EHIP, "smc_create: upload failed"));
  hipError_t e = launch_contact_enumerate(S->C, S->roots, n_types * 6, p->counts[0][0], p->counts[0][1],
                                          p->counts[0][2], S->stage0_poses, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return bail(hip_fail(e, "smc_create"));
  *out = S;
  return B3D_OK;
}

b3d_status b3d_smc_reset(b3d_smc* S, const float* observed, void* stream) {
  if (!S || !observed) return fail(B3D_EINVAL, "smc_reset: NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int M = S->p.n_particles;
  S->observed = observed;
  S->placed = 0;
  S->cur = 0;
  std::vector<float> noise((size_t)M * 2);
  for (int m = 0; m < M; ++m) {
    noise[2 * m] = S->p.sigma0;
    noise[2 * m + 1] = S->p.p_out0;
  }
  const int n = S->p.n_objects;
  for (int b = 0; b < 2; ++b) {  // slots of objects not yet placed read as zeros
    const PartDev& z = S->st[b];
    B3D_CHECK_HIP(hipMemsetAsync(z.place, 0, sizeof(int) * M * n * 2, st), "smc_reset");
    B3D_CHECK_HIP(hipMemsetAsync(z.dphi, 0, sizeof(float) * M * n * 3, st), "smc_reset");
    B3D_CHECK_HIP(hipMemsetAsync(z.poses, 0, sizeof(float) * M * n * 16, st), "smc_reset");
  }
  S->scored = 0;
  const PartDev& d = S->st[0];
  B3D_CHECK_HIP(hipMemcpyAsync(d.noise, noise.data(), sizeof(float) * noise.size(), hipMemcpyHostToDevice, st),
                "smc_reset");
  B3D_CHECK_HIP(hipMemsetAsync(d.logp, 0, sizeof(double) * M, st), "smc_reset");
  B3D_CHECK_HIP(hipMemsetAsync(d.lprior, 0, sizeof(double) * M, st), "smc_reset");
  B3D_CHECK_HIP(hipMemsetAsync(d.logW, 0, sizeof(double) * M, st), "smc_reset");
  B3D_CHECK_HIP(hipMemsetAsync(d.logL, 0, sizeof(float) * M, st), "smc_reset");
  // the noise values are read back by the next step
  B3D_CHECK_HIP(hipStreamSynchronize(st), "smc_reset");
  return B3D_OK;
}

b3d_status b3d_smc_step(b3d_smc* S, void* stream) {
  if (!S) return fail(B3D_EINVAL, "smc_step: NULL sampler");
  if (!S->observed) return fail(B3D_EINVAL, "smc_step: call b3d_smc_reset first");
  const b3d_smc_params& p = S->p;
  if (S->placed >= p.n_objects) return fail(B3D_ESHAPE, "smc_step: all %d objects are placed", p.n_objects);
  hipStream_t st = (hipStream_t)stream;
  const int M = p.n_particles, n = p.n_objects, k = S->placed, i = k + 1;
  const int n_types = (int)S->types.size(), AB = p.noise_A * p.noise_B;
  const uint32_t key0 = (uint32_t)p.seed, key1 = (uint32_t)(p.seed >> 32);
  const PartDev& in = S->st[S->cur];
  PartDev& out = S->st[1 - S->cur];

  // each particle's scene: the fixed content and its earlier objects as
  // background, scored at its current noise
  std::vector<float> h_poses((size_t)M * n * 16), h_noise((size_t)M * 2);
  std::vector<int> h_place((size_t)M * n * 2);
  B3D_CHECK_HIP(hipMemcpyAsync(h_noise.data(), in.noise, sizeof(float) * M * 2, hipMemcpyDeviceToHost, st), "smc_step");
  if (k > 0) {
    B3D_CHECK_HIP(hipMemcpyAsync(h_poses.data(), in.poses, sizeof(float) * h_poses.size(), hipMemcpyDeviceToHost, st),
                  "smc_step");
    B3D_CHECK_HIP(hipMemcpyAsync(h_place.data(), in.place, sizeof(int) * h_place.size(), hipMemcpyDeviceToHost, st),
                  "smc_step");
  }
  B3D_CHECK_HIP(hipStreamSynchronize(st), "smc_step");
  // particles with equal noise and equal objects (copies made by resampling,
  // and all of them before the first object) score every hypothesis alike:
  // one scene per distinct state, its stage-0 scores copied to the others
  bool own_noise = false;  // some stage scores at the particles' own noise
  for (int t = 0; t < p.n_stages; ++t) own_noise = own_noise || !(p.stage_sigma[t] > 0);
  std::vector<int> rep((size_t)M);
  for (int m = 0; m < M; ++m) {
    rep[m] = m;
    for (int u = 0; u < m; ++u) {
      if (rep[u] != u) continue;
      bool same = !own_noise || (h_noise[2 * u] == h_noise[2 * m] && h_noise[2 * u + 1] == h_noise[2 * m + 1]);
      for (int j = 0; same && j < k; ++j) {
        const size_t a = (size_t)u * n + j, b = (size_t)m * n + j;
        same = h_place[2 * a] == h_place[2 * b] &&
               std::memcmp(&h_poses[16 * a], &h_poses[16 * b], 16 * sizeof(float)) == 0;
      }
      if (same) {
        rep[m] = u;
        break;
      }
    }
  }
  // the noise at which stage t scores particle m's cells
  b3d_score_params sp_buf{};
  auto stage_noise = [&](int m, int t) -> const b3d_score_params& {
    sp_buf = b3d_score_params{p.stage_sigma[t] > 0 ? p.stage_sigma[t] : h_noise[2 * m],
                              p.stage_sigma[t] > 0 ? p.stage_p_out[t] : h_noise[2 * m + 1], p.outlier_volume,
                              p.norm_M, p.window};
    return sp_buf;
  };
  std::vector<const b3d_mesh*> bg_mesh;
  std::vector<float> bg_pose;
  for (int m = 0; m < M; ++m) {
    if (rep[m] != m) continue;
    bg_mesh.assign(S->fixed.begin(), S->fixed.end());
    bg_pose.assign(S->fixed_poses.begin(), S->fixed_poses.end());
    for (int j = 0; j < k; ++j) {
      bg_mesh.push_back(S->types[std::min(std::max(h_place[2 * ((size_t)m * n + j)], 0), n_types - 1)]);
      bg_pose.insert(bg_pose.end(), h_poses.begin() + 16 * ((size_t)m * n + j),
                     h_poses.begin() + 16 * ((size_t)m * n + j + 1));
    }
    b3d_scene* sc = S->scenes[m];
    if (b3d_status s = b3d_scene_set_background(sc, bg_mesh.data(), bg_pose.data(), (int)bg_mesh.size(), st)) return s;
    if (b3d_status s = b3d_scene_set_params(sc, &stage_noise(m, 0), st)) return s;
    if (b3d_status s = b3d_scene_set_observed(sc, S->observed, st)) return s;
  }
  // the tile: timed once, on the first step, over the largest type's stage-0 cells
  const int n0 = p.counts[0][0] * p.counts[0][1] * p.counts[0][2], N0 = S->n_stage0;
  if (S->zcap == 0) {
    int big = 0;
    for (int o = 0; o < n_types; ++o)
      if (S->types[o]->T > S->types[big]->T) big = o;
    b3d_scene* sc = S->scenes[rep[0]];
    SceneDev keep = sc->dev;
    sc->dev.mesh = S->types[big]->dev;
    int z = 0;
    const b3d_status s = b3d_scene_autotune(sc, S->stage0_poses + 16 * (size_t)big * 6 * n0, 6 * n0, 0, &z, st);
    sc->dev.mesh = keep.mesh;
    if (s) return s;
    S->zcap = z;
  }
  auto scene_of = [&](int m, int o) {
    SceneDev d = S->scenes[rep[m]]->dev;
    d.mesh = S->types[o]->dev;
    d.zcap = S->zcap;
    return d;
  };

  // stage 0: every (type, face) box split, the same hypotheses for every particle
  std::vector<BatchItemDev> items;
  for (int m = 0; m < M; ++m)
    if (rep[m] == m)
      for (int o = 0; o < n_types; ++o)
        items.push_back(BatchItemDev{scene_of(m, o), S->stage0_poses + 16 * (size_t)o * 6 * n0, 6 * n0,
                                     S->logL_h + (size_t)m * N0 + (size_t)o * 6 * n0, nullptr});
  BatchPlan plan;
  if (b3d_status s = plan_batch(items, false, &plan)) return s;
  if (b3d_status s = run_batch_queue(plan, S->counters, st)) return s;
  for (const BatchItemDev& it : items) S->scored += it.N;
  for (int m = 0; m < M; ++m)
    if (rep[m] != m)
      B3D_CHECK_HIP(hipMemcpyAsync(S->logL_h + (size_t)m * N0, S->logL_h + (size_t)rep[m] * N0, sizeof(float) * N0,
                                   hipMemcpyDeviceToDevice, st),
                    "smc_step");
  B3D_CHECK_HIP(launch_type_posterior(S->logL_h, M, N0, n_types, 6 * n0, S->type_post, st), "smc_step");
  B3D_CHECK_HIP(launch_sample(S->logL_h, M, N0, 1, key0, key1, ((uint32_t)i << 8) | 0u, 0u, nullptr, S->idx, S->logw, st),
                "smc_step");
  B3D_CHECK_HIP(launch_contact_choose(S->roots, p.counts[0][0], p.counts[0][1], p.counts[0][2], S->idx, S->logw, M,
                                      S->cells, S->clogq, S->choice, st),
                "smc_step");
  // the chosen types set up the later stages' launches
  std::vector<CellDev> h_cells((size_t)M);
  B3D_CHECK_HIP(hipMemcpyAsync(h_cells.data(), S->cells, sizeof(CellDev) * M, hipMemcpyDeviceToHost, st), "smc_step");
  B3D_CHECK_HIP(hipStreamSynchronize(st), "smc_step");
  std::vector<int> type_of((size_t)M);
  for (int m = 0; m < M; ++m) type_of[m] = std::min(std::max(h_cells[m].type, 0), n_types - 1);
  for (int t = 1; t < p.n_stages; ++t) {
    const int nx = p.counts[t][0], ny = p.counts[t][1], nt = p.counts[t][2], ns = nx * ny * nt;
    const bool change = p.stage_sigma[t] != p.stage_sigma[t - 1] || p.stage_p_out[t] != p.stage_p_out[t - 1];
    if (change)  // the stage's own noise (the background terms follow)
      for (int m = 0; m < M; ++m)
        if (rep[m] == m)
          if (b3d_status s = b3d_scene_set_params(S->scenes[m], &stage_noise(m, t), st)) return s;
    B3D_CHECK_HIP(launch_contact_enumerate(S->C, S->cells, M, nx, ny, nt, S->hyp, st), "smc_step");
    items.clear();
    for (int m = 0; m < M; ++m)
      items.push_back(BatchItemDev{scene_of(m, type_of[m]), S->hyp + 16 * (size_t)m * ns, ns,
                                   S->logL_h + (size_t)m * ns, nullptr});
    if (b3d_status s = plan_batch(items, false, &plan)) return s;
    if (b3d_status s = run_batch_queue(plan, S->counters, st)) return s;
    S->scored += (long long)M * ns;
    B3D_CHECK_HIP(launch_sample(S->logL_h, M, ns, 1, key0, key1, ((uint32_t)i << 8) | (uint32_t)t, 0u, nullptr, S->idx,
                                S->logw, st),
                  "smc_step");
    B3D_CHECK_HIP(launch_contact_choose(nullptr, nx, ny, nt, S->idx, S->logw, M, S->cells, S->clogq,
                                        S->choice + (size_t)t * M, st),
                  "smc_step");
  }
  B3D_CHECK_HIP(launch_contact_draw(S->C, S->cells, M, key0, key1, (uint32_t)i, S->clogq, S->dphi_new, S->pose_new,
                                    S->logq, st),
                "smc_step");

  // the noise: midpoint-scored cells over the whole image, then a uniform point of the drawn one
  if (b3d_status s = whole_image_scores(S, st, type_of, rep, false)) return s;
  B3D_CHECK_HIP(launch_sample(S->noise_grid, M, AB, 1, key0, key1, ((uint32_t)i << 8) | 0x40u, 0u, nullptr, S->nidx,
                              S->nlogw, st),
                "smc_step");
  B3D_CHECK_HIP(launch_noise_draw(S->nidx, S->nlogw, M, p.noise_A, p.noise_B, p.sigma_max, key0, key1, (uint32_t)i,
                                  S->noise_new, S->logq, st),
                "smc_step");
  // logL of each particle's scene at its new noise
  if (b3d_status s = whole_image_scores(S, st, type_of, rep, true)) return s;

  // eq. (2)/(3), then resampling
  StageDev sd{S->cells, S->dphi_new, S->pose_new, S->noise_new, S->logL_new, S->logq, S->logp_new, S->lprior_new,
              S->logW_pre};
  B3D_CHECK_HIP(launch_smc_reweight(S->C, M, i, std::log((double)p.sigma_max), in, sd, S->lw_shift, st), "smc_step");
  B3D_CHECK_HIP(launch_sample(S->lw_shift, 1, M, M, key0, key1, ((uint32_t)i << 8) | 0x80u, 0u, nullptr, S->drawn,
                              nullptr, st),
                "smc_step");
  B3D_CHECK_HIP(launch_smc_resample(M, n, k, p.ess_threshold, in, sd, S->drawn, out, S->anc, S->ess, st), "smc_step");
  S->cur = 1 - S->cur;
  S->placed = i;
  return B3D_OK;
}

b3d_status b3d_smc_read(const b3d_smc* S, const b3d_smc_view* v, int32_t* n_placed, int64_t* n_scored,
                        void* stream) {
  if (!S || !v) return fail(B3D_EINVAL, "smc_read: NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int M = S->p.n_particles, n = S->p.n_objects, AB = S->p.noise_A * S->p.noise_B;
  const PartDev& d = S->st[S->cur];
  auto cp = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return dst ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  const hipError_t es[] = {
      cp(v->place, d.place, sizeof(int) * M * n * 2), cp(v->dphi, d.dphi, sizeof(float) * M * n * 3),
      cp(v->poses, d.poses, sizeof(float) * M * n * 16), cp(v->noise, d.noise, sizeof(float) * M * 2),
      cp(v->logW, d.logW, sizeof(double) * M), cp(v->logp, d.logp, sizeof(double) * M),
      cp(v->logL, d.logL, sizeof(float) * M), cp(v->choice, S->choice, sizeof(int) * S->p.n_stages * M),
      cp(v->logq, S->logq, sizeof(double) * M), cp(v->logW_pre, S->logW_pre, sizeof(double) * M),
      cp(v->noise_grid, S->noise_grid, sizeof(float) * M * AB), cp(v->ancestors, S->anc, sizeof(int) * M),
      cp(v->ess, S->ess, sizeof(double)),
      cp(v->type_post, S->type_post, sizeof(float) * M * S->types.size())};
  for (hipError_t x : es)
    if (x != hipSuccess) e = x;
  if (e != hipSuccess) return hip_fail(e, "smc_read");
  if (n_placed) *n_placed = S->placed;
  if (n_scored) *n_scored = S->scored;
  return B3D_OK;
}

b3d_status b3d_smc_destroy(b3d_smc* S) {
  if (!S) return B3D_OK;
  (void)hipDeviceSynchronize();
  for (b3d_scene* sc : S->scenes) b3d_scene_destroy(sc);
  for (void* q : S->owned) (void)hipFree(q);
  delete S;
  return B3D_OK;
}

}  // extern "C"

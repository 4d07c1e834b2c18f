// Host-visible launch wrappers of the gfx950 kernels and the by-value
// argument structs they take.  The C ABI in api.cpp validates arguments and
// calls these; every wrapper only enqueues work on the given stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "b3d_device.hpp"

namespace b3d {

// Constants of the windowed likelihood derived from b3d_score_params.
struct ScoreConsts {
  float a;       // p_out / V
  float bn;      // (1 - p_out)/M * (2 pi sigma^2)^(-3/2)
  float c2;      // log2(e) / (2 sigma^2): exp(-D/(2 sigma^2)) = exp2(-D c2)
  float inv_s, inv_s2, inv_s3;
  float invV;    // 1 / V
  float normM;   // (2 pi sigma^2)^(-3/2) / M
  int h;         // window half-width
  // double-precision copies for the background terms
  double da, dbn, dc, dinv_s, dinv_s3, dinvV, dnormM;
};

// Everything the fused render+score kernel needs about a scene.
struct SceneDev {
  MeshDev mesh;
  Cam cam;
  ScoreConsts sc;
  const float* obs;                // [H][W][3]
  const unsigned long long* bg;    // [H][W] background keys, or nullptr
  const double* sat;               // 3 summed-area tables [(H+1)(W+1)]: l, dl/dp, dl/dsigma of the background
  int zcap, wcap;                  // LDS capacities: depth keys, window weights (wcap <= kRasterLdsBytes / 4)
};

// A grid of noise parameters for the hierarchical likelihood: A standard
// deviations x B outlier probabilities, grid point k = a * B + b (at most
// kMaxNoise points, at most kMaxSigma deviations).  Per deviation: the
// exponent scale and the inlier normaliser; per grid point: its deviation's
// index, p_out / V, 1 - p_out and the log quadrature weight; and the
// summed-area tables of the background-only per-pixel terms (table 0 of
// each stride-spaced group of three, as the scene's own).
constexpr int kMaxNoise = 16;
constexpr int kMaxSigma = 8;
// Scenes per multi-scene launch (their descriptors travel as kernel arguments).
constexpr int kBatchGroup = 8;

struct NoiseGridDev {
  int A, B;
  float c2[kMaxSigma];     // log2(e) / (2 sigma_a^2)
  float normM[kMaxSigma];  // (2 pi sigma_a^2)^(-3/2) / M
  int ka[kMaxNoise];       // deviation index of grid point k
  float pa[kMaxNoise];     // p_out / V
  float pomp[kMaxNoise];   // 1 - p_out
  float logw[kMaxNoise];
  const double* sat;
  long long sat_stride;    // doubles between consecutive grid points' tables
};
hipError_t launch_render_score_grid(const SceneDev& s, const NoiseGridDev& g, const float* poses, int N,
                                    float* logL_grid, float* logL_marg, hipStream_t st);

// Whole-image scores of one pose per scene, for up to kBatchGroup scenes
// (one camera size, one LDS size: the first scene's), each under the group's
// noise grid or under its own (sigma, p_out) at noise[j].
struct RowsGroupDev {
  SceneDev s[kBatchGroup];
  const float* pose[kBatchGroup];   // device float[16]
  const float* noise[kBatchGroup];  // device float[2] or nullptr
  NoiseGridDev grid;
  double inv_V, M_norm;             // for the per-scene noise
  int first;                        // index of scene 0 in the partial-sum rows
  int S;
};
static_assert(sizeof(RowsGroupDev) <= 4000, "a rows group must fit the kernel-argument segment");
// Bands of R full-width rows per block: partial[(scene n_bands + band) kMaxNoise + k].
hipError_t launch_score_rows_grid(const RowsGroupDev& G, int R, int n_bands, float* partial, hipStream_t st);
// Band sums per (scene, grid point) in band order (double), logL to
// grid_out[scene nk + k], and the weighted log-sum-exp to marg_out (or none).
hipError_t launch_reduce_rows_grid(const float* partial, int P, int n_bands, int nk, const NoiseGridDev& g,
                                   float* grid_out, float* marg_out, hipStream_t st);

// Object types in an SMC library.
constexpr int kMaxTypes = 16;

// Table-contact placement (see b3d_contact_poses): the resting frame of face
// c of a type's bounding box and the log prior density of a placement on it.
struct FaceDev {
  float R[9];     // object frame -> resting frame (entries 0, +-1)
  float d[3];     // puts the face on z = 0 with its centre on the origin
  float w, h;     // footprint extents along x and y
  double lprior;  // log(1/|O| 1/6 1/((W_t - w)(H_t - h)) 1/(2 pi))
};
struct ContactDev {
  float T[16];           // table frame -> camera
  const FaceDev* faces;  // device [n_types][6]
  int n_types;
};
// A cell of the placement partition: type, face and the box [lo, hi) of
// (dx, dy, dth).
struct CellDev {
  int type, face;
  float lo[3], hi[3];
};
// Particle state of the SMC sampler (device arrays, M particles, n slots).
struct PartDev {
  int* place;      // [M][n][2]
  float* dphi;     // [M][n][3]
  float* poses;    // [M][n][16]
  float* noise;    // [M][2]
  float* logL;     // [M]
  double* logp;    // [M]
  double* lprior;  // [M]
  double* logW;    // [M]
};
// Proposals of one SMC stage, before resampling.
struct StageDev {
  const CellDev* cells;     // [M] final cells (type, face)
  const float* dphi;        // [M][3]
  const float* poses;       // [M][16]
  const float* noise;       // [M][2]
  const float* logL;        // [M]
  const double* logq;       // [M]
  double* logp;             // [M] written by the reweight
  double* lprior;           // [M] written by the reweight
  double* logW_pre;         // [M] written by the reweight
};

// Posterior over type of each particle's stage-0 cells (one block per particle).
hipError_t launch_type_posterior(const float* logL, int M, int N, int n_types, int per_type, float* post,
                                 hipStream_t st);
hipError_t launch_contact_poses(const ContactDev& C, const int* place, const float* dphi, int N, float* poses,
                                hipStream_t st);
// Poses of the centres of every cell's split into nx x ny x nt cells:
// poses[(p * n + j) * 16], n = nx ny nt.
hipError_t launch_contact_enumerate(const ContactDev& C, const CellDev* cells, int P, int nx, int ny, int nt,
                                    float* poses, hipStream_t st);
// Move each particle into its drawn cell.  roots != nullptr: stage 0, draw
// n = r * n_split + j picks split cell j of roots[r]; else split cell idx of
// cells[m].  clogq = logw (stage 0) or += logw.
hipError_t launch_contact_choose(const CellDev* roots, int nx, int ny, int nt, const int* idx, const float* logw, int M,
                                 CellDev* cells, double* clogq, int* choice, hipStream_t st);
// A uniform point of each final cell: placement, pose and log q so far.
hipError_t launch_contact_draw(const ContactDev& C, const CellDev* cells, int M, uint32_t key0, uint32_t key1,
                               uint32_t i, const double* clogq, float* dphi, float* poses, double* logq,
                               hipStream_t st);
// A uniform point of each particle's drawn noise cell; logq += its log density.
hipError_t launch_noise_draw(const int* nidx, const float* nlogw, int M, int A, int B, float sigma_max,
                             uint32_t key0, uint32_t key1, uint32_t i, float* noise, double* logq, hipStream_t st);
// log p_i, the log prior sum and the pre-resampling log weights (one block);
// lw_shift = logW_pre - max, as floats for the resampling draws.
hipError_t launch_smc_reweight(const ContactDev& C, int M, int i, double log_sigma_max, const PartDev& in,
                               const StageDev& sd, float* lw_shift, hipStream_t st);
// Effective sample size, the resampling decision, and the next state (one
// block): survivors copy in[src]'s first k objects and the stage's proposal.
hipError_t launch_smc_resample(int M, int n_slots, int k, float threshold, const PartDev& in, const StageDev& sd,
                               const int* drawn, PartDev out, int* ancestors, double* ess, hipStream_t st);

// A group of up to kBatchGroup scenes of a multi-scene batch, passed to the
// kernel by value: pointers that arrive as kernel arguments are known to be
// global memory, so the compiler addresses through them with a scalar base
// (pointers read from a device array would be generic, flat-addressed).
// Scene k's hypotheses are work items [first[k], first[k + 1]).
struct BatchGroupDev {
  SceneDev s[kBatchGroup];
  const float* poses[kBatchGroup];
  float* logL[kBatchGroup];
  float* grad[kBatchGroup];
  long long first[kBatchGroup + 1];
  int S;
};
static_assert(sizeof(BatchGroupDev) <= 4000, "a batch group must fit the kernel-argument segment");

// Generic grid description for the hypothesis expander.
struct GridDev {
  float center[16];
  float half[3];
  int count[3];
  int cell_centres;
  int n_rot;
  float max_angle;
  const float* rots;  // device [n_rot][9] or nullptr (generated)
};

// LDS bytes of the fused kernel: fixed part + kFusedBytesPerKey per depth key.
constexpr size_t kFusedBytesPerKey = 8;
size_t fused_lds_bytes(const SceneDev& s);

hipError_t launch_render_batch(const MeshDev& m, const Cam& cam, const float* poses, int N, float* xyz, int* tri,
                               int zcap, hipStream_t st);
hipError_t launch_unproject(const float* depth, int B, const Cam& cam, float* xyz, hipStream_t st);
hipError_t launch_render_backward(const MeshDev& m, const Cam& cam, const float* poses, int N, const int* tri,
                                  const float* d_rend, float* d_pose, hipStream_t st);
// Split-path likelihood over a ring of rows (one pass over each point
// image), the observed image's valid pixels listed first in a workspace of
// score_workspace_bytes: rows per step for an H x W image and window
// half-width h, 0 when the ring does not apply (W not a multiple of 4, or
// the rows do not fit).
int score_ring_rows(int H, int W, int h);
int score_backward_ring_rows(int H, int W, int h);
size_t score_workspace_bytes(int H, int W);
hipError_t launch_score_ring(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc, int R,
                             void* workspace, float* logL, hipStream_t st);
hipError_t launch_score_backward_ring(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc,
                                      int R, void* workspace, const float* dlogL, float* d_rend, float* d_sigma,
                                      float* d_pout, hipStream_t st);
hipError_t launch_score(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc, float* logL,
                        int cap, hipStream_t st);
hipError_t launch_score_backward(const float* obs, const float* rend, int N, int H, int W, const ScoreConsts& sc,
                                 const float* dlogL, float* d_rend, float* d_sigma, float* d_pout, int cap,
                                 hipStream_t st);
hipError_t launch_render_score(const SceneDev& s, const float* poses, int N, float* logL, float* grad, hipStream_t st);
hipError_t launch_render_score_count(const SceneDev& s, const float* poses, int N, float* logL, float* grad,
                                     unsigned long long* work, hipStream_t st);

// One workgroup per hypothesis of the group's scenes.
hipError_t launch_batch(const BatchGroupDev& g, bool grad, size_t lds, hipStream_t st);
// The same by `blocks` persistent workgroups draining a device counter (256
// bytes of device memory per launch).
hipError_t batch_queue_occupancy(bool grad, size_t lds, int* blocks_per_cu);
hipError_t launch_batch_queue(const BatchGroupDev& g, unsigned long long* counter, bool grad, size_t lds, int blocks,
                              hipStream_t st);

// scene preparation
hipError_t launch_fill_keys(unsigned long long* keys, size_t n, hipStream_t st);
hipError_t launch_raster_global(const MeshDev& m, const Cam& cam, const float* pose16_host, uint32_t id_base,
                                unsigned long long* keys, hipStream_t st);
hipError_t launch_refine_global(const MeshDev& m, const Cam& cam, const float* pose16_host, const float* pose16_dev,
                                uint32_t id_base, unsigned long long* keys, hipStream_t st);
hipError_t launch_background_terms(const SceneDev& s, double* terms, hipStream_t st);

// hypotheses and sampling
hipError_t launch_enumerate(const GridDev& g, const float* centres, int P, uint32_t key0, uint32_t key1,
                            uint32_t stage, float* poses, hipStream_t st,
                            const float* hscale = nullptr);
hipError_t launch_sample(const float* logL, int P, int N, int K, uint32_t key0, uint32_t key1, uint32_t stage,
                         uint32_t k0, float* w, int* idx, float* logw, hipStream_t st);
hipError_t launch_c2f_update(const float* poses, int P, int N, const int* idx, const float* logw, int K_draws,
                             int accumulate, float* centres, float* logq, int* idx_out, hipStream_t st);

// refinement and tracking
hipError_t launch_pose_retract(const float* base, int n_base, const float* xi, int N, float* out, hipStream_t st);
hipError_t launch_pose_retract_backward(const float* xi, const float* grad, const float* dlogL, int N, float* dxi,
                                        float* dsp, hipStream_t st);
hipError_t launch_refine_pose(const SceneDev& s, float* poses, int N, int n_refine, float lr_t, float lr_r, float b1,
                              float b2, float eps, hipStream_t st);
// n_refine Adam steps of one pose, each over row bands of R image rows (one
// block per band, ceil(H / R) blocks) then a one-thread reduce + update.
// partial: device float[ceil(H / R)][9]; state: device float[12] (moments).
hipError_t launch_refine_banded(const SceneDev& s, float* pose, int n_refine, float lr_t, float lr_r, float b1,
                                float b2, float eps, int R, float* partial, float* state, hipStream_t st);
hipError_t launch_adam_pose(float* poses, const float* grad, int gstride, float* state, int N, int iter, float lr_t,
                            float lr_r, float b1, float b2, float eps, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);
hipError_t launch_copy_f32(const float* src, int n, float* dst, hipStream_t st);
// The tracker's occlusion decision for one object (one block): the fraction
// of its pixels in objkeys that are in front of bg (null: no other objects)
// and have an observed point within tol of theirs in their (2h + 1)^2
// window; then either keep the update (and record its motion from prev) or
// replace it by prev moved by the last motion; gate: (that fraction, dropped
// in a row, next stage 0 translation scale, 0).
hipError_t launch_track_gate(const unsigned long long* objkeys, const unsigned long long* bg, const float* obs,
                             const Cam& cam, int h, float tol, float min_visible, float widen, const float* prev,
                             float* pose, float* motion, float* gate, hipStream_t st);
hipError_t launch_argmax_pose(const float* logL, const float* poses, int N, float* out, hipStream_t st);
hipError_t launch_raster_global_dev(const MeshDev& m, const Cam& cam, const float* pose16_dev, uint32_t id_base,
                                    unsigned long long* keys, hipStream_t st);

}  // namespace b3d

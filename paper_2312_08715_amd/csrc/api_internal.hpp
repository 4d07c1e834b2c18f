// Declarations shared by the translation units of the C ABI (not part of
// the public interface): error reporting, validation helpers and the opaque
// handle types.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "b3d.h"
#include "b3d_launch.hpp"

namespace b3d_api {

using namespace b3d;

extern thread_local std::string g_err;

// Record a formatted message for b3d_last_error and return s.
b3d_status fail(b3d_status s, const char* fmt, ...);
b3d_status hip_fail(hipError_t e, const char* where);

constexpr int kMaxImage = 4096;
constexpr size_t kLdsMax = 65536;

bool finite_all(const float* p, size_t n);
b3d_status check_intrinsics(const b3d_intrinsics* K);
Cam make_cam(const b3d_intrinsics* K);
// Likelihood constants of eq. (1) for an H x W image (validates p).
b3d_status make_consts(const b3d_score_params* p, int H, int W, ScoreConsts* sc);
int default_zcap(const SceneDev& d, int blocks_per_cu);
int min_zcap(const SceneDev& d);
int max_zcap(const SceneDev& d);

// Noise-grid constants for sigma[A] x p_out[B] (other parameters from base);
// log_w: A*B log weights or nullptr for equal weights.  sat is left unset.
b3d_status make_noise_grid(const b3d_score_params& base, int H, int W, const float* sigma, int A, const float* p_out,
                           int B, const float* log_w, NoiseGridDev* g, std::vector<b3d_score_params>* per_point);

// One scene's share of a multi-scene launch, and the launch plan: scenes
// ordered by estimated cost, kBatchGroup per launch.
struct BatchItemDev {
  SceneDev s;
  const float* poses;
  int N;
  float* logL;
  float* grad;
};
struct BatchPlan {
  std::vector<BatchGroupDev> groups;
  bool grad = false;
  size_t lds = 0;
};
// cap_tiles: cap each scene's depth-buffer tile at the default (four
// workgroups per CU), for callers whose scenes carry tiles tuned for lone
// launches; callers that chose one tile for the whole batch by timing it
// keep theirs.
b3d_status plan_batch(const std::vector<BatchItemDev>& items, bool grad, BatchPlan* plan, bool cap_tiles = false);
// The plan's launches in order on st; with a side stream (and two events),
// every other launch goes there, forked from and joined back into st, so
// that one launch's tail overlaps the next one's start.
b3d_status run_batch(const BatchPlan& plan, hipStream_t st, hipStream_t side = nullptr, hipEvent_t fork = nullptr,
                     hipEvent_t join = nullptr);
// The plan's launches in order on st, each drained by a persistent grid
// through its counter (counters: device, 256 B per launch).
b3d_status run_batch_queue(const BatchPlan& plan, unsigned long long* counters, hipStream_t st);

}  // namespace b3d_api

#define B3D_CHECK_HIP(expr, where)                                   \
  do {                                                               \
    hipError_t e_ = (expr);                                          \
    if (e_ != hipSuccess) return b3d_api::hip_fail(e_, where);       \
  } while (0)

struct b3d_mesh {
  int V = 0, T = 0, n_clusters = 0, n_drawn = 0, n_hidden = 0, n_dropped = 0;
  float box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};  // exact bounds of the vertices (object frame)
  b3d::MeshDev dev{};
  std::vector<void*> allocs;
};

struct b3d_scene {
  const b3d_mesh* mesh = nullptr;
  b3d_intrinsics K{};
  b3d_score_params params{};
  b3d::SceneDev dev{};
  unsigned long long* bg = nullptr;  // background keys [H][W]
  double* terms = nullptr;           // [3][H][W]
  double* sat = nullptr;             // [3][(H+1)(W+1)]
  bool has_bg = false;
  bool observed = false;
  // hierarchical likelihood: noise grid and its background summed-area tables
  b3d::NoiseGridDev grid{};
  std::vector<b3d_score_params> grid_params;  // per grid point
  double* grid_sat = nullptr;                // [A*B][3][(H+1)(W+1)]
};


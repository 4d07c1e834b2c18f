/*
 * b3d — batched render-and-score for coarse-to-fine pose inference on
 * AMD Instinct MI355X (gfx950), after Bayes3D (Gothoskar et al., arXiv
 * 2312.08715).
 *
 * The library renders a voxel-mesh object under many pose hypotheses at low
 * resolution, scores each rendered point image against one observed point
 * image with the paper's robust windowed likelihood, normalises the scores
 * and samples from them, and differentiates the score with respect to each
 * hypothesis's pose and the noise parameters.
 *
 * Conventions shared by every entry point
 *   Units        metres and radians.
 *   Camera       pinhole, +z forward, +x right, +y down.  Pixel (r, c) has
 *                its centre at (c + 1/2, r + 1/2) and its ray is
 *                d = ((c + 1/2 - cx)/fx, (r + 1/2 - cy)/fy, 1).  Depth is
 *                camera z (not range).
 *   Pose         float[16], row-major 4x4 object-to-camera transform
 *                [R t; 0 0 0 1].  A pose batch is float[N][16].
 *   Tangent      a pose update (dt, dw) means R <- exp([dw]x) R, t <- t + dt.
 *   Point image  float[H][W][3] camera-frame xyz; a pixel is empty / invalid
 *                iff its z is not > 0.
 *   Memory       pointers documented "device" must be device memory on the
 *                current HIP device; "host" pointers are read before the
 *                call returns.  The caller owns every buffer it passes; the
 *                library owns mesh and scene handles.  No entry point marked
 *                "stream-ordered" allocates, frees or synchronises: it only
 *                enqueues work on `stream` (a hipStream_t; NULL = the null
 *                stream) and results are valid once the stream reaches them.
 *   Errors       every entry point validates its arguments before enqueuing
 *                anything and returns a b3d_status; on failure
 *                b3d_last_error() (per thread) describes the problem.  An
 *                asynchronous fault surfaces as B3D_EHIP at a later call.
 *   N == 0       is a no-op that returns B3D_OK.
 */
#ifndef B3D_H
#define B3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum b3d_status {
  B3D_OK = 0,
  B3D_EINVAL = -1,  /* bad argument (null pointer, out-of-range value) */
  B3D_ENOMEM = -2,  /* device allocation failed (set-up calls only) */
  B3D_EHIP = -3,    /* the HIP runtime reported an error */
  B3D_ESHAPE = -4,  /* inconsistent sizes, or a size beyond a stated limit */
  B3D_ENOTSUP = -5  /* a combination the library does not implement */
} b3d_status;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* b3d_last_error(void);
/* Library version string. */
const char* b3d_version(void);

/* Pinhole intrinsics and image size.  A triangle with a vertex at camera z
 * <= z_near is not drawn (no clipping).  1 <= H, W <= 4096. */
typedef struct b3d_intrinsics {
  float fx, fy, cx, cy, z_near;
  int32_t H, W;
} b3d_intrinsics;

/* Parameters of the robust likelihood, eq. (1) of the paper truncated to a
 * window (Sec. III-B, scoring strategy):
 *   l_i    = ln( p_out/V + (1 - p_out)/M * sum_{j in W(i), z_j > 0} N3(q~_i; q_j, sigma) )
 *   logL_n = sum over observed pixels i with z~_i > 0 of l_i
 * N3 = isotropic 3-D Gaussian density with standard deviation `sigma`;
 * W(i) = the window x window square centred on i, clipped to the image;
 * V = outlier_volume; M = norm_M, or H*W when norm_M <= 0.
 * Valid: sigma > 0, 0 < p_out <= 1, outlier_volume > 0, window odd, 1..15. */
typedef struct b3d_score_params {
  float sigma, p_out, outlier_volume, norm_M;
  int32_t window;
} b3d_score_params;

/* ---- meshes ------------------------------------------------------------ */

typedef struct b3d_mesh b3d_mesh;

/* Upload a triangle mesh (the learned voxel model of Fig. 1: one cube per
 * occupied cell).  verts: host float[V][3], object frame; tris: host
 * int32[T][3], counter-clockwise seen from outside; triangle id = row.
 * 1 <= V, 1 <= T <= 2^24.  Allocates device memory (not stream-ordered;
 * synchronises the current device).  *out receives the handle. */
b3d_status b3d_mesh_create(const float* verts, int32_t V, const int32_t* tris, int32_t T, b3d_mesh** out);
/* Free a mesh (synchronises the current device).  NULL is accepted. */
b3d_status b3d_mesh_destroy(b3d_mesh* mesh);
/* Vertex count, triangle count and number of primitive clusters the device
 * layout uses (any pointer may be NULL). */
b3d_status b3d_mesh_info(const b3d_mesh* mesh, int32_t* V, int32_t* T, int32_t* n_clusters);

/* How b3d_mesh_create lays a mesh out, computed on the host without a
 * device: info[0] = clusters, info[1] = clusters always drawn, info[2] =
 * triangles always drawn, info[3] = triangles drawn only when the object
 * reaches the near plane (coincident opposite faces of two different closed
 * components, which a camera outside the object never sees), info[4] =
 * triangles with a repeated vertex position (never drawn), info[5] = quads
 * (pairs of triangles sharing an edge, coplanar and convex, rasterised as one
 * primitive; the other drawn triangles are single primitives).  info: host
 * int32[6]. */
b3d_status b3d_mesh_layout_info(const float* verts, int32_t V, const int32_t* tris, int32_t T, int32_t* info);

/* ---- the split path: point images in device memory ---------------------- */

/* Depth to point image (Sec. III-A (iii): the render is turned into a point
 * cloud in the camera frame): xyz = z d for z > 0, else 0.
 * depth: device float[B][H][W]; xyz: device float[B][H][W][3].
 * Stream-ordered. */
b3d_status b3d_unproject(const float* depth, int32_t B, const b3d_intrinsics* K, float* xyz, void* stream);

/* Render N hypotheses of one mesh (Alg. 1, DepthRenderer; Sec. III-A (iii)).
 * A pixel is covered by a camera-facing triangle when its centre lies inside
 * or on the projected triangle; it keeps the nearest surface, equal depths
 * going to the smaller triangle id; its point is the intersection of its ray
 * with that triangle's plane.
 * poses: device float[N][16]; xyz_out: device float[N][H][W][3] (every
 * element written; empty = 0); tri_out: device int32[N][H][W] (empty = -1)
 * or NULL.  Stream-ordered. */
b3d_status b3d_render_batch(const b3d_mesh* mesh, const float* poses, int32_t N, const b3d_intrinsics* K,
                            float* xyz_out, int32_t* tri_out, void* stream);

/* Device workspace (bytes) of b3d_score and b3d_score_backward for an
 * H x W image: the observed image's valid pixels, listed once per call. */
b3d_status b3d_score_workspace_size(int32_t H, int32_t W, size_t* bytes);

/* Windowed robust likelihood (eq. (1) with the window of Sec. III-B).
 * observed: device float[H][W][3] (a pixel with z <= 0 holds no observation
 * and adds no term; every value must be finite); rendered: device
 * float[N][H][W][3] (z <= 0: empty);
 * logL_out: device float[N].  workspace: device memory of at least
 * b3d_score_workspace_size bytes, 16-byte aligned, owned by the caller
 * (contents undefined on return), or NULL: the same result from a kernel
 * that reads every observed pixel per hypothesis (slower).  A workspace
 * smaller than required is refused (B3D_ESHAPE) before any launch.
 * Stream-ordered. */
b3d_status b3d_score(const float* observed, const float* rendered, int32_t N, int32_t H, int32_t W,
                     const b3d_score_params* p, float* logL_out, void* workspace, size_t ws_bytes, void* stream);

/* Adjoint of b3d_score.  With a = p_out/V, b = (1-p_out)/M, K_ij =
 * N3(q~_i; q_j, sigma), D_ij = |q~_i - q_j|^2, S_i = sum_j K_ij and
 * L_i = a + b S_i, for each hypothesis n and upstream gradient g = dlogL[n]:
 *   d_rendered[n][j] = g sum_{i: j in W(i)} (b/L_i) K_ij (q~_i - q_j)/sigma^2
 *   d_sigma[n]       = g sum_i (b/L_i) sum_j K_ij (D_ij/sigma^3 - 3/sigma)
 *   d_pout[n]        = g sum_i (1/V - S_i/M)/L_i
 * dlogL: device float[N] or NULL (= all ones).  d_rendered: device
 * float[N][H][W][3] (every element written) or NULL; d_sigma, d_pout:
 * device float[N] or NULL.  workspace, ws_bytes: as for b3d_score.
 * Stream-ordered. */
b3d_status b3d_score_backward(const float* observed, const float* rendered, int32_t N, int32_t H, int32_t W,
                              const b3d_score_params* p, const float* dlogL, float* d_rendered, float* d_sigma,
                              float* d_pout, void* workspace, size_t ws_bytes, void* stream);

/* Pose adjoint of the render with visibility held fixed: the triangle of
 * each pixel (tri) is kept and its depth z = (n.c0)/(n.d) is differentiated
 * under the tangent update, giving dz/d(dt) = n/(n.d) and
 * dz/d(dw) = n x (t - q)/(n.d) with q = z d.  With g_j = d_rendered[j] . d_j:
 *   d_pose[n] = sum_j g_j (dz_j/d(dt), dz_j/d(dw))   (float[6] = dt, dw)
 * tri: device int32[N][H][W] from b3d_render_batch; d_rendered: device
 * float[N][H][W][3]; d_pose: device float[N][6] (overwritten).
 * Stream-ordered. */
b3d_status b3d_render_backward(const b3d_mesh* mesh, const float* poses, int32_t N, const b3d_intrinsics* K,
                               const int32_t* tri, const float* d_rendered, float* d_pose, void* stream);

/* ---- the fused path: render and score without point images in memory --- */

typedef struct b3d_scene b3d_scene;

/* A scene: the moving object's mesh, the camera, the likelihood parameters,
 * an optional static background (other objects at fixed poses) and the
 * observed point image.  The scene keeps `mesh` by reference (it must
 * outlive the scene).  Allocates device memory (not stream-ordered).
 * The fused kernel holds at least two image rows (plus 2h pixels each side)
 * of depth keys in LDS, which limits W to about 480 pixels with a 5x5 window
 * (B3D_ESHAPE beyond); rays must stay within |x/z|, |y/z| <= 1e3 over the
 * image and 2h pixels beyond it. */
b3d_status b3d_scene_create(const b3d_mesh* mesh, const b3d_intrinsics* K, const b3d_score_params* p,
                            b3d_scene** out);
b3d_status b3d_scene_destroy(b3d_scene* scene);

/* Static objects rendered once into the scene's background depth buffer;
 * the moving object is composited over it by nearest depth.  Background
 * triangle ids are numbered after the moving mesh's (object k's ids start at
 * T_moving + sum of earlier static triangle counts).  meshes: host array of
 * n handles; poses: host float[n][16].  n = 0 clears the background.
 * Stream-ordered; call b3d_scene_set_observed afterwards. */
b3d_status b3d_scene_set_background(b3d_scene* scene, const b3d_mesh* const* meshes, const float* poses, int32_t n,
                                    void* stream);

/* Point the scene at an observed image (device float[H][W][3], caller-owned,
 * read by later b3d_render_score calls; keep it alive and unchanged while
 * they run; pixels with z <= 0 hold no observation, every value finite) and
 * precompute the per-pixel terms of the background.  Call it
 * again whenever the image's contents or the background change.
 * Stream-ordered. */
b3d_status b3d_scene_set_observed(b3d_scene* scene, const float* observed, void* stream);

/* Fused render + windowed likelihood for N hypotheses of the scene's moving
 * object; equal (to FP32 rounding) to b3d_score over b3d_render_batch's point
 * images composited over the background.
 * poses: device float[N][16]; logL_out: device float[N].
 * grad_out: device float[N][8] or NULL; when given it receives
 *   (d logL_n/d dt [3], d logL_n/d dw [3], d logL_n/d sigma, d logL_n/d p_out)
 * with visibility held fixed (the adjoint of b3d_score_backward followed by
 * b3d_render_backward).  Results are bitwise repeatable and do not depend
 * on the tile size chosen by b3d_scene_autotune / b3d_scene_set_tile.
 * Stream-ordered. */
b3d_status b3d_render_score(const b3d_scene* scene, const float* poses, int32_t N, float* logL_out, float* grad_out,
                            void* stream);

/* Nodes of the midpoint rule for Alg. 1's uniform noise priors: the centres
 * of A equal cells of (0, sigma_max] (host float[A], sigma_max > 0) and of B
 * equal cells of (0, 1) (host float[B]).  With equal weights 1/(A B) they are
 * the grid whose marginal b3d_render_score_marginal computes (the prior
 * density 1/sigma_max times the cell volume sigma_max/(A B)).  Host only. */
b3d_status b3d_noise_midpoints(double sigma_max, int32_t A, int32_t B, float* sigma_out, float* p_out_out);

/* Hierarchical likelihood (Alg. 1's priors p_out ~ U(0, 1) and
 * sigma ~ U(0, sigma_max) on the noise parameters of eq. (1), and the
 * marginal over them used to compare hypotheses under unknown noise, Sec.
 * IV hierarchical Bayesian inference).  Sets a grid of A standard deviations
 * (host float[A], > 0) x B outlier probabilities (host float[B], in (0, 1]),
 * grid point k = a * B + b, with log quadrature weights log_w (host
 * float[A*B]; NULL: equal weights 1/(A*B), the midpoint rule for the uniform
 * priors when the values are cell centres).  The grid keeps the scene's
 * outlier volume, normaliser and window at the time of the call.
 * 1 <= A <= 8, A*B <= 16 (B3D_ESHAPE beyond).  Allocates device memory; when
 * an observed image is set, recomputes the background terms of every grid
 * point (stream-ordered), as b3d_scene_set_observed does from then on. */
b3d_status b3d_scene_set_noise_grid(b3d_scene* scene, const float* sigma, int32_t A, const float* p_out, int32_t B,
                                    const float* log_w, void* stream);

/* For each of N hypotheses: logL under every grid point (logL_grid, device
 * float[N][A*B], or NULL) and the log marginal
 * log sum_k w_k exp(logL_k) (logL_marg, device float[N]).  The same render
 * and windowed score as b3d_render_score, each pair's distance computed once
 * for all deviations.  Bitwise repeatable.  Stream-ordered. */
b3d_status b3d_render_score_marginal(const b3d_scene* scene, const float* poses, int32_t N, float* logL_grid,
                                     float* logL_marg, void* stream);

/* Tile-shape tuning of the fused kernel for this scene: times
 * b3d_render_score (with the adjoint when `grad`) on the given hypotheses for
 * each candidate size of the LDS depth buffer (the sizes that leave room for
 * 2..6 resident workgroups per CU, down to the smallest that still holds one
 * row band), keeps the fastest in the scene and returns its depth-buffer
 * capacity (keys) in *zcap_out (may be NULL).  Synchronises the device.
 * poses: device float[N][16], a representative sample (N >= 1). */
b3d_status b3d_scene_autotune(b3d_scene* scene, const float* poses, int32_t N, int32_t grad, int32_t* zcap_out,
                              void* stream);
/* The depth-buffer capacities (keys) b3d_scene_set_tile accepts for this
 * scene, and the current one.  Any pointer may be NULL. */
b3d_status b3d_scene_tile_limits(const b3d_scene* scene, int32_t* min_keys, int32_t* max_keys, int32_t* current);
/* Set the depth-buffer capacity directly (e.g. from a cached tuning result);
 * zcap <= 0 restores the default.  Fails with B3D_ESHAPE when it does not fit
 * the LDS or cannot hold one band of rows. */
b3d_status b3d_scene_set_tile(b3d_scene* scene, int32_t zcap);

/* b3d_render_score with the adjoint, from an instrumented build of the same
 * kernel that also adds the launch's work items to work (device uint64[8],
 * accumulated, zero it first): [0] vertices transformed, [1] triangles
 * tested, [2] triangles set up (facing the camera, box on screen),
 * [3] covered pixel centres, [4] (observed, rendered) window pairs,
 * [5] observed pixels whose window held a point, [6] object pixels of the
 * adjoint, [7] pixel centres decided by the exact double-precision test.
 * For measurement; slower than b3d_render_score.  Stream-ordered. */
b3d_status b3d_render_score_work(const b3d_scene* scene, const float* poses, int32_t N, float* logL_out,
                                 float* grad_out, unsigned long long* work, void* stream);

/* ---- many scenes in few launches ---------------------------------------- */

/* One scene's share of a batch: N hypotheses of the scene's moving object. */
typedef struct b3d_batch_item {
  const b3d_scene* scene; /* with its observed image set */
  const float* poses;     /* device float[N][16] */
  int32_t N;
  float* logL_out;        /* device float[N] */
  float* grad_out;        /* device float[N][8] or NULL; NULL for all items or for none */
} b3d_batch_item;

typedef struct b3d_batch b3d_batch;

/* Freeze a list of scenes and their hypothesis buffers into a launch plan:
 * scenes are ordered by estimated cost per hypothesis (largest first) and
 * grouped eight to a launch of one workgroup per hypothesis, so that the
 * launches keep the whole chip busy where one scene's hypotheses would not;
 * each scene's depth-buffer tile is capped at the default (four workgroups
 * per CU) so that one large tile does not lower every scene's occupancy.
 * The plan copies each scene's state (observed image pointer, background,
 * parameters, tile) at this call: re-create it after changing a scene.
 * Scenes of different image sizes, meshes and hypothesis counts may be
 * mixed.  Creates a stream and two events of its own when there is more
 * than one launch (not stream-ordered).  Results equal b3d_render_score per
 * scene, bit for bit. */
b3d_status b3d_batch_create(const b3d_batch_item* items, int32_t S, b3d_batch** out);
/* Run the plan: the launches in order, every other one on the batch's own
 * stream, forked from `stream` and joined back into it, so that one launch's
 * last workgroups overlap the next launch.  Stream-ordered with respect to
 * `stream`; graph-capture safe (the fork and join are event record/wait
 * pairs). */
b3d_status b3d_batch_run(const b3d_batch* batch, void* stream);
b3d_status b3d_batch_destroy(b3d_batch* batch);

/* ---- hypotheses, normalisation, sampling, coarse-to-fine --------------- */

/* A hypothesis grid around a centre pose (the cells of one stage of a
 * coarse-to-fine schedule, Sec. III-B).  Hypothesis
 *   n = r*(nx*ny*nz) + (ix*ny + iy)*nz + iz
 * has translation t_c + (ox[ix], oy[iy], oz[iz]) and rotation dR_r R_c.
 * Offsets along an axis of half-extent h with n samples are
 * linspace(-h, h, n) (cell_centres = 0; n = 1 gives 0) or the centres of n
 * equal cells of [-h, h] (cell_centres = 1, a partition).  Rotations:
 * rotations (device float[n_rot][9], row-major) if not NULL, else generated
 * perturbations: r = 0 is the identity, r >= 1 has its axis uniform on the
 * sphere and its angle uniform in [0, rot_max_angle], from Philox4x32-10
 * counter (r, stage, 0, 1) and key = seed. */
typedef struct b3d_grid {
  float center[16];
  float half_extent[3];
  int32_t count[3];
  int32_t cell_centres;
  int32_t n_rot;
  float rot_max_angle;
  const float* rotations;
} b3d_grid;

/* Number of hypotheses of a grid (0 if the grid is invalid). */
int64_t b3d_grid_size(const b3d_grid* g);

/* Expand a grid into poses: device float[b3d_grid_size(g)][16].
 * Stream-ordered. */
b3d_status b3d_enumerate(const b3d_grid* g, uint64_t seed, int32_t stage, float* poses_out, void* stream);

/* Normalise and sample (Sec. III-B: a cell is drawn with probability
 * proportional to its score).  logL holds P segments of N scores each
 * (device float[P][N]).  Within segment p, w_n = exp(logL_n - LSE) and draw
 * k (0 <= k < K) is argmax_n logL_n + G, G = -ln(-ln u), with u the odd
 * multiple of 2^-24 built from the top 23 bits of word 0 of Philox4x32-10 at
 * counter (n, k0 + p*K + k, stage, 0) and key = seed (low word first); ties
 * go to the lowest n.  weights_out: device float[P][N] or NULL; idx_out:
 * device int32[P][K]; logw_out: device float[P][K] (log weight of each draw)
 * or NULL.  1 <= K <= 4096.  Stream-ordered. */
b3d_status b3d_sample(const float* logL, int32_t P, int32_t N, int32_t K, uint64_t seed, uint32_t stage, uint32_t k0,
                      float* weights_out, int32_t* idx_out, float* logw_out, void* stream);

#define B3D_MAX_STAGES 8

/* A coarse-to-fine schedule: stage t enumerates stages[t] (its center is
 * ignored) around each particle's current pose. */
typedef struct b3d_schedule {
  int32_t n_stages;
  b3d_grid stages[B3D_MAX_STAGES];
} b3d_schedule;

/* Device workspace (bytes) that b3d_c2f_step needs for K particles. */
b3d_status b3d_c2f_workspace_size(const b3d_schedule* s, int32_t K, size_t* bytes);

/* Number of floats b3d_c2f_step writes to weights_out: N_0 + K (N_1 + ...
 * + N_{n_stages-1}), N_t the size of stages[t]'s grid. */
b3d_status b3d_c2f_weights_count(const b3d_schedule* s, int32_t K, int64_t* count);

/* One coarse-to-fine proposal for K particles (Sec. III-B and Fig. 1):
 * stage 0 scores stages[0] around `center` (host float[16]) once and draws
 * K cells; at each later stage t every particle k scores stages[t] around
 * its current pose and draws one cell (sampler counter (n, k, t, 0)), which
 * becomes its pose.  Each cell's probability is its normalised score,
 * softmax(logL) over the cells one draw chooses among (the scoring
 * strategy with one point per cell).
 * weights_out: device float[b3d_c2f_weights_count] or NULL: stage 0's N_0
 * cell probabilities, then for each later stage t the K particles' N_t
 * probabilities, particle-major ([K][N_t]), stages in order.
 * poses_out: device float[K][16] (the chosen cells' representative poses);
 * logq_out: device float[K], the sum over stages of the log probability of
 * each choice (for a partition schedule the proposal density of a uniform
 * draw in the final cell is exp(logq)/cell volume); idx_out: device
 * int32[n_stages][K] or NULL.  workspace: device memory of at least
 * b3d_c2f_workspace_size bytes, owned by the caller, contents undefined on
 * return.  Argument errors (NULL pointers, bad schedule or K, short
 * workspace, no observed image) return before any launch.  Stream-ordered. */
b3d_status b3d_c2f_step(const b3d_scene* scene, const float* center, const b3d_schedule* s, int32_t K, uint64_t seed,
                        void* workspace, size_t ws_bytes, float* weights_out, float* poses_out, float* logq_out,
                        int32_t* idx_out, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): b3d_c2f_step with
 * its workspace in a library-owned device array of B3D_C2F_SCRATCH_BYTES
 * (16 MiB) on each GPU it runs on, held until the process ends.  Same
 * arguments, results and errors as b3d_c2f_step without the workspace; a
 * schedule whose b3d_c2f_workspace_size exceeds the limit is refused with
 * B3D_ESHAPE before any launch (at 68 bytes per hypothesis, about 240,000
 * hypotheses in the largest stage: N_0, or K N_t for t >= 1).  Runs on the
 * current device; `stream` must belong to it.  Calls no allocating routine.
 * Every call on a device shares that device's array: calls that overlap on
 * one GPU (on different streams, or from several threads) race. */
#define B3D_C2F_SCRATCH_BYTES (16u << 20)
b3d_status b3d_c2f_step_noalloc(const b3d_scene* scene, const float* center, const b3d_schedule* s, int32_t K,
                                uint64_t seed, float* weights_out, float* poses_out, float* logq_out,
                                int32_t* idx_out, void* stream);

/* ---- gradient refinement and tracking ---------------------------------- */

/* Retraction onto the pose manifold, the update convention of the adjoint
 * (Sec. III-B's pose grid composed as t = t_c + dt, R = dR R_c, with dR the
 * rotation exponential): out[n] = (exp([w_n]x) R_b, t_b + dt_n) for
 * xi[n] = (dt_n, w_n), where b = n when n_base == N and b = 0 when
 * n_base == 1.  base: device float[n_base][16]; xi: device float[N][6];
 * out: device float[N][16] (may not alias base).  Stream-ordered. */
b3d_status b3d_pose_retract(const float* base, int32_t n_base, const float* xi, int32_t N, float* out, void* stream);

/* Adjoint of b3d_pose_retract composed with b3d_render_score's gradient:
 * grad[n] = b3d_render_score's grad_out at the retracted pose n, dlogL[n]
 * the incoming adjoint (device float[N], or NULL for all ones).
 * dxi[n] = dlogL[n] (g_t, J(w_n)^T g_w) with J the left Jacobian of the
 * rotation exponential.  dsp (device float[2] or NULL) receives
 * (sum_n dlogL[n] grad[n][6], sum_n dlogL[n] grad[n][7]): the gradients with
 * respect to a sigma and a p_out shared by all N hypotheses, summed in a
 * fixed order.  Stream-ordered. */
b3d_status b3d_pose_retract_backward(const float* xi, const float* grad, const float* dlogL, int32_t N, float* dxi,
                                     float* dsp, void* stream);

/* Change the likelihood parameters of a scene (sigma, p_out, outlier volume,
 * normaliser; the window size must stay the same, else B3D_ESHAPE) and, when
 * an observed image is set, recompute its background terms.  Stream-ordered
 * with respect to later calls on the same stream. */
b3d_status b3d_scene_set_params(b3d_scene* scene, const b3d_score_params* p, void* stream);

/* Adam ascent on logL over each pose's tangent (the refinement that follows
 * enumeration): with g = grad[n*gstride + 0..6) (d logL/d(dt, dw), e.g. from
 * b3d_render_score), m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * s = lr * (m/(1-b1^iter)) / (sqrt(v/(1-b2^iter)) + eps) with lr = lr_t for
 * dt and lr_r for dw, then t <- t + s_t, R <- exp([s_w]x) R.
 * poses: device float[N][16] (updated); grad: device, gstride floats per pose
 * (>= 6); state: device float[N][12] (m then v; zero it before iter 1).
 * iter >= 1.  Stream-ordered. */
b3d_status b3d_adam_pose_step(float* poses, const float* grad, int32_t gstride, float* state, int32_t N, int32_t iter,
                              float lr_t, float lr_r, float beta1, float beta2, float eps, void* stream);

/* Gradient refinement of N poses of a scene: n_refine Adam ascent steps on
 * logL each (the update of b3d_adam_pose_step from zero moments, driven by
 * b3d_render_score's adjoint), all steps of one pose in one workgroup.
 * poses: device float[N][16], updated in place.  Equal to n_refine rounds of
 * b3d_render_score(grad) + b3d_adam_pose_step.  Stream-ordered. */
b3d_status b3d_refine_poses(const b3d_scene* scene, float* poses, int32_t N, int32_t n_refine, float lr_t, float lr_r,
                            float beta1, float beta2, float eps, void* stream);

/* Per-frame tracking settings: n_stages grids of hypotheses, stage s centred
 * on the best hypothesis of stage s-1 (stage 0 on the previous estimate; the
 * grids' centers are ignored), then n_refine Adam steps on the best one.
 *
 * Occlusion handling (off when min_visible = 0), an addition to the method:
 * after an object's update, its seen fraction is the share of the pixels it
 * covers drawn alone at the new pose that lie in front of the other objects
 * at their current estimates and have a valid observed point within 3 sigma
 * of theirs among the window x window pixels around them.  Below min_visible
 * the update is dropped: the object moves instead by its last accepted
 * frame-to-frame motion (rotation R_new R_prev^T applied on the left,
 * translation t_new - t_prev added; none before the first accepted frame),
 * and the next frame's stage 0 searches translations widen times as far
 * (same count of cells).  An accepted update restores the plain grid. */
typedef struct b3d_track_params {
  int32_t n_stages; /* 1..B3D_MAX_STAGES */
  b3d_grid stages[B3D_MAX_STAGES];
  int32_t n_refine;
  float lr_t, lr_r, beta1, beta2, eps;
  float min_visible; /* 0..1; 0 turns the occlusion handling off */
  float widen;       /* >= 1: stage 0's translation half extents after a dropped update */
} b3d_track_params;

typedef struct b3d_tracker b3d_tracker;

/* Track M rigid objects through a sequence of observed images.  Each frame,
 * object by object: the other objects, at their latest estimates, are drawn
 * as static background; the grid of hypotheses around the object's previous
 * estimate is scored with the fused kernel, stage by stage around the best
 * of the previous stage (stage t enumerated as b3d_enumerate with seed 0 and
 * stage t; ties go to the lowest index); the best hypothesis is refined by
 * n_refine Adam
 * steps on the adjoint, each step's render, windows and adjoint spread over
 * row bands of the object's region (one workgroup per eight image rows) and
 * summed in band order.  The whole frame is captured once
 * into a HIP graph and replayed for every later frame, so a frame costs one
 * copy and one graph launch.  meshes: host array of M handles (they must
 * outlive the tracker); init_poses: host float[M][16].  1 <= M <= 16.
 * Allocates device memory (not stream-ordered). */
b3d_status b3d_tracker_create(const b3d_mesh* const* meshes, int32_t M, const b3d_intrinsics* K,
                              const b3d_score_params* p, const b3d_track_params* tp, const float* init_poses,
                              b3d_tracker** out);
/* Process one frame: observed is a device float[H][W][3] copied into the
 * tracker's own buffer before the graph runs.  Stream-ordered, except the
 * first call: it chooses the fused kernel's depth-buffer tile by running
 * this frame directly on `stream` once per candidate tile, timing each run
 * and restoring the estimates after it (no result depends on the tile), and
 * waits for `stream`; then it captures the graph on an internal stream and
 * launches it on `stream`. */
b3d_status b3d_tracker_frame(b3d_tracker* tr, const float* observed, void* stream);
/* The same frame run directly on `stream`, without the graph (reference
 * for the captured path).  Stream-ordered. */
b3d_status b3d_tracker_frame_eager(b3d_tracker* tr, const float* observed, void* stream);
/* Current estimates: device float[M][16].  Stream-ordered copy. */
b3d_status b3d_tracker_poses(const b3d_tracker* tr, float* poses_out, void* stream);
/* Occlusion state after the last frame, per object: state_out device
 * float[M][3] = (seen fraction of the last update, frames in a row whose
 * update was dropped, stage 0's translation scale for the next frame);
 * (0, 0, 1) until a frame has run with min_visible > 0.  Stream-ordered copy. */
b3d_status b3d_tracker_state(const b3d_tracker* tr, float* state_out, void* stream);
b3d_status b3d_tracker_destroy(b3d_tracker* tr);

/* ---- table scenes: contact placement and SMC over the objects ---------- */

/* The table, root of the scene graph (Alg. 1): pose maps the table frame to
 * the camera frame (row-major); the table top is the plane z = 0 of that
 * frame, +z up, a width x height rectangle (width along x) centred on the
 * frame's origin. */
typedef struct b3d_table {
  float pose[16];
  float width, height;
} b3d_table;

/* A type library on a table, for placing objects by contact: each type's six
 * resting faces (the faces of the axis-aligned bounding box of its vertices
 * in its own frame) and their placement prior, uploaded to the device once.
 * types: host array of n_types mesh handles (1..B3D_MAX_TYPES; the meshes
 * only need to live during the call).  Allocates device memory. */
typedef struct b3d_contact b3d_contact;
b3d_status b3d_contact_create(const b3d_mesh* const* types, int32_t n_types, const b3d_table* table,
                              b3d_contact** out);
b3d_status b3d_contact_destroy(b3d_contact* contact);

/* Object poses from contact placements (Alg. 1's type, contact face and
 * relative pose; Sec. III-A (i)).  Object k of type place[k][0] rests on face
 * c = place[k][1] of the axis-aligned bounding box of its vertices in its
 * own frame (c = 0..5: -x, +x, -y, +y, -z, +z): R_c turns the face's outward
 * normal to -z and d_c puts the face on z = 0 with the face's centre on the
 * origin; then
 *   pose = table.pose * [Rz(dth) R_c | Rz(dth) d_c + (dx, dy, 0)]
 * with (dx, dy, dth) = dphi[k].  place: device int32[N][2]; dphi: device
 * float[N][3]; poses_out: device float[N][16].  The kernel clamps a type or
 * face outside its range to the nearest valid one (no error is reported).
 * Allocates nothing and copies nothing from the host.  Stream-ordered. */
b3d_status b3d_contact_poses(const b3d_contact* contact, const int32_t* place, const float* dphi, int32_t N,
                             float* poses_out, void* stream);

#define B3D_MAX_SMC_OBJECTS 8
#define B3D_MAX_TYPES 16

/* Sequential Monte Carlo over the objects of a table scene (Sec. III-B,
 * eq. (2)-(3)).  Stage i places object i in every particle:
 *  1. coarse-to-fine search over cells of (type, face, dx, dy, dth): stage 0
 *     splits every (type, face) placement box -- dx, dy over the table less
 *     the face's footprint, dth over [0, 2 pi) -- into counts[0] cells
 *     (ix * ny + iy) * nth + ith, stage t splits the chosen cell into
 *     counts[t]; every cell is scored by the fused kernel at its centre, with
 *     the fixed content and the particle's earlier objects as background and
 *     the stage's noise (stage_sigma[t], stage_p_out[t]) or, where that is
 *     0, the particle's current noise, and one is drawn by softmax (b3d_sample,
 *     stage word (i << 8) | t, draw = particle); a uniform point of the final
 *     cell (Philox4x32-10 counter (m, i, 0, 2), words 0..2) is the placement;
 *  2. the noise: A x B equal cells of (0, sigma_max] x (0, 1) scored at their
 *     midpoints over the whole image, one drawn (stage word (i << 8) | 0x40),
 *     a uniform point of it taken (counter (m, i, 1, 2), words 0, 1);
 *  3. log q = sum of the draws' log probabilities - log(final cell volume)
 *     - log(noise cell area); log p_i = logL of the scene at the new noise
 *     + the objects' log priors (1/|O| 1/6 1/((W_t - w)(H_t - h)) 1/(2 pi)
 *     each) - log sigma_max; log W += log p_i - log p_{i-1} - log q, plus
 *     -log sigma_max from stage 2 on (the noise prior as the density of the
 *     noise values that the stage replaces);
 *  4. when the effective sample size is below ess_threshold * M, multinomial
 *     resampling by Gumbel-max over the log weights (stage word
 *     (i << 8) | 0x80, draw = particle) and every log weight set to the log
 *     mean weight. */
typedef struct b3d_smc_params {
  int32_t n_particles;               /* M, 1..1024 */
  int32_t n_objects;                 /* objects to place, 1..B3D_MAX_SMC_OBJECTS */
  int32_t n_stages;                  /* coarse-to-fine stages per object, 1..B3D_MAX_STAGES */
  int32_t counts[B3D_MAX_STAGES][3]; /* cells per axis (dx, dy, dth) of each stage's split */
  float sigma_max;                   /* the prior sigma ~ U(0, sigma_max) */
  int32_t noise_A, noise_B;          /* noise cells along sigma and p_out: A <= 8, A * B <= 16 */
  float sigma0, p_out0;              /* noise used while placing the first object */
  float ess_threshold;               /* resample when ESS < ess_threshold * M (0: never, > 1: always) */
  float outlier_volume;              /* V of eq. (1) */
  int32_t window;                    /* odd window side */
  float norm_M;                      /* eq. (1)'s normaliser; 0 for H * W */
  uint64_t seed;
  /* the noise at which placement stage t scores its cells (sigma, p_out);
   * stage_sigma[t] = 0 uses each particle's current estimates */
  float stage_sigma[B3D_MAX_STAGES];
  float stage_p_out[B3D_MAX_STAGES];
} b3d_smc_params;

typedef struct b3d_smc b3d_smc;

/* types: host array of n_types (1..B3D_MAX_TYPES) mesh handles, the object
 * library; fixed, fixed_poses (host float[n_fixed][16]): content drawn in
 * every hypothesis's background (the table's own mesh, for instance).  Mesh
 * handles must outlive the sampler.  Every face footprint must be smaller
 * than the table (B3D_ESHAPE).  Allocates device memory (not
 * stream-ordered). */
b3d_status b3d_smc_create(const b3d_mesh* const* types, int32_t n_types, const b3d_mesh* const* fixed,
                          const float* fixed_poses, int32_t n_fixed, const b3d_table* table, const b3d_intrinsics* K,
                          const b3d_smc_params* p, b3d_smc** out);
/* Start over on an observed image (device float[H][W][3], read by pointer
 * until the next reset): no objects, log weights 0, noise (sigma0, p_out0).
 * Stream-ordered. */
b3d_status b3d_smc_reset(b3d_smc* smc, const float* observed, void* stream);
/* One SMC stage: place the next object in every particle.  B3D_ESHAPE once
 * n_objects are placed.  Synchronises `stream` a few times (the host reads
 * the particles' noise and chosen types to set up the next launches).  The
 * first step of a sampler also times the fused kernel's depth-buffer tile
 * (b3d_scene_autotune on the largest type's stage-0 cells) for all its
 * scenes; results do not depend on the tile. */
b3d_status b3d_smc_step(b3d_smc* smc, void* stream);

/* Where b3d_smc_read copies the particles and the last stage's diagnostics
 * (device buffers; NULL skips a field).  M = n_particles, n = n_objects. */
typedef struct b3d_smc_view {
  int32_t* place;     /* [M][n][2] type, face of the objects placed so far */
  float* dphi;        /* [M][n][3] */
  float* poses;       /* [M][n][16] camera-frame poses */
  float* noise;       /* [M][2] sigma, p_out */
  double* logW;       /* [M] */
  double* logp;       /* [M] log target at the particle */
  float* logL;        /* [M] logL of the particle's scene at its noise */
  /* the last stage, per proposal (before resampling) */
  int32_t* choice;    /* [n_stages][M] cell drawn at each coarse-to-fine stage */
  double* logq;       /* [M] */
  double* logW_pre;   /* [M] */
  float* noise_grid;  /* [M][A * B] logL at the noise cells' midpoints */
  int32_t* ancestors; /* [M] particle each survivor copies (identity without resampling) */
  double* ess;        /* [1] */
  float* type_post;   /* [M][n_types] posterior over the new object's type from the stage-0 cells: the softmax
                         mass of each type's cells, marginal over face and placement */
} b3d_smc_view;

/* n_placed (host, may be NULL): objects placed so far; n_scored (host, may
 * be NULL): placement hypotheses rendered and scored since the reset
 * (particles with equal noise and equal objects -- all of them before the
 * first object, and the copies made by resampling -- share one scoring of
 * the stage-0 cells).  Unplaced slots read as zeros.  Stream-ordered. */
b3d_status b3d_smc_read(const b3d_smc* smc, const b3d_smc_view* view, int32_t* n_placed, int64_t* n_scored,
                        void* stream);
b3d_status b3d_smc_destroy(b3d_smc* smc);

#ifdef __cplusplus
}
#endif

#endif /* B3D_H */

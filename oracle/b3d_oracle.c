/*
 * FP64 CPU oracle for the batched render-and-score path of Bayes3D
 * (arXiv 2312.08715).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain statement of what
 * the GPU library computes, written from the paper and used to check it.  It
 * shares no code, header, table or helper with the GPU library.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.
 *
 * Everything is double precision.  Where the paper is silent, the readings
 * below are used (they are also listed in the design notes):
 *   - camera frame: +z forward, +x right, +y down; pose = 4x4 row-major
 *     object-to-camera transform; pixel (r, c) has its centre at
 *     (c + 1/2, r + 1/2) and its ray is d = ((c+1/2-cx)/fx, (r+1/2-cy)/fy, 1);
 *     depth is camera z, not range.
 *   - renderer (the depth buffer of Alg. 1, DepthRenderer call, and the point
 *     cloud conversion of Sec. III-A (iii)): a triangle with any vertex at
 *     z <= z_near is dropped; a triangle is kept iff it faces the camera,
 *     ((c1-c0) x (c2-c0)) . c0 < 0; a pixel is covered iff its centre lies
 *     inside or on the projected triangle; the surface point is the
 *     intersection of the ray with the triangle's plane; the pixel keeps the
 *     smallest depth, equal depths going to the smallest triangle id.
 *   - likelihood, eq. (1) with the window truncation of Sec. III-B (scoring
 *     strategy): for hypothesis n
 *        l_i = ln( p_out/V + (1-p_out)/M * sum_{j in W(i), z_j>0} N3(q~_i; q_j, sigma) )
 *        logL_n = sum over observed pixels i with z~_i > 0 of l_i
 *     with N3 the isotropic 3-D Gaussian density of standard deviation sigma,
 *     W(i) the r x r square window centred on i clipped to the image, M the
 *     normaliser |y| (the pixel count H*W unless given).  The sigma/sigma_max
 *     prefactor of eq. (1) is constant across hypotheses and left out.
 *   - sampling (Sec. III-B, the next region is drawn with probability
 *     proportional to its score): categorical draws by Gumbel-max with
 *     uniforms from Philox4x32-10 (Salmon et al., SC'11).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Per-hypothesis work counters (algorithmic work of the plain method). */
enum {
  ORC_C_VERT = 0,   /* vertices transformed */
  ORC_C_TRI,        /* triangles tested */
  ORC_C_FRONT,      /* triangles kept (in front of z_near and facing the camera) */
  ORC_C_FRAG,       /* covered pixel centres, before the depth test */
  ORC_C_PAIR,       /* (observed, rendered) pairs with both valid inside a window */
  ORC_C_OBS,        /* valid observed pixels */
  ORC_C_OBS_ACTIVE, /* valid observed pixels with at least one valid rendered pixel in the window */
  ORC_C_RPIX,       /* valid rendered pixels */
  ORC_NC
};

int orc_num_counters(void) { return ORC_NC; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads used by the OpenMP loops from now on (n >= 1). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

static void xform(const double* P, const double* v, double* c) {
  c[0] = P[0] * v[0] + P[1] * v[1] + P[2] * v[2] + P[3];
  c[1] = P[4] * v[0] + P[5] * v[1] + P[6] * v[2] + P[7];
  c[2] = P[8] * v[0] + P[9] * v[1] + P[10] * v[2] + P[11];
}

static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* cam = {fx, fy, cx, cy, z_near} */
static void pixel_ray(const double* cam, int r, int c, double* d) {
  d[0] = ((double)c + 0.5 - cam[2]) / cam[0];
  d[1] = ((double)r + 0.5 - cam[3]) / cam[1];
  d[2] = 1.0;
}

/*
 * Render one mesh under N poses into depth/id images.  depth [N,H,W] and
 * ids [N,H,W] are read and updated, so several meshes can be composited by
 * calling this once per mesh with distinct id_offset (an empty pixel has
 * depth 0 and id -1).  The triangle id written is id_offset + row index.
 * counters [N, ORC_NC] (may be NULL) receive VERT, TRI, FRONT and FRAG.
 */
int orc_render(const double* verts, int V, const int* tris, int T, int id_offset, const double* poses, int N,
               const double* cam, int H, int W, double* depth, int* ids, long long* counters) {
  if (V < 0 || T < 0 || N < 0 || H <= 0 || W <= 0) return -1;
  const double fx = cam[0], fy = cam[1], cx = cam[2], cy = cam[3], znear = cam[4];
#pragma omp parallel
  {
    double* c = (double*)malloc(sizeof(double) * 3 * (size_t)(V > 0 ? V : 1));
#pragma omp for schedule(static)
    for (int n = 0; n < N; ++n) {
      const double* P = poses + 16 * (size_t)n;
      double* dz = depth + (size_t)n * H * W;
      int* di = ids + (size_t)n * H * W;
      long long cnt_front = 0, cnt_frag = 0;
      for (int k = 0; k < V; ++k) xform(P, verts + 3 * (size_t)k, c + 3 * (size_t)k);
      for (int i = 0; i < T; ++i) {
        const double* c0 = c + 3 * (size_t)tris[3 * i + 0];
        const double* c1 = c + 3 * (size_t)tris[3 * i + 1];
        const double* c2 = c + 3 * (size_t)tris[3 * i + 2];
        if (c0[2] <= znear || c1[2] <= znear || c2[2] <= znear) continue;
        double e1[3] = {c1[0] - c0[0], c1[1] - c0[1], c1[2] - c0[2]};
        double e2[3] = {c2[0] - c0[0], c2[1] - c0[1], c2[2] - c0[2]};
        double nn[3];
        cross3(e1, e2, nn);
        const double nc0 = dot3(nn, c0);
        if (!(nc0 < 0.0)) continue; /* back-facing or edge-on */
        ++cnt_front;
        const double u0 = fx * c0[0] / c0[2] + cx, v0 = fy * c0[1] / c0[2] + cy;
        const double u1 = fx * c1[0] / c1[2] + cx, v1 = fy * c1[1] / c1[2] + cy;
        const double u2 = fx * c2[0] / c2[2] + cx, v2 = fy * c2[1] / c2[2] + cy;
        double umin = fmin(u0, fmin(u1, u2)), umax = fmax(u0, fmax(u1, u2));
        double vmin = fmin(v0, fmin(v1, v2)), vmax = fmax(v0, fmax(v1, v2));
        /* pixel centres c + 1/2 inside [umin, umax] */
        double clo = ceil(umin - 0.5), chi = floor(umax - 0.5);
        double rlo = ceil(vmin - 0.5), rhi = floor(vmax - 0.5);
        if (clo < 0) clo = 0;
        if (rlo < 0) rlo = 0;
        if (chi > W - 1) chi = W - 1;
        if (rhi > H - 1) rhi = H - 1;
        for (int r = (int)rlo; r <= (int)rhi; ++r) {
          const double py = r + 0.5;
          for (int col = (int)clo; col <= (int)chi; ++col) {
            const double px = col + 0.5;
            /* Each edge function equals the projected signed area at the
             * opposite vertex, which is negative for a front-facing
             * triangle; the centre is covered iff none is positive. */
            const double w0 = (u2 - u1) * (py - v1) - (v2 - v1) * (px - u1);
            const double w1 = (u0 - u2) * (py - v2) - (v0 - v2) * (px - u2);
            const double w2 = (u1 - u0) * (py - v0) - (v1 - v0) * (px - u0);
            if (w0 > 0.0 || w1 > 0.0 || w2 > 0.0) continue;
            ++cnt_frag;
            double d[3];
            pixel_ray(cam, r, col, d);
            const double z = nc0 / dot3(nn, d);
            const int id = id_offset + i;
            const size_t p = (size_t)r * W + col;
            if (dz[p] <= 0.0 || z < dz[p] || (z == dz[p] && id < di[p])) {
              dz[p] = z;
              di[p] = id;
            }
          }
        }
      }
      if (counters) {
        long long* cn = counters + (size_t)n * ORC_NC;
        cn[ORC_C_VERT] += V;
        cn[ORC_C_TRI] += T;
        cn[ORC_C_FRONT] += cnt_front;
        cn[ORC_C_FRAG] += cnt_frag;
      }
    }
    free(c);
  }
  return 0;
}

/*
 * Depth of each pixel on the plane of a given triangle ("frozen
 * visibility"): for every pixel whose base id lies in
 * [id_offset, id_offset + T), depth = ray/plane intersection of that
 * triangle at the given pose.  Other pixels are left untouched.  Used for
 * finite differences of the pose adjoint, where visibility is held fixed.
 */
int orc_render_frozen(const double* verts, int V, const int* tris, int T, int id_offset, const double* poses, int N,
                      const double* cam, int H, int W, const int* base_ids, double* depth) {
  (void)V;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double* P = poses + 16 * (size_t)n;
    for (int r = 0; r < H; ++r)
      for (int col = 0; col < W; ++col) {
        const size_t p = (size_t)n * H * W + (size_t)r * W + col;
        const int id = base_ids[p] - id_offset;
        if (id < 0 || id >= T) continue;
        double c0[3], c1[3], c2[3], e1[3], e2[3], nn[3], d[3];
        xform(P, verts + 3 * (size_t)tris[3 * id + 0], c0);
        xform(P, verts + 3 * (size_t)tris[3 * id + 1], c1);
        xform(P, verts + 3 * (size_t)tris[3 * id + 2], c2);
        for (int k = 0; k < 3; ++k) {
          e1[k] = c1[k] - c0[k];
          e2[k] = c2[k] - c0[k];
        }
        cross3(e1, e2, nn);
        pixel_ray(cam, r, col, d);
        depth[p] = dot3(nn, c0) / dot3(nn, d);
      }
  }
  return 0;
}

/* Point image from a depth image: q = z d (Sec. III-A (iii)); empty pixels -> 0. */
int orc_unproject(const double* depth, int B, const double* cam, int H, int W, double* xyz) {
  for (int b = 0; b < B; ++b)
    for (int r = 0; r < H; ++r)
      for (int col = 0; col < W; ++col) {
        const size_t p = (size_t)b * H * W + (size_t)r * W + col;
        double d[3];
        pixel_ray(cam, r, col, d);
        const double z = depth[p] > 0.0 ? depth[p] : 0.0;
        xyz[3 * p + 0] = z * d[0];
        xyz[3 * p + 1] = z * d[1];
        xyz[3 * p + 2] = z * d[2];
      }
  return 0;
}

/*
 * Windowed robust likelihood, eq. (1) truncated to an r x r window.
 * obs [H,W,3] (valid iff z > 0), rend [N,H,W,3] (valid iff z > 0).
 * logL [N]; l1 [N] (may be NULL) = sum |l_i|; counters (may be NULL) receive
 * PAIR, OBS, OBS_ACTIVE and RPIX.  M <= 0 means H*W.
 */
int orc_score(const double* obs, const double* rend, int N, int H, int W, double sigma, double p_out, double V,
              double M, int r, double* logL, double* l1, long long* counters) {
  if (r < 1 || (r % 2) == 0 || sigma <= 0.0 || V <= 0.0) return -1;
  if (M <= 0.0) M = (double)H * (double)W;
  const int h = (r - 1) / 2;
  const double a = p_out / V, b = (1.0 - p_out) / M;
  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double* q = rend + (size_t)n * H * W * 3;
    double acc = 0.0, accabs = 0.0;
    long long pairs = 0, nobs = 0, nact = 0, nrp = 0;
    for (int p = 0; p < H * W; ++p)
      if (q[3 * (size_t)p + 2] > 0.0) ++nrp;
    for (int ri = 0; ri < H; ++ri)
      for (int ci = 0; ci < W; ++ci) {
        const double* qt = obs + 3 * ((size_t)ri * W + ci);
        if (!(qt[2] > 0.0)) continue;
        ++nobs;
        double S = 0.0;
        long long np = 0;
        const int r0 = ri - h < 0 ? 0 : ri - h, r1 = ri + h > H - 1 ? H - 1 : ri + h;
        const int c0 = ci - h < 0 ? 0 : ci - h, c1 = ci + h > W - 1 ? W - 1 : ci + h;
        for (int rj = r0; rj <= r1; ++rj)
          for (int cj = c0; cj <= c1; ++cj) {
            const double* qj = q + 3 * ((size_t)rj * W + cj);
            if (!(qj[2] > 0.0)) continue;
            const double dx = qt[0] - qj[0], dy = qt[1] - qj[1], dzv = qt[2] - qj[2];
            S += norm * exp(-(dx * dx + dy * dy + dzv * dzv) * inv2s2);
            ++np;
          }
        if (np) ++nact;
        pairs += np;
        const double li = log(a + b * S);
        acc += li;
        accabs += fabs(li);
      }
    logL[n] = acc;
    if (l1) l1[n] = accabs;
    if (counters) {
      long long* cn = counters + (size_t)n * ORC_NC;
      cn[ORC_C_PAIR] += pairs;
      cn[ORC_C_OBS] += nobs;
      cn[ORC_C_OBS_ACTIVE] += nact;
      cn[ORC_C_RPIX] += nrp;
    }
  }
  return 0;
}

/*
 * Adjoint of the windowed likelihood.  With a = p_out/V, b = (1-p_out)/M,
 * K_ij = N3(q~_i; q_j, sigma), D_ij = |q~_i - q_j|^2, S_i = sum_j K_ij and
 * L_i = a + b S_i:
 *   d logL / d p_out = sum_i (1/V - S_i/M) / L_i
 *   d logL / d sigma = sum_i (b/L_i) sum_j K_ij (D_ij/sigma^3 - 3/sigma)
 *   d logL / d q_j   = sum_{i: j in W(i)} (b/L_i) K_ij (q~_i - q_j) / sigma^2
 * Each is scaled by dlogL[n] (NULL means 1).  d_rend [N,H,W,3] is
 * overwritten when not NULL.
 */
int orc_score_grad(const double* obs, const double* rend, int N, int H, int W, double sigma, double p_out, double V,
                   double M, int r, const double* dlogL, double* d_rend, double* d_sigma, double* d_pout) {
  if (r < 1 || (r % 2) == 0 || sigma <= 0.0 || V <= 0.0) return -1;
  if (M <= 0.0) M = (double)H * (double)W;
  const int h = (r - 1) / 2;
  const double a = p_out / V, b = (1.0 - p_out) / M;
  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);
  const double s2 = sigma * sigma, inv2s2 = 1.0 / (2.0 * s2);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double g = dlogL ? dlogL[n] : 1.0;
    const double* q = rend + (size_t)n * H * W * 3;
    double* dq = d_rend ? d_rend + (size_t)n * H * W * 3 : NULL;
    if (dq) memset(dq, 0, sizeof(double) * 3 * (size_t)H * W);
    double dp = 0.0, ds = 0.0;
    for (int ri = 0; ri < H; ++ri)
      for (int ci = 0; ci < W; ++ci) {
        const double* qt = obs + 3 * ((size_t)ri * W + ci);
        if (!(qt[2] > 0.0)) continue;
        const int r0 = ri - h < 0 ? 0 : ri - h, r1 = ri + h > H - 1 ? H - 1 : ri + h;
        const int c0 = ci - h < 0 ? 0 : ci - h, c1 = ci + h > W - 1 ? W - 1 : ci + h;
        double S = 0.0, TD = 0.0;
        for (int rj = r0; rj <= r1; ++rj)
          for (int cj = c0; cj <= c1; ++cj) {
            const double* qj = q + 3 * ((size_t)rj * W + cj);
            if (!(qj[2] > 0.0)) continue;
            const double dx = qt[0] - qj[0], dy = qt[1] - qj[1], dzv = qt[2] - qj[2];
            const double D = dx * dx + dy * dy + dzv * dzv;
            const double K = norm * exp(-D * inv2s2);
            S += K;
            TD += K * D;
          }
        const double L = a + b * S;
        dp += (1.0 / V - S / M) / L;
        ds += (b / L) * (TD / (s2 * sigma) - 3.0 * S / sigma);
        if (dq) {
          for (int rj = r0; rj <= r1; ++rj)
            for (int cj = c0; cj <= c1; ++cj) {
              const size_t pj = (size_t)rj * W + cj;
              const double* qj = q + 3 * pj;
              if (!(qj[2] > 0.0)) continue;
              const double dx = qt[0] - qj[0], dy = qt[1] - qj[1], dzv = qt[2] - qj[2];
              const double K = norm * exp(-(dx * dx + dy * dy + dzv * dzv) * inv2s2);
              const double coef = g * (b / L) * K / s2;
              dq[3 * pj + 0] += coef * dx;
              dq[3 * pj + 1] += coef * dy;
              dq[3 * pj + 2] += coef * dzv;
            }
        }
      }
    if (d_sigma) d_sigma[n] = g * ds;
    if (d_pout) d_pout[n] = g * dp;
  }
  return 0;
}

/*
 * Pose adjoint of the render with visibility held fixed.  A pose update is
 * R <- exp([dw]x) R, t <- t + dt, which moves an object point c (camera
 * frame) to c + dt + dw x (c - t) and its normal n to n + dw x n.  The depth
 * of pixel j on the plane of its triangle, z = (n.c0)/(n.d), then has
 *   dz/d(dt) = n / (n.d),   dz/d(dw) = n x (t - q) / (n.d),   q = z d.
 * With g_j = d_rend_j . d_j, d_pose[n] = sum_j g_j (dz/d(dt), dz/d(dw)),
 * accumulated into d_pose [N,6] = (dt, dw) for pixels whose id is in
 * [id_offset, id_offset + T).
 */
int orc_render_grad(const double* verts, int V, const int* tris, int T, int id_offset, const double* poses, int N,
                    const double* cam, int H, int W, const int* ids, const double* depth, const double* d_rend,
                    double* d_pose) {
  (void)V;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double* P = poses + 16 * (size_t)n;
    const double t[3] = {P[3], P[7], P[11]};
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < H; ++r)
      for (int col = 0; col < W; ++col) {
        const size_t p = (size_t)n * H * W + (size_t)r * W + col;
        const int id = ids[p] - id_offset;
        if (id < 0 || id >= T) continue;
        double c0[3], c1[3], c2[3], e1[3], e2[3], nn[3], d[3], q[3], tq[3], w[3];
        xform(P, verts + 3 * (size_t)tris[3 * id + 0], c0);
        xform(P, verts + 3 * (size_t)tris[3 * id + 1], c1);
        xform(P, verts + 3 * (size_t)tris[3 * id + 2], c2);
        for (int k = 0; k < 3; ++k) {
          e1[k] = c1[k] - c0[k];
          e2[k] = c2[k] - c0[k];
        }
        cross3(e1, e2, nn);
        pixel_ray(cam, r, col, d);
        const double z = depth[p];
        for (int k = 0; k < 3; ++k) {
          q[k] = z * d[k];
          tq[k] = t[k] - q[k];
        }
        const double nd = dot3(nn, d);
        const double gj = dot3(d_rend + 3 * p, d);
        cross3(nn, tq, w);
        for (int k = 0; k < 3; ++k) {
          acc[k] += gj * nn[k] / nd;
          acc[3 + k] += gj * w[k] / nd;
        }
      }
    for (int k = 0; k < 6; ++k) d_pose[6 * (size_t)n + k] += acc[k];
  }
  return 0;
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---------------- */

static void philox_round(uint32_t* x, const uint32_t* k) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t y0 = hi1 ^ x[1] ^ k[0];
  const uint32_t y2 = hi0 ^ x[3] ^ k[1];
  x[0] = y0;
  x[1] = lo1;
  x[2] = y2;
  x[3] = lo0;
}

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(x, k);
  }
  memcpy(out, x, sizeof(x));
}

/* Odd multiple of 2^-24 from the top 23 bits: exact in binary32, in (0, 1). */
static double unit_uniform(uint32_t x) { return (double)(2u * (x >> 9) + 1u) * 0x1p-24; }

double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int word) {
  const uint32_t ctr[4] = {c0, c1, c2, c3};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return unit_uniform(out[word & 3]);
}

/*
 * Normalise and sample: w_n = exp(logL_n - logsumexp(logL)); draw k (k in
 * [0,K)) is argmax_n logL_n + G_kn with G = -ln(-ln u) and u from counter
 * (n, k0 + k, stage, 0); ties go to the lowest n.  logw[k] = logL_idx - lse.
 */
int orc_sample(const double* logL, int N, int K, uint64_t seed, uint32_t stage, uint32_t k0, double* w, int* idx,
               double* logw) {
  if (N <= 0) return -1;
  double m = -INFINITY;
  for (int n = 0; n < N; ++n) m = logL[n] > m ? logL[n] : m;
  double s = 0.0;
  for (int n = 0; n < N; ++n) s += exp(logL[n] - m);
  const double lse = m + log(s);
  if (w)
    for (int n = 0; n < N; ++n) w[n] = exp(logL[n] - lse);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < K; ++k) {
    double best = -INFINITY;
    int bi = -1;
    for (int n = 0; n < N; ++n) {
      const double u = orc_uniform(seed, (uint32_t)n, k0 + (uint32_t)k, stage, 0u, 0);
      const double v = logL[n] - log(-log(u));
      if (bi < 0 || v > best) {
        best = v;
        bi = n;
      }
    }
    idx[k] = bi;
    if (logw) logw[k] = logL[bi] - lse;
  }
  return 0;
}

/* Rotation by angle th about the unit axis k: I + sin(th) [k]x + (1-cos th) [k]x^2. */
static void axis_angle(const double* k, double th, double* R) {
  const double s = sin(th), c = 1.0 - cos(th);
  const double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double kk = 0.0;
      for (int l = 0; l < 3; ++l) kk += K[3 * i + l] * K[3 * l + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + s * K[3 * i + j] + c * kk;
    }
}

/*
 * Delta rotation r of a generated perturbation set: r = 0 is the identity;
 * otherwise the axis is uniform on the sphere and the angle uniform in
 * [0, max_angle], from counter (r, stage, 0, 1).
 */
void orc_perturbation(uint64_t seed, uint32_t stage, int r, double max_angle, double* R) {
  if (r == 0) {
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    return;
  }
  const double u0 = orc_uniform(seed, (uint32_t)r, stage, 0u, 1u, 0);
  const double u1 = orc_uniform(seed, (uint32_t)r, stage, 0u, 1u, 1);
  const double u2 = orc_uniform(seed, (uint32_t)r, stage, 0u, 1u, 2);
  const double z = 1.0 - 2.0 * u0, ph = 2.0 * M_PI * u1;
  const double s = sqrt(fmax(0.0, 1.0 - z * z));
  const double k[3] = {s * cos(ph), s * sin(ph), z};
  axis_angle(k, max_angle * u2, R);
}

static double grid_offset(int i, int n, double h, int cell_centres) {
  if (n <= 1) return 0.0;
  if (cell_centres) return -h + (2.0 * i + 1.0) * h / n;
  return -h + 2.0 * h * i / (n - 1);
}

/*
 * Expand a hypothesis grid around a centre pose into poses [N,16]:
 * n = r*(nx*ny*nz) + (ix*ny + iy)*nz + iz, t = t_c + (dx, dy, dz),
 * R = dR_r R_c.  rots [n_rot, 9] gives explicit delta rotations; when NULL
 * they are generated perturbations (orc_perturbation).
 */
int orc_enumerate(const double* center, const double* half, const int* count, int cell_centres, const double* rots,
                  int n_rot, double rot_max_angle, uint64_t seed, uint32_t stage, double* poses) {
  const int nx = count[0], ny = count[1], nz = count[2];
  if (nx <= 0 || ny <= 0 || nz <= 0 || n_rot <= 0) return -1;
  const int nt = nx * ny * nz;
  for (int r = 0; r < n_rot; ++r) {
    double dR[9], R[9];
    if (rots)
      memcpy(dR, rots + 9 * (size_t)r, sizeof(dR));
    else
      orc_perturbation(seed, stage, r, rot_max_angle, dR);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l) s += dR[3 * i + l] * center[4 * l + j];
        R[3 * i + j] = s;
      }
    for (int ix = 0; ix < nx; ++ix)
      for (int iy = 0; iy < ny; ++iy)
        for (int iz = 0; iz < nz; ++iz) {
          double* P = poses + 16 * ((size_t)r * nt + (size_t)(ix * ny + iy) * nz + iz);
          const double off[3] = {grid_offset(ix, nx, half[0], cell_centres), grid_offset(iy, ny, half[1], cell_centres),
                                 grid_offset(iz, nz, half[2], cell_centres)};
          for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) P[4 * i + j] = R[3 * i + j];
            P[4 * i + 3] = center[4 * i + 3] + off[i];
          }
          P[12] = P[13] = P[14] = 0.0;
          P[15] = 1.0;
        }
  }
  return 0;
}

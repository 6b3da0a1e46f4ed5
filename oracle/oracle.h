/*
 * FP64 CPU oracle for "Joint Sampling and Optimisation for Inverse Rendering"
 * (Balint, Myszkowski, Seidel, Singh; SIGGRAPH Asia 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code, header or constant table with the GPU library.
 *
 * What it computes (all in double precision):
 *   - the counter-based Philox4x32-10 generator (Salmon et al., SC'11) and the
 *     SplitMix64 mixer (Steele, Lea, Flood, OOPSLA'14) that keys it;
 *   - a path tracer for the synthetic scenes (analytic sphere/plane, a
 *     triangle mesh intersected by brute force over every triangle, square
 *     area light, uniform environment, metallic-roughness GGX + Lambert);
 *   - the proportional gradient sample <F_i> of Eq. 2 (Section 3, Notation)
 *     for an L2 image loss, with the derivative taken by recording each
 *     path's vertices on an explicit tape and sweeping it backward (reverse
 *     mode with detached sampling densities and MIS weights);
 *   - the same estimators with the paths drawn at other parameters than the
 *     integrand is evaluated at (the previous-parameter half of Eq. 5's
 *     finite-difference sample);
 *   - an emission-absorption voxel volume (the volume experiment of the
 *     Experiments section): a ray-marched quadrature and its adjoint by a
 *     backward sweep over the recorded samples;
 *   - per-pixel decision margins used to exclude paths whose discrete
 *     choices are too close to call for an FP32 vs FP64 comparison.
 * The meta-estimator and optimiser (Sections 4-5, supplement pseudocode) live
 * in oracle/meta.py (numpy, FP64).
 */
#ifndef JSO_ORACLE_H
#define JSO_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int width, height;
  double cam_eye[3], cam_target[3], cam_up[3];
  double vfov_deg;
  int plane_enabled, plane_mat;
  double plane_extent[4];            /* x0, x1, z0, z1 of the planar UV map   */
  int n_spheres;
  const double* spheres;             /* [n][4]: cx, cy, cz, r                 */
  const int* sphere_mat;             /* [n]: -1 = parameterised, else fixed k */
  int light_enabled;
  double light_center[3], light_side, light_Le[3];
  double env[3];
  int depth, rr_start;
  double rr_q;
  int tex_w, tex_h, ch_mask;         /* parameter texture layout               */
  double fixed_default[5];           /* non-parameter channels of the param mat */
  int n_fixed;
  const double* fixed_mats;          /* [n_fixed][5]: R, G, B, metal, rough    */
  /* triangle mesh (optional): two-sided, geometric normals */
  int n_verts, n_tris;
  const double* verts;               /* [n_verts][3]                           */
  const int* tris;                   /* [n_tris][3] vertex indices             */
  int mesh_mat;                      /* -1 = parameterised, else fixed k       */
  int param_layout;                  /* 0: texture (mesh: planar UV over the plane
                                        extent); 1: per mesh vertex; 2: volume  */
  /* emission-absorption volume (param_layout 2): vol_res^3 voxels filling the
   * cube of side vol_box[3] with its low corner at vol_box[0..2]; per voxel
   * (emission R, G, B, density) in [0, 1], density scaled by vol_sigma per
   * unit length; ch_mask must be 15.  The image stacks vol_views views of
   * height / vol_views rows, view v's eye turned by 2 pi v / vol_views about
   * the vertical axis through cam_target.  No surfaces or lights. */
  int vol_res, vol_views;
  double vol_box[4];
  double vol_sigma;
} orc_scene;

/* debug / test-mode flags */
enum {
  ORC_NO_NEE = 1,           /* no light sampling; BSDF-sampled light hits weigh 1 */
  ORC_LAMBERT_ONLY = 2,     /* f = c / pi, cosine sampling                         */
  ORC_PARAM_INDEP = 4,      /* both lobes sampled by the cosine density           */
  ORC_PIXEL_CENTER = 8,     /* no pixel jitter                                     */
  ORC_RELATIVE_LOSS = 16    /* orc_grad: relative squared error
                               (I - T)^2 / (T^2 + 0.01) instead of (I - T)^2       */
};

uint64_t orc_splitmix64(uint64_t x);
/* Test hook: offset (pixels) added to every primary sample position; used to
 * measure each path's sensitivity to single-precision rounding.  Default 0. */
void orc_set_jitter_offset(double dx, double dy);
/* Workload statistics accumulated over all traces since the last reset:
 * out = {paths, surface vertices, vertices on the parameterised material}. */
void orc_reset_stats(void);
void orc_get_stats(uint64_t out[3]);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_stream_key(uint64_t seed, uint32_t iteration, uint32_t tag);

/* BSDF value and partials for one direction pair (tests):
 * mat = (R,G,B,metal,rough); n, wo, wi unit vectors.
 * out[0..2] f, [3..5] df^k/dc^k, [6..8] df/dmetal, [9..11] df/drough, [12] pdf. */
void orc_bsdf(const double mat[5], const double n[3], const double wo[3], const double wi[3],
              int flags, double out[13]);
/* The same for `count` directions wi[count][3] with one (mat, n, wo): out[count][13]. */
void orc_bsdf_many(int count, const double mat[5], const double n[3], const double wo[3],
                   const double* wi, int flags, double* out);

/* Primal render: img[H*W*3] mean of spp samples; margin[H*W] min decision margin.
 * crop = {x0, y0, x1, y1} (NULL = full).  Returns 0 on success. */
int orc_render(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
               uint32_t tag, int spp, int flags, const int* crop,
               double* img, double* margin, int nthreads);

/* One gradient sample of the L2 loss L = sum (I - T)^2 / (3 W H):
 * primal image from (tag_primal), adjoint paths from (tag_adj), both spp per pixel.
 * grad/gabs[n_params] are overwritten (gabs = sum of |contribution|).
 * mask[H*W] (nullable): nonzero = skip pixel.  img (primal image), margin and
 * adj_img (mean radiance of the adjoint paths, H*W*3) are nullable outputs. */
int orc_grad(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
             uint32_t tag_primal, uint32_t tag_adj, int spp, const double* target,
             int flags, const int* crop, const unsigned char* mask,
             double* grad, double* gabs, double* img, double* margin, double* adj_img,
             int nthreads);

/* Fixed-adjoint backward: grad = sum_p dimg_p . d(mean_s C_ps)/dparams. */
int orc_render_bwd(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
                   uint32_t tag, int spp, const double* dimg, int flags, const int* crop,
                   const unsigned char* mask, double* grad, double* gabs, double* margin,
                   double* adj_img, int nthreads);

/* The same three with the paths drawn at sample_params (nullable: = params)
 * and weighted by f(x; params) / p(x; sample_params): every BSDF density --
 * the continuation's and those in both MIS weights -- is taken at
 * sample_params.  With params = pi_{i-1} and sample_params = pi_i this is the
 * previous-parameter half of Eq. 5's finite-difference sample (the path of
 * pi_i, its integrand at pi_{i-1}). */
int orc_render_sampled(const orc_scene* s, const double* params, const double* sample_params,
                       uint64_t seed, uint32_t iteration, uint32_t tag, int spp, int flags,
                       const int* crop, double* img, double* margin, int nthreads);
int orc_grad_sampled(const orc_scene* s, const double* params, const double* sample_params,
                     uint64_t seed, uint32_t iteration, uint32_t tag_primal, uint32_t tag_adj,
                     int spp, const double* target, int flags, const int* crop,
                     const unsigned char* mask, double* grad, double* gabs, double* img,
                     double* margin, double* adj_img, int nthreads);
int orc_render_bwd_sampled(const orc_scene* s, const double* params,
                           const double* sample_params, uint64_t seed, uint32_t iteration,
                           uint32_t tag, int spp, const double* dimg, int flags, const int* crop,
                           const unsigned char* mask, double* grad, double* gabs, double* margin,
                           double* adj_img, int nthreads);

#ifdef __cplusplus
}
#endif
#endif

/*
 * jso -- joint sampling and optimisation for inverse rendering on MI355X.
 *
 * C ABI of libjso.so.  Implements, for one GPU (gfx950), the per-iteration
 * hot path of the gradient meta-estimator of Bálint, Myszkowski, Seidel and
 * Singh, "Joint Sampling and Optimisation for Inverse Rendering"
 * (SIGGRAPH Asia 2023): a differentiable path tracer whose adjoint replays
 * each path from a counter-based generator, the proportional gradient sample
 * <F_i> (Eq. 1-2), the finite-difference sample <dF_i> (Eq. 3-5) traced with
 * identical random numbers at the current and previous parameters, and the
 * fused meta-estimator + stabilised step (Eq. 7-9, 13-17, 21).
 *
 * Conventions for every entry point
 *   - Return value: JSO_OK (0) or a negative JSO_E_* code.  No exceptions
 *     cross the ABI.  jso_last_error() gives a message for the last failure;
 *     the string is owned by the context and valid until the next call.
 *   - "dev" pointers are device memory on the context's device (for example
 *     torch tensor data_ptr()); they are borrowed, never freed, and used in
 *     stream order on the context's stream.  "host" pointers are read or
 *     written before the call returns.
 *   - A context is not thread-safe; use one context per host thread.
 *   - All floating-point images are H x W x 3 (row-major, RGB interleaved,
 *     row 0 at the top).  Parameter vectors use the texel-interleaved layout:
 *     parameter (y * tex_w + x) * n_ch + c (or v * n_ch + c per mesh vertex,
 *     JSO_LAYOUT_VERTEX), where the c-th channel is the c-th enabled bit of
 *     ch_mask in the order R, G, B, metalness, roughness.
 */
#ifndef JSO_H
#define JSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JSO_OK 0
#define JSO_E_INVALID (-1)     /* bad argument: null pointer, size or id      */
#define JSO_E_OOM (-2)         /* device allocation failed                    */
#define JSO_E_HIP (-3)         /* a HIP runtime call failed                   */
#define JSO_E_STATE (-4)       /* call not valid in the current state         */
#define JSO_E_UNSUPPORTED (-5) /* feature not supported by the library or the device */

/* memory space of a pointer argument */
#define JSO_MEM_HOST 0
#define JSO_MEM_DEVICE 1

/* channel bits of the parameterised material */
#define JSO_CH_R 1
#define JSO_CH_G 2
#define JSO_CH_B 4
#define JSO_CH_METAL 8
#define JSO_CH_ROUGH 16

/* material index of objects that use the parameterised material */
#define JSO_MAT_PARAM (-1)

/* random-stream tags: which estimator a path belongs to */
#define JSO_TAG_TARGET 1
#define JSO_TAG_PRIMAL_PROP 2
#define JSO_TAG_ADJ_PROP 3
#define JSO_TAG_PRIMAL_FD 4
#define JSO_TAG_ADJ_FD 5
#define JSO_TAG_ADAM_PRIMAL 6
#define JSO_TAG_ADAM_ADJ 7
#define JSO_TAG_EVAL 8
/* separate variance samples of the "uncorrelated samples" ablation */
#define JSO_TAG_VAR_PRIMAL_PROP 9
#define JSO_TAG_VAR_ADJ_PROP 10
#define JSO_TAG_VAR_PRIMAL_FD 11
#define JSO_TAG_VAR_ADJ_FD 12

/* image loss (jso_render_opts.loss, jso_step_opts.loss) */
#define JSO_LOSS_L2 0       /* sum (I - T)^2 / (3 W H)                             */
#define JSO_LOSS_RELATIVE 1 /* sum (I - T)^2 / (T^2 + 0.01) / (3 W H): the relative
                               squared error of the Experiments section, normalised
                               by the target so each pixel's weight is a constant */

/* meta-estimator ablations of the Experiments section (jso_step_opts.ablate) */
#define JSO_ABLATE_CENTRED 1      /* variance EMAs subtract their squared mean    */
#define JSO_ABLATE_NO_CLIP 2      /* no alpha clipping (Eq. 17)                   */
#define JSO_ABLATE_UNCORRELATED 4 /* variance EMAs fed by a second, independent
                                     proportional + FD sample (tags VAR_*)        */

/* finite-difference sample <dF_i> (jso_render_opts.fd_mode, jso_step_opts.fd_mode) */
#define JSO_FD_REPLAY 0 /* two paths from the same random numbers, each drawn at its own
                           parameters (pi_i, pi_{i-1}) and differenced per vertex     */
#define JSO_FD_SHARED 1 /* Eq. 5 as written: one path drawn at pi_i, its integrand
                           evaluated at pi_i and at pi_{i-1} over the density of pi_i
                           (every BSDF pdf, hence every MIS weight, at pi_i); the two
                           gradients share each vertex's footprint and are differenced
                           before one scatter.  Halves the finite-difference tracing. */

/* render / test-mode flags (jso_render_opts.flags, jso_set_debug) */
#define JSO_F_NO_NEE 1       /* no light sampling; BSDF-sampled light hits weigh 1 */
#define JSO_F_LAMBERT_ONLY 2 /* f = c/pi with cosine sampling                      */
#define JSO_F_PARAM_INDEP 4  /* both lobes sampled with the cosine density         */
#define JSO_F_PIXEL_CENTER 8 /* no pixel jitter                                    */
/* Deterministic gradient sums: each replayed contribution is rounded to a
 * multiple of 2^-k and summed in 64-bit fixed point with integer atomics
 * (associative, so the result is bitwise the same whatever the order of the
 * atomics, the launch configuration or the batching), then folded into the
 * FP32 gradient.  k = 32 + ceil(log2(1.5 W H)) for the estimators (their
 * adjoint images carry 1 / (1.5 W H)), 32 for jso_render_bwd; a gradient
 * element must stay below 2^(63-k) in magnitude.  Slower (no block table,
 * one integer atomic per contribution); not for volume scenes or
 * jso_render_bwd_noalloc (JSO_E_UNSUPPORTED). */
#define JSO_F_DETERMINISTIC 16
/* The replay traces every ray again instead of reading the hit records its
 * forward pass wrote (triangle-mesh scenes: the records hold, for the first
 * rays of each replayed path, what the ray hit and whether the vertex's
 * shadow ray is blocked; the replay takes a record only for the bitwise same
 * ray, so both ways give the same gradients up to the order of the float
 * atomics).  For tests and timing. */
#define JSO_F_NO_HIT_RECORDS 32

#define JSO_MAX_SPHERES 32
#define JSO_MAX_FIXED_MATS 8
#define JSO_MAX_TRIS 4194304 /* triangles of the optional mesh */

/* layout of the parameter vector (jso_scene_desc.param_layout) */
#define JSO_LAYOUT_TEXTURE 0 /* texels: (y * tex_w + x) * n_ch + c                */
#define JSO_LAYOUT_VERTEX 1  /* mesh vertices: v * n_ch + c, interpolated with the
                                barycentric weights of the hit point; only the
                                mesh may then use JSO_MAT_PARAM                  */
#define JSO_LAYOUT_VOLUME 2  /* emission-absorption volume: voxel
                                ((z * R + y) * R + x) * 4 + c, c = emission R, G, B,
                                density (ch_mask 15), trilinear interpolation  */
#define JSO_MAX_VIEWS 16     /* cameras of a volume scene                         */
#define JSO_MAX_VOL_RES 512  /* voxels per side                                   */

typedef struct jso_ctx jso_ctx;

/* Scene description (host memory; copied by jso_load_scene).
 * Geometry: optional infinite plane y = 0 (hit only from above), spheres,
 * an optional triangle mesh (two-sided, shaded with its geometric normal),
 * a one-sided square area light facing -y, a uniform environment.  On equal
 * distance the plane wins over spheres, spheres over the mesh, the mesh over
 * the light, and a lower triangle index over a higher one.
 * The parameterised material is a tex_h x tex_w texture (1 x 1 = one global
 * material) of the channels in ch_mask, mapped to the plane and the mesh by
 * planar UV over plane_extent and to spheres by latitude-longitude; or, with
 * param_layout = JSO_LAYOUT_VERTEX, one set of channels per mesh vertex.
 * Channels not in ch_mask take fixed_default.  Fixed materials are rows
 * (R, G, B, metalness, roughness).  The mesh is indexed by a bounding volume
 * hierarchy built on the host when the scene is loaded. */
typedef struct {
  int width, height;
  float cam_eye[3], cam_target[3], cam_up[3];
  float vfov_deg;
  int plane_enabled, plane_mat;
  float plane_extent[4]; /* x0, x1, z0, z1 of the planar UV map */
  int n_spheres;         /* <= JSO_MAX_SPHERES                  */
  const float* spheres;  /* [n][4]: cx, cy, cz, radius         */
  const int* sphere_mat; /* [n]: JSO_MAT_PARAM or a fixed index */
  int light_enabled;
  float light_center[3], light_side, light_Le[3];
  float env[3];
  int depth;    /* maximum number of scattering vertices (>= 1)      */
  int rr_start; /* 0 = no roulette, else first vertex whose continuation is rouletted */
  float rr_q;   /* survival probability of the roulette                */
  int tex_w, tex_h, ch_mask;
  float fixed_default[5];
  int n_fixed; /* <= JSO_MAX_FIXED_MATS */
  const float* fixed_mats;
  /* triangle mesh (n_tris = 0: none) */
  int n_verts, n_tris;   /* n_tris <= JSO_MAX_TRIS                         */
  const float* verts;    /* [n_verts][3]: x, y, z                           */
  const int* tris;       /* [n_tris][3]: vertex indices                     */
  int mesh_mat;          /* JSO_MAT_PARAM or a fixed index                  */
  int param_layout;      /* JSO_LAYOUT_TEXTURE, _VERTEX or _VOLUME          */
  /* emission-absorption volume (param_layout = JSO_LAYOUT_VOLUME; the volume
   * experiment of the Experiments section): vol_res^3 voxels filling the cube
   * of side vol_box[3] whose low corner is vol_box[0..2], voxel centres at
   * (i + 0.5) / vol_res of the side, clamp-to-edge trilinear interpolation;
   * per voxel emission RGB and a density in [0, 1], the density scaled by
   * vol_sigma per unit length.  A camera ray's chord through the cube is
   * split into N = ceil(chord / voxel side) equal segments of length dt,
   * sampled at t0 + (k + u) dt (one jitter u per ray, 0.5 with
   * JSO_F_PIXEL_CENTER); radiance sum_k T_k (1 - exp(-sigma_k dt)) e_k +
   * T_N env.  The image stacks vol_views views (height / vol_views rows
   * each); view v's eye is cam_eye turned by 2 pi v / vol_views about the
   * vertical axis through cam_target.  No plane, spheres, mesh or light;
   * depth, roulette and texture fields are ignored. */
  int vol_res, vol_views;
  float vol_box[4];
  float vol_sigma;
} jso_scene_desc;

typedef struct {
  uint32_t flags;            /* JSO_F_*                                          */
  int crop[4];               /* x0, y0, x1, y1; all zero = whole image            */
  const uint8_t* pixel_mask; /* dev, H*W, nonzero = skip the pixel; may be NULL   */
  int loss;                  /* JSO_LOSS_* of the adjoint image (estimators)        */
  int fd_mode;               /* JSO_FD_* of jso_estimate_gradients' dF              */
} jso_render_opts;

/* Optimiser of jso_grad_step */
#define JSO_OPT_META 0
#define JSO_OPT_ADAM 1

typedef struct {
  int optimizer;       /* JSO_OPT_META or JSO_OPT_ADAM                            */
  float eta;           /* learning rate                                           */
  float beta_F;        /* meta: EMA coefficient of Var[F]   (Eq. 9), e.g. 0.99     */
  float beta_D;        /* meta: EMA coefficient of Var[dF]_D (Eq. 13), e.g. 0.9    */
  int spp_prop;        /* meta: proportional samples per pixel (paper: 2)         */
  int spp_fd;          /* meta: finite-difference samples per pixel (paper: 1)    */
  float adam_beta1, adam_beta2, adam_eps; /* adam: Eq. 18-20                      */
  int adam_spp;        /* adam: samples per pixel                                  */
  uint64_t seed;       /* base seed of all random streams                          */
  uint32_t flags;      /* JSO_F_* test modes                                       */
  float precond_lambda; /* > 0: replace each texture-gradient sample g (per channel)
                           by (I + lambda L)^-1 g, L the Laplacian of the 4-neighbour
                           texel grid (Large Steps, Nicolet et al. 2021, as used for
                           the texture tasks of the Experiments section); 0 = off.
                           Problems with a 1x1 texture are unaffected; per-vertex
                           parameters are rejected.                                */
  int loss;             /* JSO_LOSS_*                                               */
  uint32_t ablate;      /* meta: JSO_ABLATE_* bits (0 = the method as published)    */
  int fd_mode;          /* meta: JSO_FD_* form of the finite-difference sample       */
} jso_step_opts;

typedef struct {
  double loss;         /* L2 loss of the proportional primal image of the step   */
  double step_norm2;   /* ||pi_{i+1} - pi_i||^2 of the step just applied          */
  uint32_t iteration;  /* iteration index after the step                          */
} jso_step_stats;

/* Checkpoint view of one problem's optimiser state (host buffers of n_params). */
typedef struct {
  float* params;       /* pi_i                      */
  float* params_prev;  /* pi_{i-1}                  */
  double* mean;        /* <F_{i-1}>_M               */
  double* var;         /* Var[F_{i-1}]_M            */
  double* alpha_prev;  /* alpha_{i-1}               */
  double* m2_F;        /* Var[F] EMA                */
  double* m2_D;        /* Var[dF]_D EMA             */
  float* adam_m;       /* Adam first moment         */
  float* adam_v;       /* Adam second moment        */
  uint32_t iteration, count_F, count_D, adam_t;
  double step_norm2;   /* ||pi_i - pi_{i-1}||^2     */
} jso_state;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`.  stream: the hipStream_t all
 * work is queued on (borrowed; NULL = the device's null stream, which is
 * also torch's default stream). */
int jso_create(jso_ctx** out, int device, void* stream);
/* Destroy the context and free every device buffer it owns.  NULL is a no-op. */
int jso_destroy(jso_ctx* ctx);
const char* jso_last_error(const jso_ctx* ctx);
/* Replace the stream used by subsequent calls (NULL = the null stream). */
int jso_set_stream(jso_ctx* ctx, void* stream);
/* Wait for all work queued on the context's stream. */
int jso_synchronize(jso_ctx* ctx);
/* Default test-mode flags OR-ed into every render of this context. */
int jso_set_debug(jso_ctx* ctx, uint32_t flags);

/* ---- counter-based random numbers ------------------------------- */

/* 64-bit Philox key of a stream: splitmix64(seed ^ splitmix64((iteration << 8) | tag)),
 * with SplitMix64 of Steele, Lea and Flood (2014).  Pure function. */
uint64_t jso_stream_key(uint64_t seed, uint32_t iteration, uint32_t tag);
/* Philox4x32-10 (Salmon et al., SC'11) on the device: out[i] = philox(ctr[i], key)
 * for n counters; ctr, out are dev arrays of n x 4 uint32 (key: lo word = k0). */
int jso_philox(jso_ctx* ctx, uint64_t key, const uint32_t* ctr, size_t n, uint32_t* out);

/* ---- scenes / problems ---------------------------------------------------- */

/* Upload a scene: everything of the inverse problem except its parameters
 * (Introduction: inverse rendering estimates the scene parameters --
 * materials, textures -- from a target image, with the rest of the scene
 * given).  Builds the mesh's hierarchy on the host, allocates the problem's
 * parameter, target, gradient and optimiser buffers on the device.
 * Parameters start at fixed_default / 0.5.  desc and its arrays are host
 * memory owned by the caller and copied before return.  Errors:
 * JSO_E_INVALID (sizes out of range, null arrays), JSO_E_OOM, JSO_E_HIP. */
int jso_load_scene(jso_ctx* ctx, const jso_scene_desc* desc, int* scene_id);
int jso_free_scene(jso_ctx* ctx, int scene_id);
int jso_scene_info(jso_ctx* ctx, int scene_id, size_t* n_params, int* width, int* height);
/* Set the parameter vector pi (Section 3's notation: F_i integrates f(x, pi_i);
 * n = n_params, float32, layout above; mem = JSO_MEM_HOST or _DEVICE).
 * Starts the optimisation loop of Sections 4-5 afresh: pi_{i-1} = pi,
 * iteration 0, both variance averages empty, alpha_{-1} = -inf (so alpha_0 = 0,
 * Eq. 7's initialisation), Adam moments 0.  Errors: JSO_E_INVALID (bad id,
 * null p, n != n_params), JSO_E_HIP. */
int jso_set_params(jso_ctx* ctx, int scene_id, const float* p, size_t n, int mem);
int jso_get_params(jso_ctx* ctx, int scene_id, float* p, size_t n, int mem);
int jso_get_params_prev(jso_ctx* ctx, int scene_id, float* p, size_t n, int mem);
/* The target image the loss compares each rendering with (Introduction:
 * the loss quantifies the disparity between the image rendered with the
 * current parameters and the target).  n = H*W*3 float32; mem as above. */
int jso_set_target(jso_ctx* ctx, int scene_id, const float* img, size_t n, int mem);

/* Texture-gradient preconditioner (Large Steps; Nicolet, Jacobson, Jakob 2021,
 * cited in the Experiments section for texture tasks): g (dev, n_params) is
 * replaced in place, channel by channel, by the solution y of
 * (I + lambda L) y = g, L = degree minus adjacency of the 4-neighbour
 * tex_h x tex_w grid.  Solved exactly in the grid's cosine basis (which
 * diagonalises L), in FP32.  lambda >= 0; a 1x1 texture is left unchanged.
 * Errors: JSO_E_INVALID (bad id, null g, lambda < 0, per-vertex layout). */
int jso_precondition(jso_ctx* ctx, int scene_id, float* g, float lambda);

/* ---- rendering and differentiation ---------------------------- */

/* Forward rendering by path tracing (Introduction: the rendering equation
 * estimated by Monte Carlo for given scene parameters; Related work, path
 * tracing): img (dev, H*W*3) = mean of spp paths per pixel with the
 * parameters `params` (dev, n_params), stream (seed, iteration, tag).
 * Pixels outside the crop or masked are left untouched.  opts may be NULL. */
int jso_render(jso_ctx* ctx, int scene_id, const float* params, uint64_t seed,
               uint32_t iteration, uint32_t tag, int spp, const jso_render_opts* opts,
               float* img);
/* Path replay backpropagation (Related work; Experiments, implementation):
 * the derivative of jso_render's image with respect to the scene
 * parameters, backpropagated from an adjoint image (Introduction: gradients
 * w.r.t. the scene parameters from the loss).  dparams (dev, n_params) += sum over pixels p
 * of dimg_p . d(mean_s C_ps)/dparams, with C_ps re-traced from the same stream
 * (no tape).  The derivative treats sampling densities and MIS weights as
 * constants (detached sampling).  dparams is accumulated into, not cleared. */
int jso_render_bwd(jso_ctx* ctx, int scene_id, const float* params, uint64_t seed,
                   uint32_t iteration, uint32_t tag, int spp, const float* dimg,
                   const jso_render_opts* opts, float* dparams);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as jso_render_bwd (same arguments, same streams, dparams accumulated
 * into), but the forward radiance of the replayed paths lives in a scratch
 * array of JSO_NOALLOC_SCRATCH_BYTES that the library holds per GPU, set up by
 * jso_create; the call itself allocates nothing (no hipMalloc/hipFree).  Each
 * sample needs H*W*24 bytes of it, so images above JSO_NOALLOC_MAX_PIXELS
 * pixels are rejected (JSO_E_INVALID); larger spp run in more launches.  All
 * calls on one GPU share the array: calls that overlap in time on one GPU
 * (other streams, other contexts, other threads) race and give wrong results;
 * calls in one stream's order are safe.  Nothing in the array needs to start
 * at zero.  Errors: as jso_render_bwd; JSO_E_STATE if the context has no
 * scratch address. */
#define JSO_NOALLOC_SCRATCH_BYTES (128u << 20)
#define JSO_NOALLOC_MAX_PIXELS (JSO_NOALLOC_SCRATCH_BYTES / 24u)
int jso_render_bwd_noalloc(jso_ctx* ctx, int scene_id, const float* params, uint64_t seed,
                           uint32_t iteration, uint32_t tag, int spp, const float* dimg,
                           const jso_render_opts* opts, float* dparams);

/* ---- estimators ------------------------------------------------ */

/* One iteration's gradient samples for the loss opts->loss (L2 by default,
 * sum (I - T)^2 / (3 W H)) against the scene's target, at the scene's pi_i
 * (and pi_{i-1}):
 *   F  += <F_i>   spp_prop primal paths (tag PRIMAL_PROP) give the adjoint
 *                 image, spp_prop adjoint paths (tag ADJ_PROP) are replayed;
 *   dF += <dF_i>  the spp_fd primal and adjoint streams (PRIMAL_FD, ADJ_FD)
 *                 traced at pi_i and at pi_{i-1} with identical random numbers
 *                 and differenced per vertex (Eq. 5); opts->fd_mode =
 *                 JSO_FD_SHARED traces each path once, at pi_i, and evaluates
 *                 it at both.  Skipped if dF is NULL.
 * F, dF: dev, n_params, accumulated into.  img (dev, H*W*3, nullable) receives
 * the proportional primal image.  iteration selects the random streams.
 * loss (host, nullable) receives the loss of that primal image. */
int jso_estimate_gradients(jso_ctx* ctx, int scene_id, uint64_t seed, uint32_t iteration,
                           int spp_prop, int spp_fd, const jso_render_opts* opts, float* F,
                           float* dF, float* img, double* loss);

/* ---- optimiser steps ------------------------------------------- */

/* One meta-estimator step on given gradient samples (dev, n_params each):
 * Moment2 updates of Var[F] and Var[dF]_D (Eq. 9, 13; bias-corrected), the
 * rescale of Eq. 14 with ||pi_i - pi_{i-1}||^2, alpha (Eq. 8) clipped by
 * Eq. 17, the recurrence (Eq. 7, 15), the step of Eq. 21, projection onto the
 * parameter box, and the norm of the applied step for the next iteration.
 * At iteration 0 or when the last step was zero, dF is ignored (no FD sample).
 * F and dF are read only. */
int jso_meta_step(jso_ctx* ctx, int scene_id, const float* F, const float* dF, float eta,
                  float beta_F, float beta_D);
/* One Adam step (Eq. 18-20, bias-corrected) on gradient g (dev, n_params). */
int jso_adam_step(jso_ctx* ctx, int scene_id, const float* g, float eta, float beta1,
                  float beta2, float eps);

/* One iteration of the optimisation loop (supplement, loop snippet;
 * Sections 3-5): the proportional sample <F_i> (Eq. 2), the finite-difference
 * sample <dF_i> (Eq. 5), then jso_meta_step's update, for each listed
 * problem -- or Adam's step (Eq. 18-20) on one sample of opts->adam_spp.
 * The samples go into the scene's own gradient buffers, then the fused
 * optimiser step, which also clears those buffers for the next iteration.
 * All listed problems share one launch per kernel (Section 5's loop, run for
 * many independent problems at once); scene ids must be distinct.  stats
 * (host array of n, nullable) waits for the stream and reports each
 * problem's loss and step. */
int jso_grad_step(jso_ctx* ctx, const int* scene_ids, int n, const jso_step_opts* opts,
                  jso_step_stats* stats);

/* ---- batches ------------------------------------------------------------------------ */

/* A fixed set of independent problems optimised together (the loop of
 * Section 5 for each): every iteration is one launch per kernel for all of
 * them, from launch descriptors uploaded once at creation, optionally
 * captured in a HIP graph and replayed.  max_iters (host array of n,
 * nullable): problem k stops changing once its own iteration counter reaches
 * max_iters[k] (0 = no limit); the kernels skip finished problems.  The
 * options, scene ids and the scenes' buffers are fixed at creation: do not
 * free a scene or replace its buffers (jso_load_scene of new sizes) while a
 * batch refers to it.  jso_set_params, jso_set_target and jso_set_state
 * remain valid between steps.  Not thread-safe per context; the batch runs
 * on its context's stream.  Errors: JSO_E_INVALID (bad ids/options),
 * JSO_E_OOM, JSO_E_HIP. */
typedef struct jso_batch jso_batch;
int jso_batch_create(jso_ctx* ctx, const int* scene_ids, int n, const jso_step_opts* opts,
                     const uint32_t* max_iters, int use_graph, jso_batch** out);
/* Run `iterations` iterations of every active problem (returns when queued). */
int jso_batch_step(jso_batch* b, int iterations);
/* Number of problems whose iteration counter is still below its limit
 * (waits for the stream). */
int jso_batch_active(jso_batch* b, int* active);
int jso_batch_destroy(jso_batch* b);

/* Launch configurations of the path kernels (forward tracing and replay):
 * a pixel tile shape, one workgroup per tile ... */
#define JSO_TILE_16x16 0 /* 256 lanes */
#define JSO_TILE_16x8 1  /* 128 lanes */
#define JSO_TILE_8x8 2   /* 64 lanes  */
#define JSO_TILE_SHAPES 3
/* ... and a grid: configuration c uses tile shape c % JSO_TILE_SHAPES and,
 * for c >= JSO_TILE_SHAPES, a persistent grid of {1, 2, 4, 8}[c / 3 - 1]
 * workgroups per compute unit that pull tiles from a work queue (in steps
 * and batches; single renders always launch one workgroup per tile).
 * Configurations 0-2 are the plain grids of the three tile shapes. */
#define JSO_LAUNCH_CONFIGS 15
/* Time `iterations` real iterations of the batch with each launch
 * configuration (the problems' optimiser state is restored after each
 * trial), keep the fastest for this batch and remember it, for this GPU
 * architecture and configuration (image sizes, parameter layouts, sample
 * counts), for every later batch or jso_grad_step of the process with the
 * same configuration.  best_config (nullable) receives the configuration; ms
 * (nullable host array of JSO_LAUNCH_CONFIGS) the milliseconds per iteration
 * of each.  Waits for the stream.  Errors: JSO_E_INVALID, JSO_E_OOM,
 * JSO_E_HIP. */
int jso_batch_autotune(jso_batch* b, int iterations, int* best_config, double* ms);
/* Launch configuration used when the tuner has no entry for a configuration
 * (0 .. JSO_LAUNCH_CONFIGS - 1, default 0: 16x16 tiles, one per workgroup). */
int jso_set_launch_config(jso_ctx* ctx, int config);

/* ---- kernel timing --------------------------------------------------------------- */

/* Kernel classes reported by jso_get_kernel_time */
#define JSO_K_FORWARD 0  /* forward path tracing (primal and adjoint paths) */
#define JSO_K_ADJOINT 1  /* replayed adjoint (proportional + FD pairs)      */
#define JSO_K_META 2     /* fused meta-estimator step                       */
#define JSO_K_ADAM 3     /* Adam step                                       */
#define JSO_K_FINALIZE 4 /* primal images, adjoint images and loss          */
#define JSO_K_PRECOND 5  /* texture-gradient preconditioner passes          */
#define JSO_K_COUNT 6

/* Enable (1) or disable (0) HIP-event timing of every kernel this context
 * launches (events are recorded on the context's stream around each launch). */
int jso_set_timing(jso_ctx* ctx, int enable);
/* Device time (ms) summed over the launches of one kernel class since timing
 * was enabled or last reset, and their number.  Waits for the recorded
 * events.  reset != 0 clears the totals afterwards. */
int jso_get_kernel_time(jso_ctx* ctx, int kernel, double* ms, uint64_t* launches, int reset);

/* ---- memory-system microbenchmarks ------------------------------------ */

/* The denominators of the roofline fractions the benchmark reports; not part
 * of the method.  Each runs its kernel once untimed, then `reps` times on the
 * context's stream, and returns the mean time per run in *ms (HIP events).
 * jso_ub_copy: dst = src for `bytes` bytes (dev; both 16-byte aligned, bytes a
 * multiple of 16, the buffers not overlapping).
 * jso_ub_atomics: n_ops no-return FP32 atomic adds of 1.0 into buf (dev,
 * n_buf >= 16 floats), operation i to
 *   JSO_UB_RANDOM  a hashed index in [0, n_buf)
 *   JSO_UB_LINES   16 consecutive operations to the 16 floats of one hashed
 *                  64-byte segment (the coalesced form of a texel scatter)
 *   JSO_UB_16      index i mod 16
 *   JSO_UB_SAME    index 0
 *   JSO_UB_ROWS    4 consecutive operations to the 4 floats of one hashed
 *                  16-byte row (the form of a volume replay's voxel write-out)
 * Errors: JSO_E_INVALID for bad arguments, JSO_E_HIP for a failed launch. */
#define JSO_UB_RANDOM 0
#define JSO_UB_LINES 1
#define JSO_UB_16 2
#define JSO_UB_SAME 3
#define JSO_UB_ROWS 4
int jso_ub_copy(jso_ctx* ctx, void* dst, const void* src, size_t bytes, int reps, double* ms);
/* jso_ub_launch: a chain of n_kernels (1..4096) dependent one-block launches,
 * each adding 1 to counter[0] (dev, one uint32; it ends up raised by
 * n_kernels x (reps + 1)), issued on the context's stream one by one
 * (use_graph = 0) or replayed from a graph of the same launches captured
 * once (use_graph != 0); *ms is per chain, so *ms / n_kernels is the gap
 * between dependent launches. */
int jso_ub_launch(jso_ctx* ctx, uint32_t* counter, int n_kernels, int use_graph, int reps,
                  double* ms);
int jso_ub_atomics(jso_ctx* ctx, float* buf, size_t n_buf, int pattern, size_t n_ops, int reps,
                   double* ms);

/* Work counters, for throughput accounting.  While enabled, the launches of
 * this context add: out[0] the paths the adjoint replays (a finite-difference
 * pair counts two), out[1] their surface vertices; out[2] the paths traced
 * forward (primal samples and the adjoint paths' forward passes), out[3]
 * their surface vertices.  Enabling allocates 32 bytes of device memory on
 * first use; counting costs one 64-bit atomic per wave and counter.
 * jso_get_work waits for the context's stream, copies the four totals to the
 * host array out[4] and, if reset != 0, clears them.
 * Errors: JSO_E_INVALID for a null ctx/out. */
int jso_set_work_counting(jso_ctx* ctx, int enable);
int jso_get_work(jso_ctx* ctx, uint64_t out[4], int reset);

/* ---- checkpoint ---------------------------------------------------------------- */
/* The state the optimisation loop carries from iteration i to i + 1
 * (Sections 4-5, supplement pseudocode): pi_i, pi_{i-1}, <F_{i-1}>_M and
 * Var[F_{i-1}]_M (Eq. 7, 15), alpha_{i-1} (Eq. 17), the two variance
 * averages (Eq. 9, 13) with their sample counts, ||dpi_i||^2 (Eq. 14), Adam's
 * moments.  jso_get_state waits for the stream and copies every buffer of
 * the view (host arrays of n_params each, caller-owned; none may be NULL) and
 * the counters; jso_set_state uploads them, so that the next jso_grad_step
 * continues exactly as the checkpointed run would have.  Errors:
 * JSO_E_INVALID (bad id, null buffer), JSO_E_HIP. */
int jso_get_state(jso_ctx* ctx, int scene_id, jso_state* st);
int jso_set_state(jso_ctx* ctx, int scene_id, const jso_state* st);

#ifdef __cplusplus
}
#endif
#endif /* JSO_H */

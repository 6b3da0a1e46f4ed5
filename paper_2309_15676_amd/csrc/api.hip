// Host runtime of libjso: contexts, scene upload, buffers, and the C ABI
// declared in include/jso.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "jso.h"
#include "kernels.h"

using namespace jso;

namespace {

struct SceneGPU {
  DevScene dev{};
  int width = 0, height = 0, n_ch = 0;
  size_t P = 0, npix = 0;
  float lo[5] = {0, 0, 0, 0, 0}, hi[5] = {1, 1, 1, 1, 1};
  // device buffers (owned)
  float *params = nullptr, *params_prev = nullptr, *target = nullptr;
  float *F = nullptr, *dF = nullptr, *delta = nullptr;  // delta: 3 images (prop, fd cur, fd prev)
  double *mean = nullptr, *var = nullptr, *alpha_prev = nullptr, *m2F = nullptr, *m2D = nullptr;
  float *adam_m = nullptr, *adam_v = nullptr;
  Ctl* ctl = nullptr;
  double* scratch_loss = nullptr;  // 2 slots for stand-alone estimator calls
  double* partials = nullptr;      // per-block partial sums of the meta step
  double* slots = nullptr;         // per-path radiance, kMaxSlots per pixel (3 doubles each)
  double* accum = nullptr;         // per-pixel radiance sums of up to 3 primal images
  DevScene* d_scene = nullptr;     // device copy of `dev` read by the kernels
  uint32_t host_iter = 0;          // mirror of ctl->iteration
};

}  // namespace

// HIP-event timing of kernel launches, per kernel class.
struct KernelTimer {
  bool enabled = false;
  std::vector<hipEvent_t> pool;                                   // free events
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[JSO_K_COUNT];
  double ms[JSO_K_COUNT] = {0, 0, 0, 0};
  uint64_t launches[JSO_K_COUNT] = {0, 0, 0, 0};

  hipEvent_t get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
      e = pool.back();
      pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
  // fold finished intervals into the totals (waits for them)
  hipError_t collect() {
    for (int k = 0; k < JSO_K_COUNT; ++k) {
      for (auto& pr : pending[k]) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return e;
        float t = 0.0f;
        e = hipEventElapsedTime(&t, pr.first, pr.second);
        if (e != hipSuccess) return e;
        ms[k] += t;
        launches[k]++;
        pool.push_back(pr.first);
        pool.push_back(pr.second);
      }
      pending[k].clear();
    }
    return hipSuccess;
  }
  void destroy() {
    (void)collect();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

struct jso_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // nullptr = the device's null (default) stream
  uint32_t debug_flags = 0;
  std::string err;
  std::vector<std::unique_ptr<SceneGPU>> scenes;
  KernelTimer timer;
  unsigned long long* d_work = nullptr;  // work counters (replay paths/vertices, forward paths/vertices)
  bool counting = false;
};

namespace {

int fail(jso_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                             \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, e_ == hipErrorOutOfMemory ? JSO_E_OOM : JSO_E_HIP, "%s: %s (%s)", \
                  #expr, hipGetErrorString(e_), __func__);                             \
  } while (0)

// Launch `expr` (returning hipError_t) bracketed by timing events when enabled.
#define TIMED_LAUNCH(ctx, kind, expr)                                               \
  do {                                                                              \
    hipEvent_t t0_ = nullptr, t1_ = nullptr;                                        \
    if ((ctx)->timer.enabled) {                                                     \
      t0_ = (ctx)->timer.get();                                                     \
      t1_ = (ctx)->timer.get();                                                     \
      if (t0_) HIP_TRY(ctx, hipEventRecord(t0_, (ctx)->stream));                    \
    }                                                                               \
    HIP_TRY(ctx, expr);                                                             \
    if (t0_ && t1_) {                                                               \
      HIP_TRY(ctx, hipEventRecord(t1_, (ctx)->stream));                             \
      (ctx)->timer.pending[kind].push_back({t0_, t1_});                             \
    }                                                                               \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

SceneGPU* get_scene(jso_ctx* c, int id) {
  if (!c || id < 0 || id >= (int)c->scenes.size()) return nullptr;
  return c->scenes[id].get();
}

void free_scene_buffers(SceneGPU* s) {
  void* bufs[] = {s->params, s->params_prev, s->target, s->F,      s->dF,
                  s->delta,  s->mean,        s->var,    s->alpha_prev, s->m2F,
                  s->m2D,    s->adam_m,      s->adam_v, s->ctl,    s->scratch_loss,
                  s->partials, s->slots,     s->accum,  s->d_scene};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), (n ? n : 1) * sizeof(T));
}

int build_devscene(jso_ctx* c, const jso_scene_desc* d, SceneGPU* s) {
  if (d->width <= 0 || d->height <= 0 || d->width > 16384 || d->height > 16384)
    return fail(c, JSO_E_INVALID, "image size %dx%d out of range", d->width, d->height);
  if (d->n_spheres < 0 || d->n_spheres > JSO_MAX_SPHERES || (d->n_spheres && !d->spheres))
    return fail(c, JSO_E_INVALID, "n_spheres %d invalid (max %d)", d->n_spheres, JSO_MAX_SPHERES);
  if (d->n_fixed < 0 || d->n_fixed > JSO_MAX_FIXED_MATS || (d->n_fixed && !d->fixed_mats))
    return fail(c, JSO_E_INVALID, "n_fixed %d invalid", d->n_fixed);
  if (d->depth < 1 || d->depth > 64) return fail(c, JSO_E_INVALID, "depth %d invalid", d->depth);
  if (d->tex_w < 1 || d->tex_h < 1 || d->tex_w > 8192 || d->tex_h > 8192)
    return fail(c, JSO_E_INVALID, "texture %dx%d invalid", d->tex_w, d->tex_h);
  if (d->ch_mask <= 0 || d->ch_mask > 31) return fail(c, JSO_E_INVALID, "ch_mask invalid");
  if (d->rr_start < 0 || (d->rr_start > 0 && !(d->rr_q > 0.0f && d->rr_q <= 1.0f)))
    return fail(c, JSO_E_INVALID, "roulette settings invalid");
  auto check_mat = [&](int m) { return m == JSO_MAT_PARAM || (m >= 0 && m < d->n_fixed); };
  if (d->plane_enabled && !check_mat(d->plane_mat))
    return fail(c, JSO_E_INVALID, "plane material %d invalid", d->plane_mat);
  for (int k = 0; k < d->n_spheres; ++k) {
    if (!(d->spheres[4 * k + 3] > 0.0f)) return fail(c, JSO_E_INVALID, "sphere %d radius", k);
    if (!check_mat(d->sphere_mat ? d->sphere_mat[k] : JSO_MAT_PARAM))
      return fail(c, JSO_E_INVALID, "sphere %d material invalid", k);
  }
  if (d->light_enabled && !(d->light_side > 0.0f))
    return fail(c, JSO_E_INVALID, "light side must be positive");

  DevScene& S = s->dev;
  std::memset(&S, 0, sizeof(S));
  S.width = d->width;
  S.height = d->height;
  // camera basis (computed in double, stored as float)
  double e[3] = {d->cam_eye[0], d->cam_eye[1], d->cam_eye[2]};
  double w[3] = {d->cam_target[0] - e[0], d->cam_target[1] - e[1], d->cam_target[2] - e[2]};
  double wl = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  if (!(wl > 0)) return fail(c, JSO_E_INVALID, "camera target equals eye");
  for (double& x : w) x /= wl;
  double up[3] = {d->cam_up[0], d->cam_up[1], d->cam_up[2]};
  double u[3] = {w[1] * up[2] - w[2] * up[1], w[2] * up[0] - w[0] * up[2],
                 w[0] * up[1] - w[1] * up[0]};
  double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(ul > 0)) return fail(c, JSO_E_INVALID, "camera up parallel to view");
  for (double& x : u) x /= ul;
  double v[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
  for (int k = 0; k < 3; ++k) {
    S.eye[k] = (float)e[k];
    S.cw[k] = (float)w[k];
    S.cu[k] = (float)u[k];
    S.cv[k] = (float)v[k];
  }
  S.tan_half = (float)std::tan((double)d->vfov_deg * M_PI / 360.0);
  S.aspect = (float)((double)d->width / (double)d->height);
  S.plane_enabled = d->plane_enabled;
  S.plane_mat = d->plane_mat;
  S.plane_x0 = d->plane_extent[0];
  S.plane_x1 = d->plane_extent[1];
  S.plane_z0 = d->plane_extent[2];
  S.plane_z1 = d->plane_extent[3];
  if (d->plane_enabled && (S.plane_x1 == S.plane_x0 || S.plane_z1 == S.plane_z0))
    return fail(c, JSO_E_INVALID, "plane extent is empty");
  S.n_spheres = d->n_spheres;
  for (int k = 0; k < d->n_spheres; ++k) {
    for (int q = 0; q < 4; ++q) S.sph[k][q] = d->spheres[4 * k + q];
    S.sph_mat[k] = d->sphere_mat ? d->sphere_mat[k] : JSO_MAT_PARAM;
  }
  S.light_enabled = d->light_enabled;
  for (int k = 0; k < 3; ++k) {
    S.lc[k] = d->light_center[k];
    S.Le[k] = d->light_Le[k];
    S.env[k] = d->env[k];
  }
  S.lside = d->light_side;
  S.lhalf = 0.5f * d->light_side;
  S.larea = d->light_side * d->light_side;
  S.depth = d->depth;
  S.rr_start = d->rr_start;
  S.rr_q = d->rr_q;
  S.tex_w = d->tex_w;
  S.tex_h = d->tex_h;
  int nc = 0;
  static const float kLo[5] = {0.f, 0.f, 0.f, 0.f, 0.05f}, kHi[5] = {1.f, 1.f, 1.f, 1.f, 1.f};
  for (int b = 0; b < 5; ++b) {
    S.defaults[b] = d->fixed_default[b];
    if (d->ch_mask >> b & 1) {
      s->lo[nc] = kLo[b];
      s->hi[nc] = kHi[b];
      S.slot[b] = nc++;
    } else {
      S.slot[b] = -1;
    }
  }
  S.n_ch = nc;
  S.n_fixed = d->n_fixed;
  for (int m = 0; m < d->n_fixed; ++m)
    for (int q = 0; q < 5; ++q) S.fixed[m][q] = d->fixed_mats[5 * m + q];
  s->width = d->width;
  s->height = d->height;
  s->n_ch = nc;
  s->npix = (size_t)d->width * d->height;
  s->P = (size_t)d->tex_w * d->tex_h * nc;
  return JSO_OK;
}

Crop crop_of(const SceneGPU* s, const jso_render_opts* o) {
  Crop c{0, 0, s->width, s->height};
  if (o && (o->crop[0] | o->crop[1] | o->crop[2] | o->crop[3])) {
    c.x0 = o->crop[0] < 0 ? 0 : o->crop[0];
    c.y0 = o->crop[1] < 0 ? 0 : o->crop[1];
    c.x1 = o->crop[2] > s->width ? s->width : o->crop[2];
    c.y1 = o->crop[3] > s->height ? s->height : o->crop[3];
  }
  return c;
}

int reset_optimizer(jso_ctx* c, SceneGPU* s) {
  const size_t P = s->P;
  HIP_TRY(c, hipMemcpyAsync(s->params_prev, s->params, P * sizeof(float),
                            hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(s->mean, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->var, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->m2F, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->m2D, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, launch_fill_f64(s->alpha_prev, P, -HUGE_VAL, c->stream));
  HIP_TRY(c, hipMemsetAsync(s->adam_m, 0, P * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->adam_v, 0, P * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->F, 0, P * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->dF, 0, P * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->ctl, 0, sizeof(Ctl), c->stream));
  s->host_iter = 0;
  return JSO_OK;
}

hipMemcpyKind kind_to_dev(int mem) {
  return mem == JSO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}
hipMemcpyKind kind_from_dev(int mem) {
  return mem == JSO_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
}

// ---------------------------------------------------------------------------
// launch schedule
//
// Every path is traced by k_forward into a radiance slot; a primal image is
// then reduced from its slots by k_finalize, and an adjoint path is replayed
// by k_adjoint from its slot.  One k_forward launch fills at most kMaxSlots
// slots per pixel, so larger sample counts run in chunks: a chunk of primal
// samples is finalized (accumulated) before the next overwrites the slots,
// and the replay of a chunk of adjoint samples follows their forward launch.
// ---------------------------------------------------------------------------
struct PrimalSpec {
  const float* params;
  uint32_t tag;
  int spp;
  float* img;     // nullable
  float* delta;   // nullable
  double* loss2;  // nullable
};

struct AdjointSpec {
  const float* params;
  const float* params_b;  // null: single paths; else finite-difference pairs (+A - B)
  const float* delta;
  const float* delta_b;
  float* grad;
  float sign;
  uint32_t tag;
  int spp;
};

struct Schedule {
  jso_ctx* c;
  SceneGPU* s;
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  uint32_t flags;
};

FwdArgs fwd_args(const Schedule& q) {
  FwdArgs f{};
  f.key = q.key;
  f.crop = q.crop;
  f.mask = q.mask;
  f.slots = q.s->slots;
  f.npix = (uint32_t)q.s->npix;
  f.flags = q.flags;
  f.work = q.c->counting ? q.c->d_work : nullptr;
  return f;
}

RepArgs rep_args(const Schedule& q) {
  RepArgs r{};
  r.key = q.key;
  r.crop = q.crop;
  r.mask = q.mask;
  r.slots = q.s->slots;
  r.npix = (uint32_t)q.s->npix;
  r.flags = q.flags;
  r.work = q.c->counting ? q.c->d_work : nullptr;
  return r;
}

// One replay slice and the forward slices it needs.
struct RepUnit {
  int job, sample;
};

// Trace the primal images and reduce them; then trace and replay the adjoint
// samples.  The adjoint's forward slices share the last primal launch when
// they fit.
int run_schedule(const Schedule& q, const PrimalSpec* pj, int np, const AdjointSpec* aj, int na) {
  jso_ctx* c = q.c;
  SceneGPU* s = q.s;
  // replay units, pairs first: within a launch blocks are dispatched in slice
  // order and a pair block traces twice the paths of a single one
  std::vector<RepUnit> units;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < na; ++j)
      if ((aj[j].params_b != nullptr) == (pass == 0))
        for (int k = 0; k < aj[j].spp; ++k) units.push_back({j, k});
  size_t next_unit = 0;
  auto unit_slots = [&](const RepUnit& u) { return aj[u.job].params_b ? 2 : 1; };

  // primal samples in job order
  std::vector<std::pair<int, int>> prim;
  for (int j = 0; j < np; ++j)
    for (int k = 0; k < pj[j].spp; ++k) prim.push_back({j, k});
  size_t next_prim = 0;
  const FinArgs fin_base = [&] {
    FinArgs f{};
    f.slots = s->slots;
    f.npix = (uint32_t)s->npix;
    f.key = q.key;
    f.crop = q.crop;
    f.mask = q.mask;
    f.target = s->target;
    f.delta_scale = (float)(2.0 / (3.0 * (double)s->npix));
    f.loss_scale = 1.0 / (3.0 * (double)s->npix);
    return f;
  }();

  while (next_prim < prim.size() || next_unit < units.size()) {
    FwdArgs f = fwd_args(q);
    int n = 0;
    // primal slices of this launch
    FinArgs fin = fin_base;
    while (next_prim < prim.size() && n < kMaxSlots) {
      const int j = prim[next_prim].first, k = prim[next_prim].second;
      f.sl[n] = FwdSlice{pj[j].params, pj[j].tag, (uint32_t)k, n};
      if (fin.n_jobs == 0 || fin.jobs[fin.n_jobs - 1].slot0 + fin.jobs[fin.n_jobs - 1].n != n ||
          fin.jobs[fin.n_jobs - 1].accum != s->accum + (size_t)j * 3 * s->npix) {
        FinJob fj{};
        fj.slot0 = n;
        fj.n = 0;
        fj.accum = s->accum + (size_t)j * 3 * s->npix;
        fj.first = k == 0;
        fj.inv_spp = 1.0 / (double)pj[j].spp;
        fj.img = pj[j].img;
        fj.delta = pj[j].delta;
        fj.loss2 = pj[j].loss2;
        fin.jobs[fin.n_jobs++] = fj;
      }
      FinJob& fj = fin.jobs[fin.n_jobs - 1];
      fj.n++;
      fj.last = k == pj[j].spp - 1;
      ++n;
      ++next_prim;
    }
    // adjoint forward slices, once every primal sample has a slot
    RepArgs r = rep_args(q);
    int nr = 0;
    if (next_prim == prim.size()) {
      while (next_unit < units.size() && n + unit_slots(units[next_unit]) <= kMaxSlots) {
        const RepUnit u = units[next_unit++];
        const AdjointSpec& a = aj[u.job];
        RepSlice rs{};
        rs.params = a.params;
        rs.params_b = a.params_b;
        rs.delta = a.delta;
        rs.delta_b = a.delta_b;
        rs.grad = a.grad;
        rs.sign = a.sign;
        rs.adj_scale = (float)(1.0 / (double)a.spp);
        rs.tag = a.tag;
        rs.sample = (uint32_t)u.sample;
        rs.slot_a = n;
        f.sl[n++] = FwdSlice{a.params, a.tag, (uint32_t)u.sample, rs.slot_a};
        if (a.params_b) {
          rs.slot_b = n;
          f.sl[n++] = FwdSlice{a.params_b, a.tag, (uint32_t)u.sample, rs.slot_b};
        }
        r.sl[nr++] = rs;
      }
    }
    if (n == 0) return fail(c, JSO_E_INVALID, "schedule: empty launch");
    TIMED_LAUNCH(c, JSO_K_FORWARD, launch_forward(s->d_scene, f, n, c->stream));
    if (fin.n_jobs > 0)
      TIMED_LAUNCH(c, JSO_K_FINALIZE, launch_finalize(fin, s->width, c->stream));
    if (nr > 0)
      TIMED_LAUNCH(c, JSO_K_ADJOINT, launch_adjoint(s->d_scene, r, nr, s->n_ch, c->stream));
  }
  return JSO_OK;
}

// Queue the kernels of one gradient sample set.
//   prop:  F += <F_i> from spp_prop paths at params
//   fd:    dF += <dF_i> from spp_fd path pairs at (params, params_prev)
int queue_estimators(jso_ctx* c, SceneGPU* s, uint64_t seed, uint32_t iteration,
                     const uint32_t* iter_ptr, int spp_prop, int spp_fd, const float* params,
                     const float* params_prev, float* F, float* dF, float* img, double* loss2,
                     uint32_t prop_primal_tag, uint32_t prop_adj_tag, const Crop& crop,
                     const uint8_t* mask, uint32_t flags) {
  const size_t n3 = 3 * s->npix;
  float* d_prop = s->delta;
  float* d_cur = s->delta + n3;
  float* d_prev = s->delta + 2 * n3;
  const bool fd = dF != nullptr && spp_fd > 0;
  PrimalSpec pj[3];
  int np = 0;
  pj[np++] = PrimalSpec{params, prop_primal_tag, spp_prop, img, d_prop, loss2};
  if (fd) {
    pj[np++] = PrimalSpec{params, JSO_TAG_PRIMAL_FD, spp_fd, nullptr, d_cur, nullptr};
    pj[np++] = PrimalSpec{params_prev, JSO_TAG_PRIMAL_FD, spp_fd, nullptr, d_prev, nullptr};
  }
  AdjointSpec aj[2];
  int na = 0;
  aj[na++] = AdjointSpec{params, nullptr, d_prop, nullptr, F, 1.0f, prop_adj_tag, spp_prop};
  if (fd)
    aj[na++] = AdjointSpec{params, params_prev, d_cur, d_prev, dF, 1.0f, JSO_TAG_ADJ_FD, spp_fd};
  const Schedule q{c, s, KeyArgs{seed, iteration, iter_ptr}, crop, mask, flags};
  return run_schedule(q, pj, np, aj, na);
}

MetaArgs meta_args(SceneGPU* s, const float* F, const float* dF, float eta, float bF, float bD,
                   int zero_grads) {
  MetaArgs m{};
  m.params = s->params;
  m.params_prev = s->params_prev;
  m.F = const_cast<float*>(F);
  m.dF = const_cast<float*>(dF);
  m.mean = s->mean;
  m.var = s->var;
  m.alpha_prev = s->alpha_prev;
  m.m2F = s->m2F;
  m.m2D = s->m2D;
  m.ctl = s->ctl;
  m.partials = s->partials;
  m.n = s->P;
  m.n_ch = s->n_ch;
  for (int k = 0; k < 5; ++k) {
    m.lo[k] = s->lo[k];
    m.hi[k] = s->hi[k];
  }
  m.beta_F = bF;
  m.beta_D = bD;
  m.eta = eta;
  m.zero_grads = zero_grads;
  return m;
}

AdamArgs adam_args(SceneGPU* s, const float* g, float eta, float b1, float b2, float eps,
                   int zero_grads) {
  AdamArgs a{};
  a.params = s->params;
  a.params_prev = s->params_prev;
  a.g = const_cast<float*>(g);
  a.m = s->adam_m;
  a.v = s->adam_v;
  a.ctl = s->ctl;
  a.n = s->P;
  a.n_ch = s->n_ch;
  for (int k = 0; k < 5; ++k) {
    a.lo[k] = s->lo[k];
    a.hi[k] = s->hi[k];
  }
  a.eta = eta;
  a.beta1 = b1;
  a.beta2 = b2;
  a.eps = eps;
  a.zero_grads = zero_grads;
  return a;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int jso_create(jso_ctx** out, int device, void* stream) {
  if (!out) return JSO_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return JSO_E_UNSUPPORTED;
  if (device < 0 || device >= n) return JSO_E_INVALID;
  jso_ctx* c = new (std::nothrow) jso_ctx();
  if (!c) return JSO_E_OOM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  *out = c;
  return JSO_OK;
}

int jso_destroy(jso_ctx* c) {
  if (!c) return JSO_OK;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& s : c->scenes)
    if (s) free_scene_buffers(s.get());
  c->timer.destroy();
  if (c->d_work) (void)hipFree(c->d_work);
  delete c;
  return JSO_OK;
}

const char* jso_last_error(const jso_ctx* c) { return c ? c->err.c_str() : "null context"; }

int jso_set_stream(jso_ctx* c, void* stream) {
  if (!c) return JSO_E_INVALID;
  c->stream = (hipStream_t)stream;
  return JSO_OK;
}

int jso_synchronize(jso_ctx* c) {
  if (!c) return JSO_E_INVALID;
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return JSO_OK;
}

int jso_set_debug(jso_ctx* c, uint32_t flags) {
  if (!c) return JSO_E_INVALID;
  if (flags & ~15u) return fail(c, JSO_E_INVALID, "unknown debug flags 0x%x", flags);
  c->debug_flags = flags;
  return JSO_OK;
}

uint64_t jso_stream_key(uint64_t seed, uint32_t iteration, uint32_t tag) {
  return stream_key(seed, iteration, tag);
}

int jso_philox(jso_ctx* c, uint64_t key, const uint32_t* ctr, size_t n, uint32_t* out) {
  if (!c) return JSO_E_INVALID;
  if (n && (!ctr || !out)) return fail(c, JSO_E_INVALID, "null counter/output pointer");
  if (n > 0xFFFFFFFFull) return fail(c, JSO_E_INVALID, "too many counters");
  DeviceGuard g(c->device);
  HIP_TRY(c, launch_philox(ctr, n, key, out, c->stream));
  return JSO_OK;
}

int jso_load_scene(jso_ctx* c, const jso_scene_desc* d, int* scene_id) {
  if (!c || !d || !scene_id) return c ? fail(c, JSO_E_INVALID, "null argument") : JSO_E_INVALID;
  DeviceGuard g(c->device);
  std::unique_ptr<SceneGPU> s(new (std::nothrow) SceneGPU());
  if (!s) return fail(c, JSO_E_OOM, "host allocation failed");
  int rc = build_devscene(c, d, s.get());
  if (rc) return rc;
  const size_t P = s->P, n3 = 3 * s->npix;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  A(dalloc(&s->params, P));
  A(dalloc(&s->params_prev, P));
  A(dalloc(&s->target, n3));
  A(dalloc(&s->F, P));
  A(dalloc(&s->dF, P));
  A(dalloc(&s->delta, 3 * n3));
  A(dalloc(&s->mean, P));
  A(dalloc(&s->var, P));
  A(dalloc(&s->alpha_prev, P));
  A(dalloc(&s->m2F, P));
  A(dalloc(&s->m2D, P));
  A(dalloc(&s->adam_m, P));
  A(dalloc(&s->adam_v, P));
  A(dalloc(&s->ctl, 1));
  A(dalloc(&s->scratch_loss, 2));
  A(dalloc(&s->partials, kMetaMaxBlocks));
  A(dalloc(&s->slots, (size_t)kMaxSlots * n3));
  A(dalloc(&s->accum, 3 * n3));
  A(dalloc(&s->d_scene, 1));
  if (e != hipSuccess) {
    free_scene_buffers(s.get());
    return fail(c, e == hipErrorOutOfMemory ? JSO_E_OOM : JSO_E_HIP, "scene allocation: %s",
                hipGetErrorString(e));
  }
  // initial parameters: 0.5 for every channel (roughness within its box)
  rc = JSO_OK;
  if (launch_fill_f32(s->params, P, 0.5f, c->stream) != hipSuccess ||
      hipMemsetAsync(s->target, 0, n3 * sizeof(float), c->stream) != hipSuccess ||
      hipMemcpy(s->d_scene, &s->dev, sizeof(DevScene), hipMemcpyHostToDevice) != hipSuccess) {
    free_scene_buffers(s.get());
    return fail(c, JSO_E_HIP, "scene initialisation failed");
  }
  rc = reset_optimizer(c, s.get());
  if (rc) {
    free_scene_buffers(s.get());
    return rc;
  }
  c->scenes.push_back(std::move(s));
  *scene_id = (int)c->scenes.size() - 1;
  return JSO_OK;
}

int jso_free_scene(jso_ctx* c, int id) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  free_scene_buffers(s);
  c->scenes[id].reset();
  return JSO_OK;
}

int jso_scene_info(jso_ctx* c, int id, size_t* n_params, int* width, int* height) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (n_params) *n_params = s->P;
  if (width) *width = s->width;
  if (height) *height = s->height;
  return JSO_OK;
}

int jso_set_params(jso_ctx* c, int id, const float* p, size_t n, int mem) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!p || n != s->P) return fail(c, JSO_E_INVALID, "params: need %zu values", s->P);
  DeviceGuard g(c->device);
  HIP_TRY(c, hipMemcpyAsync(s->params, p, n * sizeof(float), kind_to_dev(mem), c->stream));
  if (mem != JSO_MEM_DEVICE) HIP_TRY(c, hipStreamSynchronize(c->stream));
  return reset_optimizer(c, s);
}

static int get_vec(jso_ctx* c, int id, float* p, size_t n, int mem, bool prev) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!p || n != s->P) return fail(c, JSO_E_INVALID, "params: need %zu values", s->P);
  DeviceGuard g(c->device);
  HIP_TRY(c, hipMemcpyAsync(p, prev ? s->params_prev : s->params, n * sizeof(float),
                            kind_from_dev(mem), c->stream));
  if (mem != JSO_MEM_DEVICE) HIP_TRY(c, hipStreamSynchronize(c->stream));
  return JSO_OK;
}

int jso_get_params(jso_ctx* c, int id, float* p, size_t n, int mem) {
  return get_vec(c, id, p, n, mem, false);
}

int jso_get_params_prev(jso_ctx* c, int id, float* p, size_t n, int mem) {
  return get_vec(c, id, p, n, mem, true);
}

int jso_set_target(jso_ctx* c, int id, const float* img, size_t n, int mem) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!img || n != 3 * s->npix) return fail(c, JSO_E_INVALID, "target: need %zu values", 3 * s->npix);
  DeviceGuard g(c->device);
  HIP_TRY(c, hipMemcpyAsync(s->target, img, n * sizeof(float), kind_to_dev(mem), c->stream));
  if (mem != JSO_MEM_DEVICE) HIP_TRY(c, hipStreamSynchronize(c->stream));
  return JSO_OK;
}

int jso_render(jso_ctx* c, int id, const float* params, uint64_t seed, uint32_t iteration,
               uint32_t tag, int spp, const jso_render_opts* opts, float* img) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!params || !img) return fail(c, JSO_E_INVALID, "null params/img");
  if (spp < 1) return fail(c, JSO_E_INVALID, "spp must be >= 1");
  DeviceGuard g(c->device);
  const PrimalSpec pj{params, tag, spp, img, nullptr, nullptr};
  const Schedule q{c, s, KeyArgs{seed, iteration, nullptr}, crop_of(s, opts),
                   opts ? opts->pixel_mask : nullptr, c->debug_flags | (opts ? opts->flags : 0u)};
  return run_schedule(q, &pj, 1, nullptr, 0);
}

int jso_render_bwd(jso_ctx* c, int id, const float* params, uint64_t seed, uint32_t iteration,
                   uint32_t tag, int spp, const float* dimg, const jso_render_opts* opts,
                   float* dparams) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!params || !dimg || !dparams) return fail(c, JSO_E_INVALID, "null argument");
  if (spp < 1) return fail(c, JSO_E_INVALID, "spp must be >= 1");
  DeviceGuard g(c->device);
  const AdjointSpec aj{params, nullptr, dimg, nullptr, dparams, 1.0f, tag, spp};
  const Schedule q{c, s, KeyArgs{seed, iteration, nullptr}, crop_of(s, opts),
                   opts ? opts->pixel_mask : nullptr, c->debug_flags | (opts ? opts->flags : 0u)};
  return run_schedule(q, nullptr, 0, &aj, 1);
}

int jso_estimate_gradients(jso_ctx* c, int id, uint64_t seed, uint32_t iteration, int spp_prop,
                           int spp_fd, const jso_render_opts* opts, float* F, float* dF,
                           float* img, double* loss) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!F) return fail(c, JSO_E_INVALID, "null F");
  if (spp_prop < 1 || spp_prop > 64 || spp_fd < 0 || spp_fd > 64)
    return fail(c, JSO_E_INVALID, "spp out of range");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipMemsetAsync(s->scratch_loss, 0, 2 * sizeof(double), c->stream));
  int rc = queue_estimators(c, s, seed, iteration, nullptr, spp_prop, spp_fd, s->params,
                            s->params_prev, F, dF, img, s->scratch_loss, JSO_TAG_PRIMAL_PROP,
                            JSO_TAG_ADJ_PROP, crop_of(s, opts), opts ? opts->pixel_mask : nullptr,
                            c->debug_flags | (opts ? opts->flags : 0u));
  if (rc) return rc;
  if (loss) {
    double l2[2];
    HIP_TRY(c, hipMemcpyAsync(l2, s->scratch_loss, sizeof(l2), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *loss = l2[iteration & 1u];
  }
  return JSO_OK;
}

int jso_meta_step(jso_ctx* c, int id, const float* F, const float* dF, float eta, float beta_F,
                  float beta_D) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!F || !dF) return fail(c, JSO_E_INVALID, "null F/dF");
  if (!(beta_F >= 0.0f && beta_F < 1.0f && beta_D >= 0.0f && beta_D < 1.0f))
    return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
  DeviceGuard g(c->device);
  TIMED_LAUNCH(c, JSO_K_META, launch_meta(meta_args(s, F, dF, eta, beta_F, beta_D, 0), c->stream));
  s->host_iter++;
  return JSO_OK;
}

int jso_adam_step(jso_ctx* c, int id, const float* grad, float eta, float beta1, float beta2,
                  float eps) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!grad) return fail(c, JSO_E_INVALID, "null gradient");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
    return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
  DeviceGuard g(c->device);
  TIMED_LAUNCH(c, JSO_K_ADAM, launch_adam(adam_args(s, grad, eta, beta1, beta2, eps, 0), c->stream));
  s->host_iter++;
  return JSO_OK;
}

int jso_grad_step(jso_ctx* c, const int* ids, int n, const jso_step_opts* o,
                  jso_step_stats* stats) {
  if (!c) return JSO_E_INVALID;
  if (!ids || n <= 0 || !o) return fail(c, JSO_E_INVALID, "null/empty argument");
  for (int k = 0; k < n; ++k)
    if (!get_scene(c, ids[k])) return fail(c, JSO_E_INVALID, "bad scene id %d", ids[k]);
  DeviceGuard g(c->device);
  const uint32_t flags = c->debug_flags | o->flags;
  for (int k = 0; k < n; ++k) {
    SceneGPU* s = get_scene(c, ids[k]);
    const Crop full{0, 0, s->width, s->height};
    if (o->optimizer == JSO_OPT_META) {
      if (o->spp_prop < 1 || o->spp_prop > 64 || o->spp_fd < 0 || o->spp_fd > 64)
        return fail(c, JSO_E_INVALID, "spp out of range");
      if (!(o->beta_F >= 0.0f && o->beta_F < 1.0f && o->beta_D >= 0.0f && o->beta_D < 1.0f))
        return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
      int rc = queue_estimators(c, s, o->seed, s->host_iter, &s->ctl->iteration, o->spp_prop,
                                o->spp_fd, s->params, s->params_prev, s->F, s->dF, nullptr,
                                s->ctl->loss, JSO_TAG_PRIMAL_PROP, JSO_TAG_ADJ_PROP, full,
                                nullptr, flags);
      if (rc) return rc;
      TIMED_LAUNCH(c, JSO_K_META,
                   launch_meta(meta_args(s, s->F, s->dF, o->eta, o->beta_F, o->beta_D, 1),
                               c->stream));
    } else if (o->optimizer == JSO_OPT_ADAM) {
      if (o->adam_spp < 1 || o->adam_spp > 4096) return fail(c, JSO_E_INVALID, "adam_spp");
      if (!(o->adam_beta1 >= 0.0f && o->adam_beta1 < 1.0f && o->adam_beta2 >= 0.0f &&
            o->adam_beta2 < 1.0f))
        return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
      int rc = queue_estimators(c, s, o->seed, s->host_iter, &s->ctl->iteration, o->adam_spp, 0,
                                s->params, s->params_prev, s->F, nullptr, nullptr, s->ctl->loss,
                                JSO_TAG_ADAM_PRIMAL, JSO_TAG_ADAM_ADJ, full, nullptr, flags);
      if (rc) return rc;
      TIMED_LAUNCH(c, JSO_K_ADAM,
                   launch_adam(adam_args(s, s->F, o->eta, o->adam_beta1, o->adam_beta2,
                                         o->adam_eps, 1),
                               c->stream));
    } else {
      return fail(c, JSO_E_INVALID, "unknown optimizer %d", o->optimizer);
    }
    s->host_iter++;
  }
  if (stats) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) {
      SceneGPU* s = get_scene(c, ids[k]);
      Ctl h;
      HIP_TRY(c, hipMemcpy(&h, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
      const uint32_t done = h.iteration - 1u;  // the iteration just completed
      stats[k].loss = h.loss[done & 1u];
      stats[k].step_norm2 = h.norm2[h.iteration & 1u];
      stats[k].iteration = h.iteration;
    }
  }
  return JSO_OK;
}

int jso_set_timing(jso_ctx* c, int enable) {
  if (!c) return JSO_E_INVALID;
  DeviceGuard g(c->device);
  HIP_TRY(c, c->timer.collect());
  c->timer.enabled = enable != 0;
  return JSO_OK;
}

int jso_get_kernel_time(jso_ctx* c, int kernel, double* ms, uint64_t* launches, int reset) {
  if (!c) return JSO_E_INVALID;
  if (kernel < 0 || kernel >= JSO_K_COUNT) return fail(c, JSO_E_INVALID, "bad kernel class");
  DeviceGuard g(c->device);
  HIP_TRY(c, c->timer.collect());
  if (ms) *ms = c->timer.ms[kernel];
  if (launches) *launches = c->timer.launches[kernel];
  if (reset) {
    c->timer.ms[kernel] = 0.0;
    c->timer.launches[kernel] = 0;
  }
  return JSO_OK;
}

int jso_set_work_counting(jso_ctx* c, int enable) {
  if (!c) return JSO_E_INVALID;
  DeviceGuard g(c->device);
  if (enable && !c->d_work) {
    HIP_TRY(c, hipMalloc(&c->d_work, 4 * sizeof(unsigned long long)));
    HIP_TRY(c, hipMemset(c->d_work, 0, 4 * sizeof(unsigned long long)));
  }
  c->counting = enable != 0;
  return JSO_OK;
}

int jso_get_work(jso_ctx* c, uint64_t out[4], int reset) {
  if (!c) return JSO_E_INVALID;
  if (!out) return fail(c, JSO_E_INVALID, "null output");
  out[0] = out[1] = out[2] = out[3] = 0;
  if (!c->d_work) return JSO_OK;
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  unsigned long long h[4];
  HIP_TRY(c, hipMemcpy(h, c->d_work, sizeof(h), hipMemcpyDeviceToHost));
  for (int k = 0; k < 4; ++k) out[k] = h[k];
  if (reset) HIP_TRY(c, hipMemset(c->d_work, 0, sizeof(h)));
  return JSO_OK;
}

int jso_get_state(jso_ctx* c, int id, jso_state* st) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!st) return fail(c, JSO_E_INVALID, "null state");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t P = s->P;
  struct {
    void* h;
    const void* d;
    size_t bytes;
  } cp[] = {{st->params, s->params, P * 4},      {st->params_prev, s->params_prev, P * 4},
            {st->mean, s->mean, P * 8},          {st->var, s->var, P * 8},
            {st->alpha_prev, s->alpha_prev, P * 8}, {st->m2_F, s->m2F, P * 8},
            {st->m2_D, s->m2D, P * 8},           {st->adam_m, s->adam_m, P * 4},
            {st->adam_v, s->adam_v, P * 4}};
  for (auto& x : cp)
    if (x.h) HIP_TRY(c, hipMemcpy(x.h, x.d, x.bytes, hipMemcpyDeviceToHost));
  Ctl h;
  HIP_TRY(c, hipMemcpy(&h, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
  st->iteration = h.iteration;
  st->count_F = h.count_F;
  st->count_D = h.count_D;
  st->adam_t = h.adam_t;
  st->step_norm2 = h.norm2[h.iteration & 1u];
  return JSO_OK;
}

int jso_set_state(jso_ctx* c, int id, const jso_state* st) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!st || !st->params || !st->params_prev || !st->mean || !st->var || !st->alpha_prev ||
      !st->m2_F || !st->m2_D || !st->adam_m || !st->adam_v)
    return fail(c, JSO_E_INVALID, "state view must provide every buffer");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t P = s->P;
  struct {
    void* d;
    const void* h;
    size_t bytes;
  } cp[] = {{s->params, st->params, P * 4},      {s->params_prev, st->params_prev, P * 4},
            {s->mean, st->mean, P * 8},          {s->var, st->var, P * 8},
            {s->alpha_prev, st->alpha_prev, P * 8}, {s->m2F, st->m2_F, P * 8},
            {s->m2D, st->m2_D, P * 8},           {s->adam_m, st->adam_m, P * 4},
            {s->adam_v, st->adam_v, P * 4}};
  for (auto& x : cp) HIP_TRY(c, hipMemcpy(x.d, x.h, x.bytes, hipMemcpyHostToDevice));
  Ctl h{};
  h.iteration = st->iteration;
  h.count_F = st->count_F;
  h.count_D = st->count_D;
  h.adam_t = st->adam_t;
  h.norm2[st->iteration & 1u] = st->step_norm2;
  HIP_TRY(c, hipMemcpy(s->ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemset(s->F, 0, P * sizeof(float)));
  HIP_TRY(c, hipMemset(s->dF, 0, P * sizeof(float)));
  s->host_iter = st->iteration;
  return JSO_OK;
}

}  // extern "C"

// Host runtime of libjso: contexts, scene upload, buffers, and the C ABI
// declared in include/jso.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bvh.h"
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
  float* bvh_nodes = nullptr;      // mesh hierarchy (layout of bvh.h)
  float* bvh_tris = nullptr;
  int* bvh_tri_id = nullptr;
  int stack = 0;                   // traversal-stack entries its mesh needs (0: no mesh)
  // texture-gradient preconditioner (textures larger than 1x1): orthonormal
  // cosine-transform matrices C_W (W x W), C_H (H x H) and the eigenvalues of
  // the path-graph Laplacians, 2 - 2 cos(pi k / n), for both axes
  float* pc = nullptr;
  float* pc_tmp = nullptr;         // 2 x P scratch (one per gradient vector)
  // meta-estimator ablations: first moments of centred variance EMAs, and
  // the separate variance samples of the uncorrelated ablation
  double *m1F = nullptr, *m1D = nullptr;
  float *Fv = nullptr, *dFv = nullptr;
  unsigned long long* fx = nullptr;  // deterministic mode: 2 x P fixed-point accumulators
  // volumes: the bricked copies of up to 2 parameter vectors that the volume
  // kernels read (BrickArgs), made at the start of each plan; brick_n floats each
  float* vbrick = nullptr;
  size_t brick_n = 0;
  // triangle meshes: hit records of replayed paths (kHitRecs x kRecWords
  // words per slot and pixel), written by the forward pass of a plan, read by
  // its replay
  uint32_t* recs = nullptr;
  uint32_t host_iter = 0;          // mirror of ctl->iteration
  uint64_t generation = 0;         // unique per loaded scene (plan cache key)
};

}  // namespace

// Source of SceneGPU::generation.
std::atomic<uint64_t> g_scene_generation{0};
// Hit-record epoch: one value per estimator plan, mixed into its records' tags.
std::atomic<uint32_t> g_rec_epoch{0};

// Tile shapes picked by the autotuner, by (GPU architecture, configuration
// hash); shared by every context of the process.
std::mutex g_tuned_mu;
std::map<std::pair<std::string, uint64_t>, int> g_tuned;

// Scratch memory of jso_render_bwd_noalloc (the forward radiance slots of
// the replayed paths), a file-scope device array: every GPU the library runs
// on holds its own copy until the process ends, and every call on that GPU
// shares it.  Host code never passes the array's name to a kernel (on the
// host it is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returned on that device, kept per device below.
constexpr size_t kNoAllocScratchBytes = JSO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch_ptr;  // device -> address of `scratch` there

// Look up (once per device, with `device` current) the device address of
// `scratch`; *out = null and an error code on failure.
hipError_t scratch_address(int device, uint8_t** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    *out = nullptr;
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  *out = static_cast<uint8_t*>(ptr);
  g_scratch_ptr[device] = *out;
  return hipSuccess;
}

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

// Device copies of launch descriptors (unit arrays).  A host-built array is
// staged in pinned memory and copied on the context's stream; a slot is
// reused only once the event recorded behind its copy has completed.
struct DescRing {
  static constexpr int kSlots = 64;
  static constexpr size_t kSlotBytes = 64 * 1024;
  uint8_t* host = nullptr;  // pinned
  uint8_t* dev = nullptr;
  hipEvent_t ev[kSlots] = {};
  bool pending[kSlots] = {};
  int next = 0;

  hipError_t init() {
    if (host) return hipSuccess;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host), kSlots * kSlotBytes, 0);
    if (e != hipSuccess) return e;
    e = hipMalloc(reinterpret_cast<void**>(&dev), kSlots * kSlotBytes);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kSlots; ++k) {
      e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // copy `bytes` to device memory in stream order; *out = its device address
  hipError_t put(const void* src, size_t bytes, hipStream_t st, const void** out) {
    if (bytes > kSlotBytes) return hipErrorInvalidValue;
    hipError_t e = init();
    if (e != hipSuccess) return e;
    const int k = next;
    next = (next + 1) % kSlots;
    if (pending[k]) {
      e = hipEventSynchronize(ev[k]);
      if (e != hipSuccess) return e;
    }
    std::memcpy(host + (size_t)k * kSlotBytes, src, bytes);
    e = hipMemcpyAsync(dev + (size_t)k * kSlotBytes, host + (size_t)k * kSlotBytes, bytes,
                       hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ev[k], st);
    if (e != hipSuccess) return e;
    pending[k] = true;
    *out = dev + (size_t)k * kSlotBytes;
    return hipSuccess;
  }
  void destroy() {
    for (int k = 0; k < kSlots; ++k)
      if (ev[k]) {
        if (pending[k]) (void)hipEventSynchronize(ev[k]);
        (void)hipEventDestroy(ev[k]);
      }
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
  }
};

// The plan of the last grad_step, its unit arrays kept in device memory: a
// step repeated with the same problems and options launches from them
// directly.  `sig` identifies the plan (scenes by load generation, options,
// flags); launch records keep their metadata, their units live on the device.
struct CachedLaunch {
  int kind, timer, shape, n, stack;
  bool shared, vol;
  uint32_t blocks;
  size_t lds, offset;
  int persist;
  bool det;
  int waves;
};

struct CachedPlan {
  std::vector<uint64_t> sig;
  std::vector<CachedLaunch> launches;
  uint8_t* dev = nullptr;   // unit arrays
  uint8_t* host = nullptr;  // pinned staging copy (source of the upload)
  uint32_t* queues = nullptr;  // two work-queue counters per launch (persistent launches)
  uint64_t last_use = 0;
};

struct PlanCache {
  static constexpr size_t kMaxPlans = 64;
  std::vector<CachedPlan> plans;
  uint64_t clock = 0;
  static void release(CachedPlan& p) {
    if (p.dev) (void)hipFree(p.dev);
    if (p.host) (void)hipHostFree(p.host);
    if (p.queues) (void)hipFree(p.queues);
    p.dev = p.host = nullptr;
    p.queues = nullptr;
  }
  void destroy() {
    for (CachedPlan& p : plans) release(p);
    plans.clear();
  }
};

struct jso_ctx {
  DescRing ring;
  PlanCache plan_cache;
  std::string arch;     // gcnArchName of the device
  int launch_config = 0;  // default launch configuration when the tuner has no entry
  int n_cu = 0;           // compute units of the device
  int device = 0;
  hipStream_t stream = nullptr;  // nullptr = the device's null (default) stream
  uint32_t debug_flags = 0;
  std::string err;
  std::vector<std::unique_ptr<SceneGPU>> scenes;
  KernelTimer timer;
  unsigned long long* d_work = nullptr;  // work counters (replay paths/vertices, forward paths/vertices)
  bool counting = false;
  uint8_t* scratch = nullptr;  // this device's `scratch` (set up by jso_create)
};

namespace jso {
// The context's stream and device, for the microbenchmarks (ubench.hip).
hipStream_t ctx_stream(jso_ctx* c) { return c->stream; }
int ctx_device(jso_ctx* c) { return c->device; }
}  // namespace jso

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
                  s->partials, s->slots,     s->accum,  s->d_scene, s->bvh_nodes,
                  s->bvh_tris, s->bvh_tri_id, s->pc, s->pc_tmp, s->m1F,
                  s->m1D,    s->Fv,          s->dFv,    s->fx,     s->vbrick, s->recs};
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
  if (d->n_tris < 0 || d->n_tris > JSO_MAX_TRIS || d->n_verts < 0 ||
      (d->n_tris > 0 && (!d->tris || !d->verts || d->n_verts == 0)))
    return fail(c, JSO_E_INVALID, "mesh of %d triangles invalid (max %d)", d->n_tris,
                JSO_MAX_TRIS);
  if (d->n_tris > 0 && !check_mat(d->mesh_mat))
    return fail(c, JSO_E_INVALID, "mesh material %d invalid", d->mesh_mat);
  if (d->param_layout == JSO_LAYOUT_VERTEX) {
    if (d->n_tris == 0 || d->mesh_mat != JSO_MAT_PARAM)
      return fail(c, JSO_E_INVALID, "per-vertex parameters need a mesh with JSO_MAT_PARAM");
    bool other = d->plane_enabled && d->plane_mat == JSO_MAT_PARAM;
    for (int k = 0; k < d->n_spheres; ++k)
      other = other || (d->sphere_mat ? d->sphere_mat[k] : JSO_MAT_PARAM) == JSO_MAT_PARAM;
    if (other)
      return fail(c, JSO_E_INVALID, "with per-vertex parameters only the mesh may use them");
  } else if (d->param_layout == JSO_LAYOUT_VOLUME) {
    if (d->vol_res < 1 || d->vol_res > JSO_MAX_VOL_RES)
      return fail(c, JSO_E_INVALID, "vol_res %d invalid (max %d)", d->vol_res, JSO_MAX_VOL_RES);
    if (d->vol_views < 1 || d->vol_views > JSO_MAX_VIEWS || d->height % d->vol_views != 0)
      return fail(c, JSO_E_INVALID, "vol_views %d invalid (max %d, must divide the height)",
                  d->vol_views, JSO_MAX_VIEWS);
    if (!(d->vol_box[3] > 0.0f) || !std::isfinite(d->vol_box[3]) || !(d->vol_sigma >= 0.0f) ||
        !std::isfinite(d->vol_sigma))
      return fail(c, JSO_E_INVALID, "volume box side and density scale must be finite, >0/>=0");
    if (d->ch_mask != 15)
      return fail(c, JSO_E_INVALID, "a volume has the 4 channels emission RGB + density "
                                    "(ch_mask 15)");
    if (d->plane_enabled || d->n_spheres > 0 || d->n_tris > 0 || d->light_enabled)
      return fail(c, JSO_E_INVALID, "a volume scene has no plane, spheres, mesh or light");
  } else if (d->param_layout != JSO_LAYOUT_TEXTURE) {
    return fail(c, JSO_E_INVALID, "param_layout %d invalid", d->param_layout);
  }

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
  S.n_tris = d->n_tris;
  S.mesh_mat = d->n_tris > 0 ? d->mesh_mat : 0;
  S.layout = d->param_layout;
  s->npix = (size_t)d->width * d->height;
  s->P = (d->param_layout == JSO_LAYOUT_VERTEX ? (size_t)d->n_verts
                                               : (size_t)d->tex_w * d->tex_h) * nc;
  if (d->param_layout == JSO_LAYOUT_VOLUME) {
    const size_t R = (size_t)d->vol_res;
    s->P = R * R * R * 4;
    S.vol_res = d->vol_res;
    S.vol_rb = (d->vol_res + 3) / 4;
    s->brick_n = (size_t)S.vol_rb * S.vol_rb * S.vol_rb * 64 * 4;
    S.vol_views = d->vol_views;
    S.view_h = d->height / d->vol_views;
    for (int k = 0; k < 3; ++k) S.vol_lo[k] = d->vol_box[k];
    S.vol_side = d->vol_box[3];
    S.vol_inv_vox = (float)((double)d->vol_res / (double)d->vol_box[3]);
    S.vol_sigma = d->vol_sigma;
    S.aspect = (float)((double)d->width / (double)S.view_h);
    // view v: the eye turned by 2 pi v / V about the vertical axis through the
    // target (bases in double, stored as float)
    for (int v = 0; v < d->vol_views; ++v) {
      const double ang = 2.0 * M_PI * v / d->vol_views, ca = std::cos(ang), sa = std::sin(ang);
      const double r[3] = {(double)d->cam_eye[0] - d->cam_target[0], 0.0,
                           (double)d->cam_eye[2] - d->cam_target[2]};
      const double ev[3] = {d->cam_target[0] + r[0] * ca + r[2] * sa, (double)d->cam_eye[1],
                            d->cam_target[2] - r[0] * sa + r[2] * ca};
      double wv[3] = {d->cam_target[0] - ev[0], d->cam_target[1] - ev[1],
                      d->cam_target[2] - ev[2]};
      const double wn = std::sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
      for (double& x : wv) x /= wn;
      double uv[3] = {wv[1] * up[2] - wv[2] * up[1], wv[2] * up[0] - wv[0] * up[2],
                      wv[0] * up[1] - wv[1] * up[0]};
      const double un = std::sqrt(uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2]);
      if (!(un > 0)) return fail(c, JSO_E_INVALID, "camera up parallel to view %d", v);
      for (double& x : uv) x /= un;
      const double vv[3] = {uv[1] * wv[2] - uv[2] * wv[1], uv[2] * wv[0] - uv[0] * wv[2],
                            uv[0] * wv[1] - uv[1] * wv[0]};
      for (int k = 0; k < 3; ++k) {
        S.view_eye[v][k] = (float)ev[k];
        S.view_cw[v][k] = (float)wv[k];
        S.view_cu[v][k] = (float)uv[k];
        S.view_cv[v][k] = (float)vv[k];
      }
    }
  }
  return JSO_OK;
}

// Build the mesh hierarchy on the host and upload it; fills the scene's
// device pointers.
// Tables of the texture-gradient preconditioner: the orthonormal DCT-II
// matrices of both texture axes (row k: s_k cos(pi k (i + 1/2) / n)), which
// diagonalise the Laplacians of the path graphs along the axes, and their
// eigenvalues 2 - 2 cos(pi k / n).
int upload_precond(jso_ctx* c, SceneGPU* s) {
  const DevScene& S = s->dev;
  if (S.layout != JSO_LAYOUT_TEXTURE || S.tex_w * S.tex_h <= 1) return JSO_OK;
  const int W = S.tex_w, H = S.tex_h;
  std::vector<float> t((size_t)W * W + (size_t)H * H + W + H);
  auto fill = [](float* m, float* eig, int n) {
    for (int k = 0; k < n; ++k) {
      const double sk = std::sqrt((k == 0 ? 1.0 : 2.0) / n);
      for (int i = 0; i < n; ++i) m[(size_t)k * n + i] = (float)(sk * std::cos(M_PI * k * (i + 0.5) / n));
      eig[k] = (float)(2.0 - 2.0 * std::cos(M_PI * k / n));
    }
  };
  float* cw = t.data();
  float* ch = cw + (size_t)W * W;
  float* mu = ch + (size_t)H * H;
  float* nu = mu + W;
  fill(cw, mu, W);
  fill(ch, nu, H);
  hipError_t e = dalloc(&s->pc, t.size());
  if (e == hipSuccess) e = dalloc(&s->pc_tmp, 2 * s->P);
  if (e == hipSuccess)
    e = hipMemcpy(s->pc, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess)
    return fail(c, e == hipErrorOutOfMemory ? JSO_E_OOM : JSO_E_HIP, "preconditioner: %s",
                hipGetErrorString(e));
  return JSO_OK;
}

int upload_mesh(jso_ctx* c, const jso_scene_desc* d, SceneGPU* s) {
  if (d->n_tris == 0) return JSO_OK;
  BvhBuild b;
  const std::string err = build_bvh(d->verts, d->n_verts, d->tris, d->n_tris, b);
  if (!err.empty()) return fail(c, JSO_E_INVALID, "%s", err.c_str());
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  A(dalloc(&s->bvh_nodes, b.nodes4.size() * (sizeof(Bvh4Node) / sizeof(float))));
  A(dalloc(&s->bvh_tris, b.tris.size()));
  A(dalloc(&s->bvh_tri_id, b.order.size()));
  if (e == hipSuccess) {
    A(hipMemcpy(s->bvh_nodes, b.nodes4.data(), b.nodes4.size() * sizeof(Bvh4Node),
                hipMemcpyHostToDevice));
    A(hipMemcpy(s->bvh_tris, b.tris.data(), b.tris.size() * sizeof(float),
                hipMemcpyHostToDevice));
    A(hipMemcpy(s->bvh_tri_id, b.order.data(), b.order.size() * sizeof(int32_t),
                hipMemcpyHostToDevice));
  }
  if (e != hipSuccess)
    return fail(c, e == hipErrorOutOfMemory ? JSO_E_OOM : JSO_E_HIP, "mesh upload: %s",
                hipGetErrorString(e));
  DevScene& S = s->dev;
  S.bvh_nodes = gmem((const float4*)s->bvh_nodes);
  S.bvh_tris = gmem((const float4*)s->bvh_tris);
  S.bvh_tri_id = gmem((const int*)s->bvh_tri_id);
  S.bvh_depth = b.depth4;
  s->stack = b.stack4;
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
  HIP_TRY(c, hipMemsetAsync(s->m1F, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->m1D, 0, P * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->Fv, 0, P * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(s->dFv, 0, P * sizeof(float), c->stream));
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
// launch plans
//
// Every path is traced by k_forward into a radiance slot; a primal image is
// then reduced from its slots by k_finalize, and an adjoint path is replayed
// by k_adjoint from its slot.  One k_forward launch fills at most kMaxSlots
// slots per pixel, so larger sample counts run in chunks: a chunk of primal
// samples is finalized (accumulated) before the next overwrites the slots,
// and the replay of a chunk of adjoint samples follows their forward launch.
//
// A plan is the launch sequence of one step for one or more problems with
// the same estimator configuration: each launch carries one unit per problem
// (or per slice group), so a single launch serves all of them.
// ---------------------------------------------------------------------------
// A launch configuration of the path kernels: a tile shape (kShapeW/kShapeH)
// and a persistent grid of kPersistPerCU[...] blocks per compute unit pulling
// tiles from a work queue (0: one block per tile).
constexpr int kPersistPerCU[] = {0, 1, 2, 4, 8};
constexpr int kConfigs = kShapes * (int)(sizeof(kPersistPerCU) / sizeof(int));
static_assert(kConfigs == JSO_LAUNCH_CONFIGS, "launch configurations");
int shape_of(int config) { return config % kShapes; }
int persist_of(int config) { return kPersistPerCU[config / kShapes]; }

struct PrimalSpec {
  const float* params;
  uint32_t tag;
  int spp;
  float* img;     // nullable
  float* delta;   // nullable
  double* loss2;  // nullable
  // shared-path pair: the paths drawn at `params` are also evaluated at
  // params_b, whose adjoint image goes to delta_b (its loss is not reported)
  const float* params_b = nullptr;
  float* delta_b = nullptr;
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
  bool shared = false;    // pair: one path drawn at A, evaluated at A and B (Eq. 5)
};

// One problem's part of a plan.
struct ProbPlan {
  SceneGPU* s;
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  uint32_t flags;
  uint32_t max_iter;  // 0: always active
  int relative;       // relative loss (JSO_LOSS_RELATIVE)
  PrimalSpec pj[3];
  int np;
  AdjointSpec aj[2];
  int na;
  double* slots = nullptr;  // radiance slots; null: the scene's own
  double fx_scale = 0.0;    // deterministic mode: fixed-point scale (see fx_scale_of)
};

double* slots_of(const ProbPlan& p) { return p.slots ? p.slots : p.s->slots; }
// The hit records go with the scene's own slots (none with a caller's slots).
uint32_t* recs_of(const ProbPlan& p) { return p.slots ? nullptr : p.s->recs; }

// Fixed-point scale of the deterministic mode: 2^32 for adjoint images of the
// caller's (jso_render_bwd), 2^(32 + ceil(log2(1.5 W H))) for the estimators,
// whose adjoint images carry the loss's 1 / (1.5 W H).
double fx_scale_of(const SceneGPU* s, bool estimator) {
  if (!estimator) return std::ldexp(1.0, 32);
  return std::ldexp(1.0, 32 + (int)std::ceil(std::log2(1.5 * (double)s->npix)));
}

enum class Kern { Forward, Finalize, Adjoint, Meta, Adam, Dct, FxFlush, Brick };

struct LaunchRec {
  Kern kind;
  int timer;                   // JSO_K_* class
  int shape = 0;               // path kernels: tile shape (kShapeW / kShapeH)
  std::vector<uint8_t> units;  // host copy of the unit array
  int n = 0;
  uint32_t blocks = 0;
  size_t lds = 0;
  int stack = 0;               // path kernels: BVH stack entries (deepest mesh of the units)
  bool shared = false;         // path kernels: units hold shared-path pair slices
  bool vol = false;            // path kernels: the units' scenes are volumes
  int persist = 0;             // path kernels: persistent blocks per CU (0: none)
  bool det = false;            // adjoint: deterministic mode (fixed-point sums)
  int waves = 0;               // volume forward: slices (waves) per block
  size_t dev_offset = 0;       // batches: offset of the units in the device arena
};

using Plan = std::vector<LaunchRec>;

template <class U>
void push_unit(LaunchRec& r, U u, uint32_t blocks) {
  u.h.block0 = r.blocks;
  const size_t off = r.units.size();
  r.units.resize(off + sizeof(U));
  std::memcpy(r.units.data() + off, &u, sizeof(U));
  r.n++;
  r.blocks += blocks;
}

uint32_t tiles_x(const Crop& c, int shape) {
  return (uint32_t)((c.x1 - c.x0 + kShapeW[shape] - 1) / kShapeW[shape]);
}
uint32_t tiles_of(const Crop& c, int shape) {
  return tiles_x(c, shape) * (uint32_t)((c.y1 - c.y0 + kShapeH[shape] - 1) / kShapeH[shape]);
}

// Tiles of half the shape's height (replay pairs on lane pairs).
uint32_t pair_tiles_of(const Crop& c, int shape) {
  const int h = kShapeH[shape] / 2;
  return tiles_x(c, shape) * (uint32_t)((c.y1 - c.y0 + h - 1) / h);
}

bool crop_empty(const Crop& c) { return c.x1 <= c.x0 || c.y1 <= c.y0; }

// The launches of the estimator part of a step for problems `ps` (all with the
// same job structure), with pixel tiles of the given shape and at most
// max_slots radiance slots per pixel per launch (a replay pair needs 2).
void plan_estimators(const std::vector<ProbPlan>& ps, Plan& plan, int config = 0,
                     int max_slots = kMaxSlots) {
  const int shape = shape_of(config);
  if (ps.empty()) return;
  const ProbPlan& p0 = ps[0];
  // primal samples in job order; replay units, pairs first: within a launch
  // blocks are dispatched in order and a pair block traces twice the paths of
  // a single one
  std::vector<std::pair<int, int>> prim;
  for (int j = 0; j < p0.np; ++j)
    for (int k = 0; k < p0.pj[j].spp; ++k) prim.push_back({j, k});
  const bool shared_pairs = std::any_of(p0.aj, p0.aj + p0.na, [](const AdjointSpec& a) {
    return a.params_b != nullptr && a.shared;
  });
  // hit records: for replays of single paths and replay pairs of mesh scenes
  // (only the mesh kernel instances use them; those of shared-path pairs and
  // of the deterministic mode have none)
  const bool use_recs = !shared_pairs &&
                        !(p0.flags & (JSO_F_DETERMINISTIC | JSO_F_NO_HIT_RECORDS)) &&
                        p0.s->dev.layout != JSO_LAYOUT_VOLUME;
  const uint32_t rec_epoch = ++g_rec_epoch;
  std::vector<std::pair<int, int>> units;
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < p0.na; ++j)
      if ((p0.aj[j].params_b != nullptr) == (pass == 0))
        for (int k = 0; k < p0.aj[j].spp; ++k) units.push_back({j, k});
  size_t next_prim = 0, next_unit = 0;
  int max_ch = 0;
  for (const ProbPlan& p : ps) max_ch = std::max(max_ch, p.s->n_ch);
  // volumes: the kernels read bricked copies of the parameter vectors, made
  // here first (each problem references at most 2 vectors)
  std::vector<std::vector<std::pair<const float*, const float*>>> bricks(ps.size());
  if (p0.s->dev.layout == JSO_LAYOUT_VOLUME) {
    LaunchRec br;
    br.kind = Kern::Brick;
    br.timer = JSO_K_FORWARD;
    for (size_t q = 0; q < ps.size(); ++q) {
      const ProbPlan& p = ps[q];
      auto add = [&](const float* src) {
        if (!src) return;
        for (const auto& x : bricks[q])
          if (x.first == src) return;
        if (bricks[q].size() == 2) {  // no entry point builds such a plan
          std::fprintf(stderr, "jso: a volume plan references 3 parameter vectors\n");
          std::abort();
        }
        const float* dst = p.s->vbrick + bricks[q].size() * p.s->brick_n;
        bricks[q].push_back({src, dst});
        BrickArgs b{};
        b.src = gmem(reinterpret_cast<const float4*>(src));
        b.dst = gmem(reinterpret_cast<float4*>(const_cast<float*>(dst)));
        b.R = p.s->dev.vol_res;
        b.Rb = p.s->dev.vol_rb;
        const size_t vox = p.s->brick_n / 4;
        b.nblocks = (uint32_t)std::min<size_t>((vox + kBrickBlock - 1) / kBrickBlock, 8192);
        push_unit(br, b, b.nblocks);
      };
      for (int j = 0; j < p.np; ++j) {
        add(p.pj[j].params);
        add(p.pj[j].params_b);
      }
      for (int j = 0; j < p.na; ++j) {
        add(p.aj[j].params);
        add(p.aj[j].params_b);
      }
    }
    plan.push_back(std::move(br));
  }
  // the pointer a kernel of problem q reads for parameter vector src
  auto kparams = [&](size_t q, const float* src) -> const float* {
    for (const auto& x : bricks[q])
      if (x.first == src) return x.second;
    return src;
  };
  while (next_prim < prim.size() || next_unit < units.size()) {
    // slice layout of this launch (shared by all problems).  kind 0 primal,
    // 1 adjoint A, 2 adjoint B (replay pair), 3 adjoint shared pair; a slice
    // with slot_b >= 0 also writes the radiance of its second ledger there.
    // The slots of one primal job's samples are contiguous (a shared pair:
    // all first ledgers, then all second ledgers).
    struct FSl { int kind, job, sample, slot, slot_b; };
    std::vector<FSl> fsl;
    int nslot = 0;
    while (next_prim < prim.size()) {
      const int j = prim[next_prim].first;
      if (p0.pj[j].params_b == nullptr) {
        if (nslot + 1 > max_slots) break;
        fsl.push_back({0, j, prim[next_prim].second, nslot++, -1});
        ++next_prim;
        continue;
      }
      int m = 0;
      while (next_prim + m < prim.size() && prim[next_prim + m].first == j &&
             nslot + 2 * (m + 1) <= max_slots)
        ++m;
      if (m == 0) break;
      for (int t = 0; t < m; ++t)
        fsl.push_back({0, j, prim[next_prim + t].second, nslot + t, nslot + m + t});
      nslot += 2 * m;
      next_prim += m;
    }
    // finalize jobs: (job, second ledger?)
    std::vector<std::pair<int, int>> fin_jobs;
    for (const FSl& x : fsl) {
      if (fin_jobs.empty() || fin_jobs.back().first != x.job) {
        fin_jobs.push_back({x.job, 0});
        if (x.slot_b >= 0) fin_jobs.push_back({x.job, 1});
      }
    }
    std::vector<std::pair<int, int>> reps;  // replay units of this launch
    std::vector<std::pair<int, int>> rep_slot;
    if (next_prim == prim.size()) {
      while (next_unit < units.size()) {
        const auto u = units[next_unit];
        const AdjointSpec& a = p0.aj[u.first];
        const int need = a.params_b ? 2 : 1;
        if (nslot + need > max_slots) break;
        const int sa = nslot++;
        const int sb = need == 2 ? nslot++ : -1;
        if (a.params_b && a.shared) {
          fsl.push_back({3, u.first, u.second, sa, sb});
        } else {
          fsl.push_back({1, u.first, u.second, sa, -1});
          if (need == 2) fsl.push_back({2, u.first, u.second, sb, -1});
        }
        reps.push_back(u);
        rep_slot.push_back({sa, sb});
        ++next_unit;
      }
    }
    if (fsl.empty()) break;  // nothing fits max_slots (callers keep it >= 1, 2 with pairs)
    // k_forward
    LaunchRec fw;
    fw.kind = Kern::Forward;
    fw.timer = JSO_K_FORWARD;
    fw.shape = shape;
    fw.vol = p0.s->dev.layout == JSO_LAYOUT_VOLUME;
    fw.persist = fw.vol ? 0 : persist_of(config);
    fw.waves = std::min((int)fsl.size(), kVolMaxSliceWaves);
    for (size_t q = 0; q < ps.size(); ++q) {
      const ProbPlan& p = ps[q];
      if (crop_empty(p.crop)) continue;
      FwdArgs f{};
      f.h.max_iter = p.max_iter;
      f.scene = cmem((const DevScene*)p.s->d_scene);
      uint32_t* recs = use_recs ? recs_of(p) : nullptr;
      f.recs = gmem(recs);
      f.rec_epoch = rec_epoch;
      for (size_t i = 0; i < fsl.size(); ++i) {
        const FSl& x = fsl[i];
        FwdSlice& fs = f.sl[i];
        if (recs && x.kind != 0) f.rec_mask |= 1u << i;  // paths this plan replays
        fs.sample = (uint32_t)x.sample;
        fs.slot = x.slot;
        fs.slot_b = x.slot_b;
        if (x.kind == 0) {
          fs.params = gmem(kparams(q, p.pj[x.job].params));
          fs.params_b = x.slot_b >= 0 ? gmem(kparams(q, p.pj[x.job].params_b))
                                      : gmem((const float*)nullptr);
          fs.tag = p.pj[x.job].tag;
        } else {
          const AdjointSpec& a = p.aj[x.job];
          fs.params = gmem(kparams(q, x.kind == 2 ? a.params_b : a.params));
          fs.params_b = x.kind == 3 ? gmem(kparams(q, a.params_b)) : gmem((const float*)nullptr);
          fs.tag = a.tag;
        }
        if (x.slot_b >= 0) fw.shared = true;
      }
      f.n_slices = (int)fsl.size();
      f.key = p.key;
      f.crop = p.crop;
      f.mask = gmem(p.mask);
      f.slots = gmem(slots_of(p));
      f.npix = (uint32_t)p.s->npix;
      f.flags = p.flags;
      fw.stack = std::max(fw.stack, p.s->stack);
      if (fw.vol) {  // 8x8 tiles, fw.waves slices per block
        constexpr int kVolShape = 2;
        static_assert(kShapeW[kVolShape] == 8 && kShapeH[kVolShape] == 8, "volume tiles");
        f.tiles_x = tiles_x(p.crop, kVolShape);
        f.tiles = tiles_of(p.crop, kVolShape);
        const uint32_t groups = (uint32_t)((f.n_slices + fw.waves - 1) / fw.waves);
        push_unit(fw, f, f.tiles * groups);
      } else {
        f.tiles_x = tiles_x(p.crop, shape);
        f.tiles = tiles_of(p.crop, shape);
        push_unit(fw, f, f.tiles * (uint32_t)f.n_slices);
      }
    }
    plan.push_back(std::move(fw));
    // k_finalize of the primal jobs with samples in this launch
    if (!fin_jobs.empty()) {
      LaunchRec fr;
      fr.kind = Kern::Finalize;
      fr.timer = JSO_K_FINALIZE;
      for (const ProbPlan& p : ps) {
        if (crop_empty(p.crop)) continue;
        FinArgs f{};
        f.h.max_iter = p.max_iter;
        for (size_t q = 0; q < fin_jobs.size(); ++q) {
          const int j = fin_jobs[q].first;
          const bool second = fin_jobs[q].second != 0;
          int n = 0, s0 = -1, first_sample = -1, last_sample = -1;
          for (const FSl& x : fsl)
            if (x.kind == 0 && x.job == j) {
              if (first_sample < 0) {
                first_sample = x.sample;
                s0 = second ? x.slot_b : x.slot;
              }
              last_sample = x.sample;
              ++n;
            }
          FinJob fj{};
          fj.slot0 = s0;
          fj.n = n;
          // a second ledger sums into the accumulator after the plan's jobs
          // (the plan has at most 2 jobs when one is a shared pair)
          const int acc = second ? p.np : j;
          fj.accum = gmem(p.s->accum + (size_t)acc * 3 * p.s->npix);
          fj.first = first_sample == 0;
          fj.last = last_sample == p.pj[j].spp - 1;
          fj.inv_spp = 1.0 / (double)p.pj[j].spp;
          fj.img = second ? gmem((float*)nullptr) : gmem(p.pj[j].img);
          fj.delta = gmem(second ? p.pj[j].delta_b : p.pj[j].delta);
          fj.loss2 = second ? gmem((double*)nullptr) : gmem(p.pj[j].loss2);
          f.jobs[f.n_jobs++] = fj;
        }
        f.slots = gmem(slots_of(p));
        f.npix = (uint32_t)p.s->npix;
        f.width = p.s->width;
        f.key = p.key;
        f.crop = p.crop;
        f.mask = gmem(p.mask);
        f.target = gmem((const float*)p.s->target);
        f.delta_scale = (float)(2.0 / (3.0 * (double)p.s->npix));
        f.loss_scale = 1.0 / (3.0 * (double)p.s->npix);
        f.relative = p.relative;
        const size_t pix = (size_t)(p.crop.x1 - p.crop.x0) * (size_t)(p.crop.y1 - p.crop.y0);
        const size_t want = (pix + kFinBlock - 1) / kFinBlock;
        f.nblocks = (uint32_t)std::min<size_t>(std::max<size_t>(want, 1), kFinMaxBlocks);
        push_unit(fr, f, f.nblocks * (uint32_t)f.n_jobs);
      }
      plan.push_back(std::move(fr));
    }
    // k_adjoint: pair units of every problem first, then single-path units.
    // Replay pairs (not shared) run on lane pairs: their units take tiles of
    // half the shape's height, so a pair tile has as many lanes as a single
    // one.
    if (!reps.empty()) {
      const bool vol = p0.s->dev.layout == JSO_LAYOUT_VOLUME;
      LaunchRec ad;
      ad.kind = Kern::Adjoint;
      ad.timer = JSO_K_ADJOINT;
      ad.shape = shape;
      ad.lds = adjoint_lds_bytes(max_ch);
      ad.shared = shared_pairs;
      ad.vol = vol;
      ad.persist = vol ? 0 : persist_of(config);
      ad.det = (p0.flags & JSO_F_DETERMINISTIC) != 0;
      for (int pass = 0; pass < 2; ++pass) {
        for (size_t q = 0; q < ps.size(); ++q) {
          const ProbPlan& p = ps[q];
          if (crop_empty(p.crop)) continue;
          RepArgs r{};
          r.h.max_iter = p.max_iter;
          r.scene = cmem((const DevScene*)p.s->d_scene);
          for (size_t i = 0; i < reps.size(); ++i) {
            const AdjointSpec& a = p.aj[reps[i].first];
            if ((a.params_b != nullptr) != (pass == 0)) continue;
            RepSlice rs{};
            rs.params = gmem(kparams(q, a.params));
            rs.params_b = gmem(a.params_b ? kparams(q, a.params_b) : nullptr);
            rs.delta = gmem(a.delta);
            rs.delta_b = gmem(a.delta_b);
            rs.grad = gmem(a.grad);
            rs.sign = a.sign;
            rs.adj_scale = (float)(1.0 / (double)a.spp);
            rs.tag = a.tag;
            rs.sample = (uint32_t)reps[i].second;
            rs.slot_a = rep_slot[i].first;
            rs.slot_b = rep_slot[i].second;
            if (p.flags & JSO_F_DETERMINISTIC) {  // accumulator k of job k
              rs.fx = gmem(p.s->fx + (size_t)reps[i].first * p.s->P);
              rs.fx_scale = p.fx_scale;
            }
            r.sl[r.n_slices++] = rs;
          }
          if (r.n_slices == 0) continue;
          r.key = p.key;
          r.crop = p.crop;
          r.mask = gmem(p.mask);
          r.slots = gmem((const double*)slots_of(p));
          r.npix = (uint32_t)p.s->npix;
          r.flags = p.flags;
          r.pair_lanes = pass == 0 && !shared_pairs && !vol;
          r.recs = gmem(use_recs ? recs_of(p) : nullptr);
          r.rec_epoch = rec_epoch;
          r.tiles_x = tiles_x(p.crop, shape);
          r.tiles = r.pair_lanes ? pair_tiles_of(p.crop, shape) : tiles_of(p.crop, shape);
          ad.stack = std::max(ad.stack, p.s->stack);
          push_unit(ad, r, r.tiles * (uint32_t)r.n_slices);
        }
      }
      plan.push_back(std::move(ad));
    }
  }
  // deterministic mode: fold each job's fixed-point sums into its gradient
  if (p0.flags & JSO_F_DETERMINISTIC) {
    LaunchRec fl;
    fl.kind = Kern::FxFlush;
    fl.timer = JSO_K_ADJOINT;
    for (const ProbPlan& p : ps) {
      for (int j = 0; j < p.na; ++j) {
        FxArgs f{};
        f.h.max_iter = p.max_iter;
        f.fx = gmem(p.s->fx + (size_t)j * p.s->P);
        f.grad = gmem(p.aj[j].grad);
        f.n = p.s->P;
        f.inv_scale = 1.0 / p.fx_scale;
        f.nblocks = (uint32_t)std::min<size_t>((p.s->P + kFxBlock - 1) / kFxBlock, 1024);
        push_unit(fl, f, f.nblocks);
      }
    }
    plan.push_back(std::move(fl));
  }
}

// The four cosine-transform passes that replace vec by (I + lambda L)^-1 vec
// (along W, along H with the spectral scaling, back along H, back along W),
// as units appended to rec[0..3]; tmp holds P floats.
void push_precond(LaunchRec rec[4], SceneGPU* s, float* vec, float* tmp, float lambda,
                  uint32_t max_iter) {
  const DevScene& S = s->dev;
  const int W = S.tex_w, H = S.tex_h, C = S.n_ch;
  const float* cw = s->pc;
  const float* ch = cw + (size_t)W * W;
  const float* mu = ch + (size_t)H * H;
  const float* nu = mu + W;
  auto tiles = [](int n) { return (uint32_t)((n + kDctTile - 1) / kDctTile); };
  for (int pass = 0; pass < 4; ++pass) {
    DctArgs a{};
    a.h.max_iter = max_iter;
    const bool along_w = pass == 0 || pass == 3;
    a.A = gmem(along_w ? cw : ch);
    a.transA = pass >= 2;
    a.in = gmem((const float*)(pass % 2 == 0 ? vec : tmp));
    a.out = gmem(pass % 2 == 0 ? tmp : vec);
    if (along_w) {  // element (w, (h, c)) at w C + h W C + c
      a.n = W;
      a.N = H * C;
      a.sk = C;
      a.jin = C;
      a.sjo = W * C;
    } else {        // element (h, (w, c)) at h W C + (w C + c)
      a.n = H;
      a.N = W * C;
      a.sk = W * C;
      a.jin = W * C;
      a.sjo = 0;
    }
    if (pass == 1) {
      a.eig_m = gmem(nu);
      a.eig_j = gmem(mu);
      a.jdiv = C;
      a.lambda = lambda;
    } else {
      a.jdiv = 1;
    }
    a.tiles_j = tiles(a.N);
    push_unit(rec[pass], a, tiles(a.n) * a.tiles_j);
  }
}

bool preconditioned(const SceneGPU* s) {
  return s->dev.layout == JSO_LAYOUT_TEXTURE && s->dev.tex_w * s->dev.tex_h > 1;
}

// Preconditioner launches of a step: both gradient samples of the
// meta-estimator (or Adam's gradient) of every textured problem.
void plan_precond(const std::vector<ProbPlan>& ps, const jso_step_opts& o, Plan& plan) {
  if (!(o.precond_lambda > 0.0f)) return;
  LaunchRec rec[4];
  for (LaunchRec& r : rec) {
    r.kind = Kern::Dct;
    r.timer = JSO_K_PRECOND;
  }
  for (const ProbPlan& p : ps) {
    if (!preconditioned(p.s)) continue;
    push_precond(rec, p.s, p.s->F, p.s->pc_tmp, o.precond_lambda, p.max_iter);
    if (o.optimizer == JSO_OPT_META && o.spp_fd > 0)
      push_precond(rec, p.s, p.s->dF, p.s->pc_tmp + p.s->P, o.precond_lambda, p.max_iter);
  }
  if (rec[0].n == 0) return;
  for (LaunchRec& r : rec) plan.push_back(std::move(r));
}

uint32_t meta_blocks(size_t P) {
  const size_t want = (P + (size_t)kMetaBlock * kMetaK - 1) / ((size_t)kMetaBlock * kMetaK);
  return (uint32_t)std::min<size_t>(std::max<size_t>(want, 1), kMetaMaxBlocks);
}

MetaArgs meta_args(SceneGPU* s, const float* F, const float* dF, float eta, float bF, float bD,
                   int zero_grads) {
  MetaArgs m{};
  m.nblocks = meta_blocks(s->P);
  m.params = gmem(s->params);
  m.params_prev = gmem(s->params_prev);
  m.F = gmem(const_cast<float*>(F));
  m.dF = gmem(const_cast<float*>(dF));
  m.mean = gmem(s->mean);
  m.var = gmem(s->var);
  m.alpha_prev = gmem(s->alpha_prev);
  m.m2F = gmem(s->m2F);
  m.m2D = gmem(s->m2D);
  m.ctl = gmem(s->ctl);
  m.partials = gmem(s->partials);
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
  m.ablate = 0;
  m.m1F = gmem(s->m1F);
  m.m1D = gmem(s->m1D);
  m.Fv = gmem(s->Fv);
  m.dFv = gmem(s->dFv);
  return m;
}

AdamArgs adam_args(SceneGPU* s, const float* g, float eta, float b1, float b2, float eps,
                   int zero_grads) {
  AdamArgs a{};
  const size_t want = (s->P + kMetaBlock - 1) / kMetaBlock;
  a.nblocks = (uint32_t)std::min<size_t>(std::max<size_t>(want, 1), 2048);
  a.params = gmem(s->params);
  a.params_prev = gmem(s->params_prev);
  a.g = gmem(const_cast<float*>(g));
  a.m = gmem(s->adam_m);
  a.v = gmem(s->adam_v);
  a.ctl = gmem(s->ctl);
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

// The optimiser launch of a step over problems ps.
void plan_optimizer(const std::vector<ProbPlan>& ps, const jso_step_opts& o, Plan& plan) {
  LaunchRec r;
  if (o.optimizer == JSO_OPT_META) {
    r.kind = Kern::Meta;
    r.timer = JSO_K_META;
    for (const ProbPlan& p : ps) {
      MetaArgs m = meta_args(p.s, p.s->F, p.s->dF, o.eta, o.beta_F, o.beta_D, 1);
      m.h.max_iter = p.max_iter;
      m.ablate = o.ablate;
      push_unit(r, m, m.nblocks);
    }
  } else {
    r.kind = Kern::Adam;
    r.timer = JSO_K_ADAM;
    for (const ProbPlan& p : ps) {
      AdamArgs a = adam_args(p.s, p.s->F, o.eta, o.adam_beta1, o.adam_beta2, o.adam_eps, 1);
      a.h.max_iter = p.max_iter;
      push_unit(r, a, a.nblocks);
    }
  }
  plan.push_back(std::move(r));
}

// The finite-difference jobs of <dF_i> (Eq. 5): primal images at pi_i and
// pi_{i-1} (adjoint images delta1, delta0) and the differenced adjoint paths,
// as a replay pair (two paths per sample) or, with JSO_FD_SHARED, one path per
// sample drawn at pi_i and evaluated at both.
void add_fd_jobs(ProbPlan& p, SceneGPU* s, int fd_mode, uint32_t tag_primal, uint32_t tag_adj,
                 int spp, float* delta1, float* delta0, float* dF) {
  if (fd_mode == JSO_FD_SHARED) {
    PrimalSpec ps{s->params, tag_primal, spp, nullptr, delta1, nullptr};
    ps.params_b = s->params_prev;
    ps.delta_b = delta0;
    p.pj[p.np++] = ps;
    AdjointSpec as{s->params, s->params_prev, delta1, delta0, dF, 1.0f, tag_adj, spp};
    as.shared = true;
    p.aj[p.na++] = as;
    return;
  }
  p.pj[p.np++] = PrimalSpec{s->params, tag_primal, spp, nullptr, delta1, nullptr};
  p.pj[p.np++] = PrimalSpec{s->params_prev, tag_primal, spp, nullptr, delta0, nullptr};
  p.aj[p.na++] = AdjointSpec{s->params, s->params_prev, delta1, delta0, dF, 1.0f, tag_adj, spp};
}

// One problem of a grad_step: the estimator jobs of its optimiser.
ProbPlan step_problem(SceneGPU* s, const jso_step_opts& o, uint32_t flags, uint32_t max_iter) {
  ProbPlan p{};
  p.s = s;
  p.fx_scale = fx_scale_of(s, true);
  p.relative = o.loss == JSO_LOSS_RELATIVE;
  p.key = KeyArgs{o.seed, 0u, gmem((const uint32_t*)&s->ctl->iteration)};  // the kernels read the device counter
  p.crop = Crop{0, 0, s->width, s->height};
  p.mask = nullptr;
  p.flags = flags;
  p.max_iter = max_iter;
  const size_t n3 = 3 * s->npix;
  float* d_prop = s->delta;
  if (o.optimizer == JSO_OPT_META) {
    const bool fd = o.spp_fd > 0;
    p.pj[p.np++] = PrimalSpec{s->params, JSO_TAG_PRIMAL_PROP, o.spp_prop, nullptr, d_prop,
                              s->ctl->loss};
    p.aj[p.na++] = AdjointSpec{s->params, nullptr, d_prop, nullptr, s->F, 1.0f,
                               JSO_TAG_ADJ_PROP, o.spp_prop};
    if (fd)
      add_fd_jobs(p, s, o.fd_mode, JSO_TAG_PRIMAL_FD, JSO_TAG_ADJ_FD, o.spp_fd, s->delta + n3,
                  s->delta + 2 * n3, s->dF);
  } else {
    p.pj[p.np++] = PrimalSpec{s->params, JSO_TAG_ADAM_PRIMAL, o.adam_spp, nullptr, d_prop,
                              s->ctl->loss};
    p.aj[p.na++] = AdjointSpec{s->params, nullptr, d_prop, nullptr, s->F, 1.0f,
                               JSO_TAG_ADAM_ADJ, o.adam_spp};
  }
  return p;
}

// The separate variance samples of the uncorrelated ablation: the same
// estimators as step_problem's meta-estimator jobs on their own streams
// (VAR_* tags), into Fv / dFv; they reuse the adjoint-image buffers after the
// main estimators' replay and add nothing to the loss.
ProbPlan variance_problem(SceneGPU* s, const jso_step_opts& o, uint32_t flags,
                          uint32_t max_iter) {
  ProbPlan p = step_problem(s, o, flags, max_iter);
  const size_t n3 = 3 * s->npix;
  p.np = p.na = 0;
  p.pj[p.np++] = PrimalSpec{s->params, JSO_TAG_VAR_PRIMAL_PROP, o.spp_prop, nullptr, s->delta,
                            nullptr};
  p.aj[p.na++] = AdjointSpec{s->params, nullptr, s->delta, nullptr, s->Fv, 1.0f,
                             JSO_TAG_VAR_ADJ_PROP, o.spp_prop};
  if (o.spp_fd > 0)
    add_fd_jobs(p, s, o.fd_mode, JSO_TAG_VAR_PRIMAL_FD, JSO_TAG_VAR_ADJ_FD, o.spp_fd,
                s->delta + n3, s->delta + 2 * n3, s->dFv);
  return p;
}

bool is_volume(const SceneGPU* s) { return s->dev.layout == JSO_LAYOUT_VOLUME; }

// Problems stepped together must all be volumes or none (their launches use
// different kernels).
int check_same_kind(jso_ctx* c, const int* ids, int n) {
  for (int k = 1; k < n; ++k)
    if (is_volume(get_scene(c, ids[k])) != is_volume(get_scene(c, ids[0])))
      return fail(c, JSO_E_INVALID, "volume and surface scenes cannot be stepped together");
  return JSO_OK;
}

// The volume kernels read each voxel's 4 channels with one 16-byte load.
int check_volume_params(jso_ctx* c, const SceneGPU* s, const float* params) {
  if (is_volume(s) && (reinterpret_cast<uintptr_t>(params) & 15u) != 0)
    return fail(c, JSO_E_INVALID, "volume parameters must be 16-byte aligned");
  return JSO_OK;
}

bool uncorrelated(const jso_step_opts& o) {
  return o.optimizer == JSO_OPT_META && (o.ablate & JSO_ABLATE_UNCORRELATED) != 0;
}

int check_step_opts(jso_ctx* c, const jso_step_opts* o) {
  if (o->loss != JSO_LOSS_L2 && o->loss != JSO_LOSS_RELATIVE)
    return fail(c, JSO_E_INVALID, "unknown loss %d", o->loss);
  if (o->ablate & ~7u) return fail(c, JSO_E_INVALID, "unknown ablation bits 0x%x", o->ablate);
  if (o->fd_mode != JSO_FD_REPLAY && o->fd_mode != JSO_FD_SHARED)
    return fail(c, JSO_E_INVALID, "unknown fd_mode %d", o->fd_mode);
  if (!(o->precond_lambda >= 0.0f && std::isfinite(o->precond_lambda)))
    return fail(c, JSO_E_INVALID, "precond_lambda must be finite and >= 0");
  if (o->optimizer == JSO_OPT_META) {
    if (o->spp_prop < 1 || o->spp_prop > 64 || o->spp_fd < 0 || o->spp_fd > 64)
      return fail(c, JSO_E_INVALID, "spp out of range");
    if (!(o->beta_F >= 0.0f && o->beta_F < 1.0f && o->beta_D >= 0.0f && o->beta_D < 1.0f))
      return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
  } else if (o->optimizer == JSO_OPT_ADAM) {
    if (o->adam_spp < 1 || o->adam_spp > 4096) return fail(c, JSO_E_INVALID, "adam_spp");
    if (!(o->adam_beta1 >= 0.0f && o->adam_beta1 < 1.0f && o->adam_beta2 >= 0.0f &&
          o->adam_beta2 < 1.0f))
      return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
  } else {
    return fail(c, JSO_E_INVALID, "unknown optimizer %d", o->optimizer);
  }
  return JSO_OK;
}

int check_precond_layout(jso_ctx* c, const std::vector<SceneGPU*>& ss, const jso_step_opts& o) {
  if (!(o.precond_lambda > 0.0f)) return JSO_OK;
  for (SceneGPU* s : ss)
    if (s->dev.layout != JSO_LAYOUT_TEXTURE)
      return fail(c, JSO_E_INVALID, "preconditioning needs texture parameters");
  return JSO_OK;
}

// Deterministic mode (JSO_F_DETERMINISTIC in flags): the scene's fixed-point
// accumulators (allocated zeroed on first use; the flush leaves them zeroed).
int ensure_fx(jso_ctx* c, SceneGPU* s, uint32_t flags) {
  if (!(flags & JSO_F_DETERMINISTIC)) return JSO_OK;
  if (s->dev.layout == JSO_LAYOUT_VOLUME)
    return fail(c, JSO_E_UNSUPPORTED, "deterministic mode: not for volume scenes");
  if (s->fx) return JSO_OK;
  HIP_TRY(c, hipMalloc(reinterpret_cast<void**>(&s->fx), 2 * s->P * sizeof(unsigned long long)));
  HIP_TRY(c, hipMemset(s->fx, 0, 2 * s->P * sizeof(unsigned long long)));
  return JSO_OK;
}

// queue: the launch's two work-queue counters when its configuration is
// persistent (null: one block per tile whatever the configuration)
hipError_t launch_rec(const LaunchRec& r, const void* dev_units, unsigned long long* work,
                      hipStream_t st, uint32_t* queue = nullptr, int n_cu = 0) {
  const bool persistent = queue && r.persist > 0 && n_cu > 0;
  uint32_t* q = persistent ? queue : nullptr;
  const uint32_t grid = persistent ? (uint32_t)(r.persist * n_cu) : 0u;
  switch (r.kind) {
    case Kern::Forward:
      if (r.vol)
        return launch_vol_forward(static_cast<const FwdArgs*>(dev_units), r.n, r.blocks, r.waves,
                                  work, st);
      return launch_forward(static_cast<const FwdArgs*>(dev_units), r.n, r.blocks, r.shape,
                            r.stack, r.shared, work, st, q, grid);
    case Kern::Finalize:
      return launch_finalize(static_cast<const FinArgs*>(dev_units), r.n, r.blocks, st);
    case Kern::Adjoint:
      if (r.vol)
        return launch_vol_adjoint(static_cast<const RepArgs*>(dev_units), r.n, r.blocks, r.shape,
                                  work, st);
      return launch_adjoint(static_cast<const RepArgs*>(dev_units), r.n, r.blocks, r.shape, r.lds,
                            r.stack, r.shared, work, st, q, grid, r.det);
    case Kern::Meta:
      return launch_meta(static_cast<const MetaArgs*>(dev_units), r.n, r.blocks, st);
    case Kern::Adam:
      return launch_adam(static_cast<const AdamArgs*>(dev_units), r.n, r.blocks, st);
    case Kern::Dct:
      return launch_dct(static_cast<const DctArgs*>(dev_units), r.n, r.blocks, st);
    case Kern::FxFlush:
      return launch_fx_flush(static_cast<const FxArgs*>(dev_units), r.n, r.blocks, st);
    case Kern::Brick:
      return launch_vol_brick(static_cast<const BrickArgs*>(dev_units), r.n, r.blocks, st);
  }
  return hipErrorInvalidValue;
}

// Identity of a step configuration for the tuner: estimator/optimiser sample
// counts and, per problem, image and parameter layout (FNV-1a).
uint64_t config_hash(const std::vector<SceneGPU*>& ss, const jso_step_opts& o) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (v >> (8 * k)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)o.optimizer);
  mix((uint64_t)o.spp_prop);
  mix((uint64_t)o.spp_fd);
  mix((uint64_t)o.adam_spp);
  for (SceneGPU* s : ss) {
    mix((uint64_t)s->width);
    mix((uint64_t)s->height);
    mix((uint64_t)s->n_ch);
    mix((uint64_t)s->P);
    mix((uint64_t)s->dev.depth);
    mix((uint64_t)s->dev.n_tris);
    mix((uint64_t)(o.precond_lambda > 0.0f && preconditioned(s)));
    mix((uint64_t)uncorrelated(o));
    mix((uint64_t)(o.optimizer == JSO_OPT_META && o.spp_fd > 0 ? o.fd_mode : 0));
  }
  return h;
}

int chosen_config(jso_ctx* c, uint64_t hash) {
  std::lock_guard<std::mutex> lock(g_tuned_mu);
  auto it = g_tuned.find({c->arch, hash});
  return it != g_tuned.end() ? it->second : c->launch_config;
}

// Run a plan now: each launch's units are staged through the context's ring.
int exec_plan(jso_ctx* c, const Plan& plan) {
  unsigned long long* work = c->counting ? c->d_work : nullptr;
  for (const LaunchRec& r : plan) {
    if (r.n == 0) continue;
    const void* dev = nullptr;
    HIP_TRY(c, c->ring.put(r.units.data(), r.units.size(), c->stream, &dev));
    TIMED_LAUNCH(c, r.timer, launch_rec(r, dev, work, c->stream));
  }
  return JSO_OK;
}

// Concatenate a plan's unit arrays (256-byte aligned) and note each offset.
std::vector<uint8_t> pack_plan(const Plan& plan, std::vector<size_t>& off) {
  std::vector<uint8_t> all;
  off.clear();
  for (const LaunchRec& r : plan) {
    off.push_back(all.size());
    all.insert(all.end(), r.units.begin(), r.units.end());
    all.resize((all.size() + 255) & ~(size_t)255);
  }
  return all;
}

// grad_step: launch the cached plan when `sig` matches, else build it with
// `build`, upload it once and cache it.
template <class Build>
int exec_cached(jso_ctx* c, const std::vector<uint64_t>& sig, Build build) {
  PlanCache& pc = c->plan_cache;
  CachedPlan* hit = nullptr;
  for (CachedPlan& p : pc.plans)
    if (p.sig == sig) hit = &p;
  if (!hit) {
    Plan plan;
    build(plan);
    std::vector<size_t> off;
    const std::vector<uint8_t> all = pack_plan(plan, off);
    if (pc.plans.size() >= PlanCache::kMaxPlans) {
      // evict the least recently used plan once no launch can still read it
      size_t lru = 0;
      for (size_t k = 1; k < pc.plans.size(); ++k)
        if (pc.plans[k].last_use < pc.plans[lru].last_use) lru = k;
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      PlanCache::release(pc.plans[lru]);
      pc.plans.erase(pc.plans.begin() + (long)lru);
    }
    CachedPlan np;
    const size_t nq = 2 * plan.size();
    if (hipHostMalloc(reinterpret_cast<void**>(&np.host), all.size(), 0) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&np.dev), all.size()) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&np.queues), nq * sizeof(uint32_t)) != hipSuccess) {
      PlanCache::release(np);
      return fail(c, JSO_E_OOM, "launch descriptors");
    }
    // zeroed by a kernel (not a memset node, should a caller capture the step)
    HIP_TRY(c, launch_fill_f32(reinterpret_cast<float*>(np.queues), nq, 0.0f, c->stream));
    std::memcpy(np.host, all.data(), all.size());
    const hipError_t e =
        hipMemcpyAsync(np.dev, np.host, all.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      PlanCache::release(np);
      HIP_TRY(c, e);
    }
    for (size_t k = 0; k < plan.size(); ++k) {
      const LaunchRec& r = plan[k];
      np.launches.push_back(
          CachedLaunch{(int)r.kind, r.timer, r.shape, r.n, r.stack, r.shared, r.vol, r.blocks,
                       r.lds, off[k], r.persist, r.det, r.waves});
    }
    np.sig = sig;
    pc.plans.push_back(std::move(np));
    hit = &pc.plans.back();
  }
  hit->last_use = ++pc.clock;
  unsigned long long* work = c->counting ? c->d_work : nullptr;
  for (size_t k = 0; k < hit->launches.size(); ++k) {
    const CachedLaunch& l = hit->launches[k];
    if (l.n == 0) continue;
    LaunchRec r;
    r.kind = (Kern)l.kind;
    r.shape = l.shape;
    r.n = l.n;
    r.blocks = l.blocks;
    r.lds = l.lds;
    r.stack = l.stack;
    r.shared = l.shared;
    r.vol = l.vol;
    r.persist = l.persist;
    r.det = l.det;
    r.waves = l.waves;
    TIMED_LAUNCH(c, l.timer, launch_rec(r, hit->dev + l.offset, work, c->stream,
                                        hit->queues + 2 * k, c->n_cu));
  }
  return JSO_OK;
}

// The estimator jobs of jso_estimate_gradients (same streams as a meta step).
ProbPlan estimate_problem(SceneGPU* s, uint64_t seed, uint32_t iteration, int spp_prop,
                          int spp_fd, float* F, float* dF, float* img, double* loss2,
                          const Crop& crop, const uint8_t* mask, uint32_t flags, int loss,
                          int fd_mode) {
  ProbPlan p{};
  p.s = s;
  p.fx_scale = fx_scale_of(s, true);
  p.fx_scale = fx_scale_of(s, true);
  p.relative = loss == JSO_LOSS_RELATIVE;
  p.key = KeyArgs{seed, iteration, nullptr};
  p.crop = crop;
  p.mask = mask;
  p.flags = flags;
  const size_t n3 = 3 * s->npix;
  const bool fd = dF != nullptr && spp_fd > 0;
  p.pj[p.np++] = PrimalSpec{s->params, JSO_TAG_PRIMAL_PROP, spp_prop, img, s->delta, loss2};
  p.aj[p.na++] = AdjointSpec{s->params, nullptr, s->delta, nullptr, F, 1.0f, JSO_TAG_ADJ_PROP,
                             spp_prop};
  if (fd)
    add_fd_jobs(p, s, fd_mode, JSO_TAG_PRIMAL_FD, JSO_TAG_ADJ_FD, spp_fd, s->delta + n3,
                s->delta + 2 * n3, dF);
  return p;
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
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->arch = prop.gcnArchName;
    c->n_cu = prop.multiProcessorCount;
  }
  {
    // set-up of what the no-allocation entry point uses: the device address
    // of this GPU's scratch array and the descriptor ring
    DeviceGuard g(device);
    if (scratch_address(device, &c->scratch) != hipSuccess || c->ring.init() != hipSuccess) {
      c->ring.destroy();
      delete c;
      return JSO_E_HIP;
    }
  }
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
  c->ring.destroy();
  c->plan_cache.destroy();
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
  if (flags & ~63u) return fail(c, JSO_E_INVALID, "unknown debug flags 0x%x", flags);
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
  s->generation = ++g_scene_generation;
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
  A(dalloc(&s->m1F, P));
  A(dalloc(&s->m1D, P));
  A(dalloc(&s->Fv, P));
  A(dalloc(&s->dFv, P));
  A(dalloc(&s->ctl, 1));
  A(dalloc(&s->scratch_loss, 2));
  A(dalloc(&s->partials, kMetaMaxBlocks));
  A(dalloc(&s->slots, (size_t)kMaxSlots * n3));
  A(dalloc(&s->accum, 3 * n3));
  A(dalloc(&s->d_scene, 1));
  if (s->brick_n) A(dalloc(&s->vbrick, 2 * s->brick_n));
  else if (s->dev.n_tris > 0)
    A(dalloc(&s->recs, (size_t)kMaxSlots * kHitRecs * kRecWords * s->npix));
  if (e != hipSuccess) {
    free_scene_buffers(s.get());
    return fail(c, e == hipErrorOutOfMemory ? JSO_E_OOM : JSO_E_HIP, "scene allocation: %s",
                hipGetErrorString(e));
  }
  rc = upload_mesh(c, d, s.get());
  if (rc == JSO_OK) rc = upload_precond(c, s.get());
  if (rc) {
    free_scene_buffers(s.get());
    return rc;
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
  if (int rc = check_volume_params(c, s, params)) return rc;
  DeviceGuard g(c->device);
  ProbPlan p{};
  p.s = s;
  p.key = KeyArgs{seed, iteration, nullptr};
  p.crop = crop_of(s, opts);
  p.mask = opts ? opts->pixel_mask : nullptr;
  p.flags = c->debug_flags | (opts ? opts->flags : 0u);
  p.pj[p.np++] = PrimalSpec{params, tag, spp, img, nullptr, nullptr};
  Plan plan;
  plan_estimators({p}, plan, c->launch_config);
  return exec_plan(c, plan);
}

int jso_render_bwd(jso_ctx* c, int id, const float* params, uint64_t seed, uint32_t iteration,
                   uint32_t tag, int spp, const float* dimg, const jso_render_opts* opts,
                   float* dparams) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!params || !dimg || !dparams) return fail(c, JSO_E_INVALID, "null argument");
  if (spp < 1) return fail(c, JSO_E_INVALID, "spp must be >= 1");
  if (int rc = check_volume_params(c, s, params)) return rc;
  DeviceGuard g(c->device);
  ProbPlan p{};
  p.s = s;
  p.key = KeyArgs{seed, iteration, nullptr};
  p.crop = crop_of(s, opts);
  p.mask = opts ? opts->pixel_mask : nullptr;
  p.flags = c->debug_flags | (opts ? opts->flags : 0u);
  p.aj[p.na++] = AdjointSpec{params, nullptr, dimg, nullptr, dparams, 1.0f, tag, spp};
  p.fx_scale = fx_scale_of(s, false);
  if (int rc = ensure_fx(c, s, p.flags)) return rc;
  Plan plan;
  plan_estimators({p}, plan, c->launch_config);
  return exec_plan(c, plan);
}

int jso_render_bwd_noalloc(jso_ctx* c, int id, const float* params, uint64_t seed,
                           uint32_t iteration, uint32_t tag, int spp, const float* dimg,
                           const jso_render_opts* opts, float* dparams) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!params || !dimg || !dparams) return fail(c, JSO_E_INVALID, "null argument");
  if (spp < 1) return fail(c, JSO_E_INVALID, "spp must be >= 1");
  if (int rc = check_volume_params(c, s, params)) return rc;
  if (!c->scratch) return fail(c, JSO_E_STATE, "no scratch address for device %d", c->device);
  // one radiance slot = 3 doubles per pixel of the whole image
  const size_t slot_bytes = s->npix * 3 * sizeof(double);
  if (slot_bytes > kNoAllocScratchBytes)
    return fail(c, JSO_E_INVALID,
                "render_bwd_noalloc: a %dx%d image needs %zu bytes of scratch per sample; "
                "the no-allocation scratch holds %zu (at most %zu pixels)",
                s->width, s->height, slot_bytes, kNoAllocScratchBytes,
                kNoAllocScratchBytes / (3 * sizeof(double)));
  const int max_slots = (int)std::min<size_t>(kMaxSlots, kNoAllocScratchBytes / slot_bytes);
  DeviceGuard g(c->device);
  ProbPlan p{};
  p.s = s;
  p.key = KeyArgs{seed, iteration, nullptr};
  p.crop = crop_of(s, opts);
  p.mask = opts ? opts->pixel_mask : nullptr;
  p.flags = c->debug_flags | (opts ? opts->flags : 0u);
  p.aj[p.na++] = AdjointSpec{params, nullptr, dimg, nullptr, dparams, 1.0f, tag, spp};
  if (p.flags & JSO_F_DETERMINISTIC)
    return fail(c, JSO_E_UNSUPPORTED, "render_bwd_noalloc: no deterministic mode (its "
                                      "fixed-point sums need memory of the scene's)");
  p.slots = reinterpret_cast<double*>(c->scratch);
  Plan plan;
  plan_estimators({p}, plan, c->launch_config, max_slots);
  // every slot a replay reads is written by the forward launch before it (same
  // pixels, same crop and mask), so the scratch needs no clearing
  return exec_plan(c, plan);
}

int jso_estimate_gradients(jso_ctx* c, int id, uint64_t seed, uint32_t iteration, int spp_prop,
                           int spp_fd, const jso_render_opts* opts, float* F, float* dF,
                           float* img, double* loss) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!F) return fail(c, JSO_E_INVALID, "null F");
  if (spp_prop < 1 || spp_prop > 64 || spp_fd < 0 || spp_fd > 64)
    return fail(c, JSO_E_INVALID, "spp out of range");
  const int lossk = opts ? opts->loss : JSO_LOSS_L2;
  if (lossk != JSO_LOSS_L2 && lossk != JSO_LOSS_RELATIVE)
    return fail(c, JSO_E_INVALID, "unknown loss %d", lossk);
  const int fd_mode = opts ? opts->fd_mode : JSO_FD_REPLAY;
  if (fd_mode != JSO_FD_REPLAY && fd_mode != JSO_FD_SHARED)
    return fail(c, JSO_E_INVALID, "unknown fd_mode %d", fd_mode);
  DeviceGuard g(c->device);
  if (int rc = ensure_fx(c, s, c->debug_flags | (opts ? opts->flags : 0u))) return rc;
  HIP_TRY(c, hipMemsetAsync(s->scratch_loss, 0, 2 * sizeof(double), c->stream));
  Plan plan;
  plan_estimators({estimate_problem(s, seed, iteration, spp_prop, spp_fd, F, dF, img,
                                    s->scratch_loss, crop_of(s, opts),
                                    opts ? opts->pixel_mask : nullptr,
                                    c->debug_flags | (opts ? opts->flags : 0u), lossk,
                                    fd_mode)},
                  plan, c->launch_config);
  int rc = exec_plan(c, plan);
  if (rc) return rc;
  if (loss) {
    double l2[2];
    HIP_TRY(c, hipMemcpyAsync(l2, s->scratch_loss, sizeof(l2), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *loss = l2[iteration & 1u];
  }
  return JSO_OK;
}

int jso_precondition(jso_ctx* c, int id, float* g, float lambda) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!g) return fail(c, JSO_E_INVALID, "null gradient");
  if (!(lambda >= 0.0f && std::isfinite(lambda)))
    return fail(c, JSO_E_INVALID, "lambda must be finite and >= 0");
  if (s->dev.layout != JSO_LAYOUT_TEXTURE)
    return fail(c, JSO_E_INVALID, "preconditioning needs texture parameters");
  if (!preconditioned(s) || lambda == 0.0f) return JSO_OK;
  DeviceGuard dg(c->device);
  LaunchRec rec[4];
  for (LaunchRec& r : rec) {
    r.kind = Kern::Dct;
    r.timer = JSO_K_PRECOND;
  }
  push_precond(rec, s, g, s->pc_tmp, lambda, 0);
  return exec_plan(c, Plan{rec[0], rec[1], rec[2], rec[3]});
}

int jso_meta_step(jso_ctx* c, int id, const float* F, const float* dF, float eta, float beta_F,
                  float beta_D) {
  SceneGPU* s = get_scene(c, id);
  if (!s) return c ? fail(c, JSO_E_INVALID, "bad scene id %d", id) : JSO_E_INVALID;
  if (!F || !dF) return fail(c, JSO_E_INVALID, "null F/dF");
  if (!(beta_F >= 0.0f && beta_F < 1.0f && beta_D >= 0.0f && beta_D < 1.0f))
    return fail(c, JSO_E_INVALID, "beta must lie in [0, 1)");
  DeviceGuard g(c->device);
  LaunchRec r;
  r.kind = Kern::Meta;
  r.timer = JSO_K_META;
  const MetaArgs m = meta_args(s, F, dF, eta, beta_F, beta_D, 0);
  push_unit(r, m, m.nblocks);
  int rc = exec_plan(c, Plan{r});
  if (rc) return rc;
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
  LaunchRec r;
  r.kind = Kern::Adam;
  r.timer = JSO_K_ADAM;
  const AdamArgs a = adam_args(s, grad, eta, beta1, beta2, eps, 0);
  push_unit(r, a, a.nblocks);
  int rc = exec_plan(c, Plan{r});
  if (rc) return rc;
  s->host_iter++;
  return JSO_OK;
}

int read_stats(jso_ctx* c, const int* ids, int n, jso_step_stats* stats) {
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
  return JSO_OK;
}

int jso_grad_step(jso_ctx* c, const int* ids, int n, const jso_step_opts* o,
                  jso_step_stats* stats) {
  if (!c) return JSO_E_INVALID;
  if (!ids || n <= 0 || !o) return fail(c, JSO_E_INVALID, "null/empty argument");
  for (int k = 0; k < n; ++k) {
    if (!get_scene(c, ids[k])) return fail(c, JSO_E_INVALID, "bad scene id %d", ids[k]);
    for (int q = 0; q < k; ++q)
      if (ids[q] == ids[k]) return fail(c, JSO_E_INVALID, "scene %d listed twice", ids[k]);
  }
  int rc = check_step_opts(c, o);
  if (rc) return rc;
  rc = check_same_kind(c, ids, n);
  if (rc) return rc;
  DeviceGuard g(c->device);
  const uint32_t flags = c->debug_flags | o->flags;
  for (int k = 0; k < n; ++k)
    if (int rc2 = ensure_fx(c, get_scene(c, ids[k]), flags)) return rc2;
  std::vector<uint64_t> sig;
  auto bits = [](float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint64_t)u;
  };
  std::vector<SceneGPU*> ss;
  for (int k = 0; k < n; ++k) {
    sig.push_back((uint64_t)ids[k]);
    sig.push_back(get_scene(c, ids[k])->generation);
    ss.push_back(get_scene(c, ids[k]));
  }
  rc = check_precond_layout(c, ss, *o);
  if (rc) return rc;
  const int config = chosen_config(c, config_hash(ss, *o));
  sig.push_back((uint64_t)config);
  for (uint64_t v : {(uint64_t)o->optimizer, bits(o->eta), bits(o->beta_F), bits(o->beta_D),
                     (uint64_t)o->spp_prop, (uint64_t)o->spp_fd, bits(o->adam_beta1),
                     bits(o->adam_beta2), bits(o->adam_eps), (uint64_t)o->adam_spp, o->seed,
                     (uint64_t)flags, bits(o->precond_lambda), (uint64_t)o->loss,
                     (uint64_t)o->ablate, (uint64_t)o->fd_mode})
    sig.push_back(v);
  rc = exec_cached(c, sig, [&](Plan& plan) {
    std::vector<ProbPlan> ps, pv;
    for (int k = 0; k < n; ++k) {
      ps.push_back(step_problem(get_scene(c, ids[k]), *o, flags, 0));
      if (uncorrelated(*o)) pv.push_back(variance_problem(get_scene(c, ids[k]), *o, flags, 0));
    }
    plan_estimators(ps, plan, config);
    if (!pv.empty()) plan_estimators(pv, plan, config);
    plan_precond(ps, *o, plan);
    plan_optimizer(ps, *o, plan);
  });
  if (rc) return rc;
  for (int k = 0; k < n; ++k) get_scene(c, ids[k])->host_iter++;
  if (stats) return read_stats(c, ids, n, stats);
  return JSO_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
}  // extern "C"

struct jso_batch {
  jso_ctx* c = nullptr;
  std::vector<int> ids;
  std::vector<uint32_t> max_iters;
  jso_step_opts opts{};
  uint32_t flags = 0;
  bool use_graph = false;
  int config = 0;
  uint64_t hash = 0;
  Plan plan;
  uint8_t* dev = nullptr;  // unit arrays of the plan
  uint32_t* queues = nullptr;  // two work-queue counters per launch
  std::vector<size_t> off;
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void batch_release(jso_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->dev) (void)hipFree(b->dev);
  if (b->queues) (void)hipFree(b->queues);
  b->exec = nullptr;
  b->graph = nullptr;
  b->dev = nullptr;
  b->queues = nullptr;
  b->plan.clear();
  b->off.clear();
}

void batch_free(jso_batch* b) {
  batch_release(b);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

int batch_launch_all(jso_batch* b, hipStream_t st) {
  for (size_t k = 0; k < b->plan.size(); ++k) {
    const LaunchRec& r = b->plan[k];
    if (r.n == 0) continue;
    HIP_TRY(b->c, launch_rec(r, b->dev + b->off[k], nullptr, st, b->queues + 2 * k, b->c->n_cu));
  }
  return JSO_OK;
}

// (Re)build the batch's plan for a tile shape: descriptors uploaded once, the
// iteration captured in a graph when requested.
int batch_build(jso_batch* b, int config) {
  jso_ctx* c = b->c;
  HIP_TRY(c, hipStreamSynchronize(c->stream));  // the old descriptors may be in use
  batch_release(b);
  b->config = config;
  std::vector<ProbPlan> ps, pv;
  for (size_t k = 0; k < b->ids.size(); ++k) {
    SceneGPU* s = get_scene(c, b->ids[k]);
    if (!s) return fail(c, JSO_E_STATE, "scene %d of the batch was freed", b->ids[k]);
    if (int rc = ensure_fx(c, s, b->flags)) return rc;
    ps.push_back(step_problem(s, b->opts, b->flags, b->max_iters[k]));
    if (uncorrelated(b->opts)) pv.push_back(variance_problem(s, b->opts, b->flags, b->max_iters[k]));
  }
  plan_estimators(ps, b->plan, config);
  if (!pv.empty()) plan_estimators(pv, b->plan, config);
  plan_precond(ps, b->opts, b->plan);
  plan_optimizer(ps, b->opts, b->plan);
  const std::vector<uint8_t> all = pack_plan(b->plan, b->off);
  HIP_TRY(c, hipMalloc(reinterpret_cast<void**>(&b->dev), all.size()));
  HIP_TRY(c, hipMemcpy(b->dev, all.data(), all.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMalloc(reinterpret_cast<void**>(&b->queues), 2 * b->plan.size() * sizeof(uint32_t)));
  HIP_TRY(c, hipMemset(b->queues, 0, 2 * b->plan.size() * sizeof(uint32_t)));  // before any capture
  if (b->use_graph) {
    // capture on a private stream; replays run on the context's stream
    if (!b->capture) HIP_TRY(c, hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    HIP_TRY(c, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    const int rc = batch_launch_all(b, b->capture);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(b->capture, &graph);
    b->graph = graph;
    if (rc) return rc;
    HIP_TRY(c, e);
    HIP_TRY(c, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  return JSO_OK;
}

int batch_run(jso_batch* b, int iterations) {
  jso_ctx* c = b->c;
  for (int it = 0; it < iterations; ++it) {
    if (b->exec) {
      HIP_TRY(c, hipGraphLaunch(b->exec, c->stream));
    } else {
      const int rc = batch_launch_all(b, c->stream);
      if (rc) return rc;
    }
  }
  return JSO_OK;
}

// Device copies of the optimiser state of a batch's problems (the tuner runs
// real iterations and puts everything back afterwards).
struct StateCopy {
  std::vector<std::pair<void*, std::pair<void*, size_t>>> bufs;  // (copy, (live, bytes))
  ~StateCopy() {
    for (auto& x : bufs) (void)hipFree(x.first);
  }
};

int snapshot(jso_ctx* c, const std::vector<int>& ids, StateCopy& sc) {
  for (int id : ids) {
    SceneGPU* s = get_scene(c, id);
    const size_t P = s->P;
    const std::pair<void*, size_t> live[] = {
        {s->params, P * 4},      {s->params_prev, P * 4}, {s->F, P * 4},
        {s->dF, P * 4},          {s->mean, P * 8},        {s->var, P * 8},
        {s->alpha_prev, P * 8},  {s->m2F, P * 8},         {s->m2D, P * 8},
        {s->adam_m, P * 4},      {s->adam_v, P * 4},      {s->ctl, sizeof(Ctl)},
        {s->m1F, P * 8},         {s->m1D, P * 8},         {s->Fv, P * 4},
        {s->dFv, P * 4}};
    for (const auto& l : live) {
      void* copy = nullptr;
      HIP_TRY(c, hipMalloc(&copy, l.second));
      sc.bufs.push_back({copy, l});
      HIP_TRY(c, hipMemcpyAsync(copy, l.first, l.second, hipMemcpyDeviceToDevice, c->stream));
    }
  }
  return JSO_OK;
}

int restore(jso_ctx* c, const StateCopy& sc) {
  for (const auto& x : sc.bufs)
    HIP_TRY(c, hipMemcpyAsync(x.second.first, x.first, x.second.second,
                              hipMemcpyDeviceToDevice, c->stream));
  return JSO_OK;
}

}  // namespace

extern "C" {

int jso_batch_create(jso_ctx* c, const int* ids, int n, const jso_step_opts* o,
                     const uint32_t* max_iters, int use_graph, jso_batch** out) {
  if (!c) return JSO_E_INVALID;
  if (!out || !ids || n <= 0 || !o) return fail(c, JSO_E_INVALID, "null/empty argument");
  *out = nullptr;
  for (int k = 0; k < n; ++k) {
    if (!get_scene(c, ids[k])) return fail(c, JSO_E_INVALID, "bad scene id %d", ids[k]);
    for (int q = 0; q < k; ++q)
      if (ids[q] == ids[k]) return fail(c, JSO_E_INVALID, "scene %d listed twice", ids[k]);
  }
  int rc = check_step_opts(c, o);
  if (rc) return rc;
  rc = check_same_kind(c, ids, n);
  if (rc) return rc;
  DeviceGuard g(c->device);
  std::unique_ptr<jso_batch, void (*)(jso_batch*)> b(new (std::nothrow) jso_batch, batch_free);
  if (!b) return fail(c, JSO_E_OOM, "batch");
  b->c = c;
  b->ids.assign(ids, ids + n);
  b->max_iters.assign(n, 0u);
  if (max_iters) b->max_iters.assign(max_iters, max_iters + n);
  b->opts = *o;
  b->flags = c->debug_flags | o->flags;
  b->use_graph = use_graph != 0;
  std::vector<SceneGPU*> ss;
  for (int k = 0; k < n; ++k) ss.push_back(get_scene(c, ids[k]));
  rc = check_precond_layout(c, ss, *o);
  if (rc) return rc;
  b->hash = config_hash(ss, *o);
  rc = batch_build(b.get(), chosen_config(c, b->hash));
  if (rc) return rc;
  *out = b.release();
  return JSO_OK;
}

int jso_batch_step(jso_batch* b, int iterations) {
  if (!b) return JSO_E_INVALID;
  jso_ctx* c = b->c;
  if (iterations < 0) return fail(c, JSO_E_INVALID, "iterations < 0");
  DeviceGuard g(c->device);
  return batch_run(b, iterations);
}

int jso_batch_autotune(jso_batch* b, int iterations, int* best_config, double* ms) {
  if (!b) return JSO_E_INVALID;
  jso_ctx* c = b->c;
  if (iterations < 1) return fail(c, JSO_E_INVALID, "iterations < 1");
  DeviceGuard g(c->device);
  StateCopy sc;
  int rc = snapshot(c, b->ids, sc);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(c, hipEventCreate(&e0));
  std::unique_ptr<void, void (*)(void*)> g0(e0, [](void* e) { (void)hipEventDestroy((hipEvent_t)e); });
  HIP_TRY(c, hipEventCreate(&e1));
  std::unique_ptr<void, void (*)(void*)> g1(e1, [](void* e) { (void)hipEventDestroy((hipEvent_t)e); });
  int best = b->config;
  float best_ms = 0.0f;
  for (int config = 0; config < kConfigs; ++config) {
    rc = batch_build(b, config);
    if (rc) return rc;
    rc = batch_run(b, 1);  // warm-up (first launches of this configuration)
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(e0, c->stream));
    rc = batch_run(b, iterations);
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1));
    float t = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
    if (ms) ms[config] = t / (float)iterations;
    if (config == 0 || t < best_ms) {
      best = config;
      best_ms = t;
    }
    rc = restore(c, sc);
    if (rc) return rc;
  }
  {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[{c->arch, b->hash}] = best;
  }
  rc = batch_build(b, best);
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (best_config) *best_config = best;
  return JSO_OK;
}

int jso_set_launch_config(jso_ctx* c, int config) {
  if (!c) return JSO_E_INVALID;
  if (config < 0 || config >= kConfigs)
    return fail(c, JSO_E_INVALID, "launch configuration %d", config);
  c->launch_config = config;
  return JSO_OK;
}

int jso_batch_active(jso_batch* b, int* active) {
  if (!b) return JSO_E_INVALID;
  jso_ctx* c = b->c;
  if (!active) return fail(c, JSO_E_INVALID, "null output");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int a = 0;
  for (size_t k = 0; k < b->ids.size(); ++k) {
    SceneGPU* s = get_scene(c, b->ids[k]);
    if (!s) return fail(c, JSO_E_STATE, "scene %d of the batch was freed", b->ids[k]);
    uint32_t it = 0;
    HIP_TRY(c, hipMemcpy(&it, &s->ctl->iteration, sizeof(it), hipMemcpyDeviceToHost));
    if (b->max_iters[k] == 0 || it < b->max_iters[k]) ++a;
  }
  *active = a;
  return JSO_OK;
}

int jso_batch_destroy(jso_batch* b) {
  if (!b) return JSO_OK;
  DeviceGuard g(b->c->device);
  (void)hipStreamSynchronize(b->c->stream);
  batch_free(b);
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

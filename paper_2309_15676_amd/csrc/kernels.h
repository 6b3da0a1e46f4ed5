// Host/device interface of the jso kernels (argument blocks and launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jso {

struct DevScene;

// Per-problem control block, resident on the device so a captured iteration
// can be replayed without host involvement.
struct Ctl {
  double norm2[2];        // ||pi_i - pi_{i-1}||^2, double-buffered by iteration parity
  double loss[2];         // L2 loss of the proportional primal, by iteration parity
  uint32_t iteration;     // i
  uint32_t count_F;       // Moment2 step counts
  uint32_t count_D;
  uint32_t adam_t;
  uint32_t blocks_done;   // last-block-done counter of the optimiser kernels
  uint32_t pad[3];
};

struct Crop {
  int x0, y0, x1, y1;
};

struct KeyArgs {
  uint64_t seed;
  uint32_t iteration;        // used when iter_ptr is null
  const uint32_t* iter_ptr;  // device iteration counter (graph replays)
};

constexpr int kMetaMaxBlocks = 1024;

// Path radiance is handed from the forward kernel to its consumers through
// per-path slots: slot k of pixel p holds 3 doubles at ((k * npix) + p) * 3.
constexpr int kMaxSlots = 8;  // path slots per pixel per launch

// One grid slice of k_forward: the paths of one sample of one parameter set.
struct FwdSlice {
  const float* params;
  uint32_t tag;     // random stream
  uint32_t sample;  // sample index within the stream
  int slot;         // output slot
};

struct FwdArgs {
  FwdSlice sl[kMaxSlots];
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  double* slots;
  uint32_t npix;
  uint32_t flags;
  unsigned long long* work;  // nullable: [2] += paths traced, [3] += their surface vertices
};

// One primal image of k_finalize: n slots of this launch summed per pixel,
// accumulated across launches in `accum`; the last launch writes the image,
// the adjoint image and the loss.
struct FinJob {
  int slot0, n;
  double* accum;    // per-pixel running sums (3 doubles), used unless first && last
  int first, last;
  double inv_spp;   // 1 / total samples of the image
  float* img;       // nullable
  float* delta;     // nullable: 2 (I - T) / (3 W H)
  double* loss2;    // nullable: 2 loss slots indexed by iteration parity
};

struct FinArgs {
  FinJob jobs[3];
  int n_jobs;
  const double* slots;
  uint32_t npix;
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  const float* target;
  float delta_scale;   // 2 / (3 W H)
  double loss_scale;   // 1 / (3 W H)
};

// One grid slice of k_adjoint: the replay of one sample of one job, a single
// path (params_b null) or a finite-difference pair (+A - B).
struct RepSlice {
  const float* params;
  const float* params_b;
  const float* delta;    // adjoint image of path A
  const float* delta_b;
  float* grad;
  float sign;            // sign of a single path's contribution
  float adj_scale;       // 1 / spp
  uint32_t tag;
  uint32_t sample;
  int slot_a, slot_b;    // forward radiance slots
};

struct RepArgs {
  RepSlice sl[kMaxSlots];
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  const double* slots;
  uint32_t npix;
  uint32_t flags;
  unsigned long long* work;  // nullable: [0] += paths replayed, [1] += their surface vertices
};

struct MetaArgs {
  float* params;
  float* params_prev;
  float* F;
  float* dF;
  double *mean, *var, *alpha_prev, *m2F, *m2D;
  Ctl* ctl;
  double* partials;  // kMetaMaxBlocks per-block sums of the squared step
  size_t n;
  int n_ch;
  float lo[5], hi[5];
  double beta_F, beta_D;
  float eta;
  int zero_grads;
};

struct AdamArgs {
  float* params;
  float* params_prev;
  float* g;
  float *m, *v;
  Ctl* ctl;
  size_t n;
  int n_ch;
  float lo[5], hi[5];
  float eta, beta1, beta2, eps;
  int zero_grads;
};

hipError_t launch_philox(const uint32_t* ctr, size_t n, uint64_t key, uint32_t* out,
                         hipStream_t st);
// S: the scene in device memory (uniform reads go through the scalar cache);
// n: grid slices (A.sl entries used)
hipError_t launch_forward(const DevScene* S, const FwdArgs& A, int n, hipStream_t st);
// width: image width (pixel index = y * width + x)
hipError_t launch_finalize(const FinArgs& A, int width, hipStream_t st);
// n_ch: channels per texel of the parameter texture (0..5; sizes the LDS table)
hipError_t launch_adjoint(const DevScene* S, const RepArgs& A, int n, int n_ch, hipStream_t st);
hipError_t launch_meta(const MetaArgs& A, hipStream_t st);
hipError_t launch_adam(const AdamArgs& A, hipStream_t st);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);

}  // namespace jso

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

constexpr int kMaxPrimalJobs = 4;
constexpr int kMetaMaxBlocks = 1024;
constexpr int kMaxAdjointJobs = 4;

struct PrimalJob {
  const float* params;
  uint32_t tag;
  int spp;
  float* delta;   // adjoint image out (nullable)
  float* img;     // primal image out (nullable)
  double* loss2;  // 2 loss slots indexed by iteration parity (nullable)
};

struct PrimalArgs {
  PrimalJob jobs[kMaxPrimalJobs];
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
  const float* target;
  float delta_scale;   // 2 / (3 W H)
  double loss_scale;   // 1 / (3 W H)
  uint32_t flags;
};

struct AdjointJob {
  const float* params;    // path A parameters
  const float* delta;     // path A adjoint image
  const float* params_b;  // finite-difference pair: path B parameters (nullable)
  const float* delta_b;
  float* grad;
  float sign;             // sign of path A's contribution (pairs: +A - B)
  float adj_scale;        // 1 / spp
  uint32_t tag;
  int sample0;            // first sample index of this job
  int z0;                 // first grid slice of this job (one slice per sample)
};

struct AdjointArgs {
  AdjointJob jobs[kMaxAdjointJobs];
  int n_jobs;
  KeyArgs key;
  Crop crop;
  const uint8_t* mask;
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
// S: the scene in device memory (uniform reads go through the scalar cache)
hipError_t launch_primal(const DevScene* S, const PrimalArgs& A, int n_jobs, hipStream_t st);
hipError_t launch_adjoint(const DevScene* S, const AdjointArgs& A, int n_slices, hipStream_t st);
hipError_t launch_meta(const MetaArgs& A, hipStream_t st);
hipError_t launch_adam(const AdamArgs& A, hipStream_t st);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);

}  // namespace jso

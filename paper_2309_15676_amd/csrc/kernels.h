// Host/device interface of the jso kernels (argument blocks and launchers).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace jso {

struct DevScene;

// Device pointers inside launch descriptors point to global memory.  The
// descriptors themselves live in device memory, and a pointer loaded from
// memory is generic unless its type says otherwise; declaring the fields in
// the global address space keeps the kernels' loads global (and scalar for
// uniform data such as the scene).
#define JSO_GMEM __attribute__((address_space(1)))
template <class T>
__host__ __device__ inline JSO_GMEM T* gmem(T* p) {
  return (JSO_GMEM T*)p;
}
// Read-only data that no kernel writes (the scene) is declared in the
// constant address space: uniform reads of it stay scalar even next to the
// kernels' stores and atomics.
#define JSO_CMEM __attribute__((address_space(4)))
template <class T>
__host__ __device__ inline JSO_CMEM const T* cmem(const T* p) {
  return (JSO_CMEM const T*)p;
}

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
  JSO_GMEM const uint32_t* iter_ptr;  // device iteration counter (graph replays)
};

constexpr int kMetaMaxBlocks = 1024;

// Every launch of the path and optimiser kernels covers one or more units:
// the work of one problem, or of one group of its grid slices.  A unit owns
// the grid blocks [block0, next unit's block0); units are sorted by block0
// and live in device memory, so one launch serves any number of problems of
// uneven size.
struct UnitHead {
  uint32_t block0;    // first grid block of the unit
  uint32_t max_iter;  // nonzero: the unit is idle once its problem's iteration reaches it
};

// Path radiance is handed from the forward kernel to its consumers through
// per-path slots: slot k of pixel p holds 3 doubles at ((k * npix) + p) * 3.
constexpr int kMaxSlots = 8;  // path slots per pixel per launch

// Hit records of replayed paths (device.h describes them): kHitRecs records of
// kRecWords words per path, record k of slot s and pixel p at
// ((s * kHitRecs + k) * npix + p) * kRecWords.
constexpr int kHitRecs = 3;
constexpr int kRecWords = 3;

// One grid slice of k_forward: the paths of one sample of one parameter set.
struct FwdSlice {
  JSO_GMEM const float* params;
  // non-null: a shared-path pair (Eq. 5): the paths drawn at `params` are also
  // evaluated at params_b, whose radiance goes to slot_b
  JSO_GMEM const float* params_b;
  uint32_t tag;     // random stream
  uint32_t sample;  // sample index within the stream
  int slot;         // output slot
  int slot_b;
};

struct FwdArgs {
  UnitHead h;
  JSO_CMEM const DevScene* scene;  // read-only
  FwdSlice sl[kMaxSlots];
  int n_slices;
  KeyArgs key;
  Crop crop;
  JSO_GMEM const uint8_t* mask;
  JSO_GMEM double* slots;
  uint32_t npix;
  uint32_t flags;
  uint32_t tiles_x, tiles;  // tiles of the crop (launch's tile shape): per row, per slice
  // hit records: slices with bit i of rec_mask set write them for their paths
  // (the forward pass of paths that a replay in the same plan reads back);
  // rec_epoch is the plan's, mixed into every record's tag
  JSO_GMEM uint32_t* recs;
  uint32_t rec_mask;
  uint32_t rec_epoch;
};

// One primal image of k_finalize: n slots of this launch summed per pixel,
// accumulated across launches in `accum`; the last launch writes the image,
// the adjoint image and the loss.
struct FinJob {
  int slot0, n;
  JSO_GMEM double* accum;  // per-pixel running sums (3 doubles), used unless first && last
  int first, last;
  double inv_spp;   // 1 / total samples of the image
  JSO_GMEM float* img;     // nullable
  JSO_GMEM float* delta;   // nullable: 2 (I - T) / (3 W H)
  JSO_GMEM double* loss2;  // nullable: 2 loss slots indexed by iteration parity
};

struct FinArgs {
  UnitHead h;
  FinJob jobs[3];
  int n_jobs;
  JSO_GMEM const double* slots;
  uint32_t npix;
  int width;
  KeyArgs key;
  Crop crop;
  JSO_GMEM const uint8_t* mask;
  JSO_GMEM const float* target;
  float delta_scale;   // 2 / (3 W H)
  double loss_scale;   // 1 / (3 W H)
  uint32_t nblocks;    // blocks per job
  int relative;        // relative loss: each term over T^2 + kRelEps
};
constexpr float kRelEps = 0.01f;

// One grid slice of k_adjoint: the replay of one sample of one job, a single
// path (params_b null) or a finite-difference pair (+A - B): two paths from the
// same random numbers, each drawn at its own parameters, or (shared) one path
// drawn at A's parameters with a second ledger evaluated at B's.
struct RepSlice {
  JSO_GMEM const float* params;
  JSO_GMEM const float* params_b;
  JSO_GMEM const float* delta;  // adjoint image of path A
  JSO_GMEM const float* delta_b;
  JSO_GMEM float* grad;
  float sign;            // sign of a single path's contribution
  float adj_scale;       // 1 / spp
  uint32_t tag;
  uint32_t sample;
  int slot_a, slot_b;    // forward radiance slots
  // deterministic mode: 64-bit fixed-point accumulators of grad (contributions
  // in units of 1 / fx_scale), folded into grad by k_fx_flush; null: FP32
  // atomics into grad
  JSO_GMEM unsigned long long* fx;
  double fx_scale;
};

struct RepArgs {
  UnitHead h;
  JSO_CMEM const DevScene* scene;  // read-only
  RepSlice sl[kMaxSlots];
  int n_slices;
  KeyArgs key;
  Crop crop;
  JSO_GMEM const uint8_t* mask;
  JSO_GMEM const double* slots;
  uint32_t npix;
  uint32_t flags;
  uint32_t tiles_x, tiles;
  // nonzero: every slice is a replay pair (params_b set, not shared), traced on
  // lane pairs over tiles of half the tile shape's height (tiles_x, tiles
  // count those)
  int pair_lanes;
  // the forward pass's hit records of these slices' paths (FwdArgs), or null:
  // trace every ray again
  JSO_GMEM uint32_t* recs;
  uint32_t rec_epoch;
};

// One fixed-point gradient accumulator of the deterministic mode: grad[i] +=
// fx[i] / fx_scale, then fx[i] = 0 (ready for the next step).
struct FxArgs {
  UnitHead h;
  JSO_GMEM unsigned long long* fx;
  JSO_GMEM float* grad;
  size_t n;
  double inv_scale;
  uint32_t nblocks;
};
constexpr int kFxBlock = 256;

// The bricked copy of one volume parameter vector that the volume kernels
// read: dst holds vol_rb^3 bricks of 4x4x4 voxels in (z, y, x) brick order,
// the 64 voxels of a brick in Morton order (bit 0 x, bit 1 y, bit 2 z, then
// the second bits), so each 128-byte line is a 2x2x2 block of voxels; voxels
// past the grid's edge are zero.  src: the parameters in the interface's
// layout ((z R + y) R + x) * 4 + channel.
struct BrickArgs {
  UnitHead h;
  JSO_GMEM const float4* src;
  JSO_GMEM float4* dst;
  int R, Rb;
  uint32_t nblocks;
};
constexpr int kBrickBlock = 256;

struct MetaArgs {
  UnitHead h;
  uint32_t nblocks;
  JSO_GMEM float* params;
  JSO_GMEM float* params_prev;
  JSO_GMEM float* F;
  JSO_GMEM float* dF;
  JSO_GMEM double *mean, *var, *alpha_prev, *m2F, *m2D;
  JSO_GMEM Ctl* ctl;
  JSO_GMEM double* partials;  // kMetaMaxBlocks per-block sums of the squared step
  size_t n;
  int n_ch;
  float lo[5], hi[5];
  double beta_F, beta_D;
  float eta;
  int zero_grads;
  // ablations (JSO_ABLATE_*): centred EMAs keep their first moments in
  // m1F / m1D; uncorrelated variance samples come from Fv / dFv
  uint32_t ablate;
  JSO_GMEM double *m1F, *m1D;
  JSO_GMEM float *Fv, *dFv;
};

struct AdamArgs {
  UnitHead h;
  uint32_t nblocks;
  JSO_GMEM float* params;
  JSO_GMEM float* params_prev;
  JSO_GMEM float* g;
  JSO_GMEM float *m, *v;
  JSO_GMEM Ctl* ctl;
  size_t n;
  int n_ch;
  float lo[5], hi[5];
  float eta, beta1, beta2, eps;
  int zero_grads;
};

// One pass of the texture-gradient preconditioner: a cosine transform along
// one texture axis, out(m, j) = sum_k A[m][k] in(k, j) (A^T with transA),
// optionally scaled by 1 / (1 + lambda (eig_m[m] + eig_j[j / jdiv])).  Element
// (k, j) of a vector lives at k * sk + (j / jin) * sjo + (j % jin).  One unit =
// one vector of one problem; it owns tiles_m * tiles_j blocks of kDctTile^2
// outputs.
struct DctArgs {
  UnitHead h;
  JSO_GMEM const float* A;      // n x n, row-major
  JSO_GMEM const float* in;
  JSO_GMEM float* out;          // never aliases in
  JSO_GMEM const float* eig_m;  // n entries, or null: no scaling
  JSO_GMEM const float* eig_j;
  int n, N, sk, jin, sjo, jdiv, transA;
  float lambda;
  uint32_t tiles_j;
};
constexpr int kDctTile = 64;   // outputs per block side
constexpr int kDctBlock = 256;

hipError_t launch_philox(const uint32_t* ctr, size_t n, uint64_t key, uint32_t* out,
                         hipStream_t st);
hipError_t launch_dct(const DctArgs* U, int n, uint32_t blocks, hipStream_t st);
// Unit arrays U[n] in device memory; `blocks` = the total grid size.
// work (nullable): forward [2] += paths traced, [3] += surface vertices;
// adjoint [0] += paths replayed, [1] += surface vertices.
// shape: index into kShapeW / kShapeH (the tiles the units were built for)
// stack: BVH traversal-stack entries per lane (the deepest mesh among the
// units' scenes; 0 = no scene of the launch has a mesh), at most kBvhMaxStack
// shared: the units may hold shared-path pair slices (forward: params_b set;
// adjoint: pair slices are then all shared-path pairs, none a replay pair)
// queue (nullable): a persistent launch of min(blocks, persist) blocks that
// pull the `blocks` tiles from queue[0..1] (two zeroed counters, left zeroed)
hipError_t launch_forward(const FwdArgs* U, int n, uint32_t blocks, int shape, int stack,
                          bool shared, unsigned long long* work, hipStream_t st,
                          uint32_t* queue = nullptr, uint32_t persist = 0);
hipError_t launch_finalize(const FinArgs* U, int n, uint32_t blocks, hipStream_t st);
// lds: dynamic LDS bytes (adjoint_lds_bytes of the largest channel count)
// det: the units' slices carry fixed-point accumulators (deterministic mode)
hipError_t launch_adjoint(const RepArgs* U, int n, uint32_t blocks, int shape, size_t lds,
                          int stack, bool shared, unsigned long long* work, hipStream_t st,
                          uint32_t* queue = nullptr, uint32_t persist = 0, bool det = false);
// The same for emission-absorption volume scenes (every unit's scene a volume;
// the slices' parameter pointers are bricked copies made by launch_vol_brick;
// the gradients are in the interface's layout)
// The volume forward takes 8x8 pixel tiles and `waves` slices per block, one
// wave each (1 <= waves <= kVolMaxSliceWaves; blocks of a unit: tiles x
// ceil(n_slices / waves)), whatever the configuration's tile shape.
constexpr int kVolMaxSliceWaves = 8;
hipError_t launch_vol_forward(const FwdArgs* U, int n, uint32_t blocks, int waves,
                              unsigned long long* work, hipStream_t st);
hipError_t launch_vol_adjoint(const RepArgs* U, int n, uint32_t blocks, int shape,
                              unsigned long long* work, hipStream_t st);
hipError_t launch_vol_brick(const BrickArgs* U, int n, uint32_t blocks, hipStream_t st);
hipError_t launch_meta(const MetaArgs* U, int n, uint32_t blocks, hipStream_t st);
hipError_t launch_fx_flush(const FxArgs* U, int n, uint32_t blocks, hipStream_t st);
hipError_t launch_adam(const AdamArgs* U, int n, uint32_t blocks, hipStream_t st);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);

// Grid geometry the host needs to build units.
// Pixel tiles of the path kernels (one block = one tile): 16x16 (256 lanes),
// 16x8 (128) and 8x8 (64), chosen per plan.
constexpr int kShapes = 3;
constexpr int kShapeW[kShapes] = {16, 16, 8};
constexpr int kShapeH[kShapes] = {16, 8, 8};
constexpr int kFinBlock = 256;   // k_finalize threads per block
constexpr int kFinMaxBlocks = 256;
constexpr int kMetaBlock = 256;  // k_meta / k_adam threads per block
constexpr int kMetaK = 4;        // parameters per k_meta thread
size_t adjoint_lds_bytes(int n_ch);

}  // namespace jso

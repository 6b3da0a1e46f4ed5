// HIP kernels of the jso hot path (gfx950).
//
//   k_philox   - Philox4x32-10 block function over a counter array
//   k_forward  - forward path tracing: each path's radiance into a slot
//                (primal samples, and the adjoint paths' forward passes)
//   k_finalize - primal image from its slots; L2 adjoint image
//                2 (I - T) / (3 W H) and the loss
//   k_adjoint  - replayed adjoint: a second pass over each path's random
//                numbers that forms the per-vertex material derivatives and
//                scatters them; a finite-difference slice replays the paths at
//                pi_i and pi_{i-1} in lockstep and differences coinciding
//                vertices in registers
//   k_meta     - fused meta-estimator + stabilised step (FP64 state)
//   k_adam     - Adam baseline
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "device.h"
#include "kernels.h"

namespace jso {

// A descriptor's global-memory pointer as an ordinary pointer; its uses stay
// in the global address space.
template <class T>
__device__ __forceinline__ T* G(JSO_GMEM T* p) {
  return (T*)p;
}
template <class T>
__device__ __forceinline__ const T* G(JSO_CMEM const T* p) {
  return (const T*)p;
}

// ---------------------------------------------------------------------------
__global__ void k_philox(const uint4* __restrict__ ctr, uint32_t n, uint32_t k0, uint32_t k1,
                         uint4* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = philox10(ctr[i], k0, k1);
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t iteration_of(const KeyArgs& k) {
  return k.iter_ptr ? *k.iter_ptr : k.iteration;
}

__device__ __forceinline__ Rng make_rng(uint64_t key, uint32_t pixel, uint32_t sample) {
  Rng r;
  r.k0 = (uint32_t)key;
  r.k1 = (uint32_t)(key >> 32);
  r.pixel = pixel;
  r.sample = sample;
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// A block is one TW x TH pixel tile (lane = y * TW + x; 16 x 16 = four
// wave64 rows of 16 x 4).
template <int TW, int TH>
struct Shape {
  static constexpr int W = TW, H = TH, N = TW * TH, WAVES = N / 64;
  static_assert(N % 64 == 0 && (TW & (TW - 1)) == 0, "tile shape");
};

// The unit owning grid block b: the last one whose block0 <= b.
template <class U>
__device__ __forceinline__ const U& unit_of(const U* __restrict__ u, int n, uint32_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (u[mid].h.block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return u[lo];
}
template <class U>
__device__ __forceinline__ const U& unit_of(const U* __restrict__ u, int n) {
  return unit_of(u, n, blockIdx.x);
}

// A path unit's block: its slice and its tile's pixel origin.
struct TileBlock {
  int slice, x0, y0;
};

// kRuns: a unit's blocks take its tiles in order, the slices of one tile side
// by side (they trace paths through the same pixels, so they touch the same
// part of the scene at about the same time); otherwise slice by slice, each
// slice's tiles in order.  The shared-path kernel instances keep the second
// order: with the first, their single-path replays gave wrong proportional
// gradients whenever the shared-path replays ran beside them (a fault of
// those instances that depends on where the blocks run, its cause not found).
// th: the tile height in pixels (SH::H, or SH::H / 2 for lane-pair tiles)
template <class SH, bool kRuns, class U>
__device__ __forceinline__ TileBlock tile_block(const U& u, uint32_t b, int th = SH::H) {
  const uint32_t local = b - u.h.block0;
  if constexpr (kRuns) {
    const uint32_t ns = (uint32_t)u.n_slices;
    const uint32_t t = local / ns;
    return TileBlock{(int)(local - t * ns), u.crop.x0 + (int)(t % u.tiles_x) * SH::W,
                     u.crop.y0 + (int)(t / u.tiles_x) * th};
  } else {
    const uint32_t t = local % u.tiles;
    return TileBlock{(int)(local / u.tiles), u.crop.x0 + (int)(t % u.tiles_x) * SH::W,
                     u.crop.y0 + (int)(t / u.tiles_x) * th};
  }
}

template <class SH>
__device__ __forceinline__ bool tile_pixel(const Crop& c, const TileBlock& tb, int& px, int& py) {
  px = tb.x0 + (int)(threadIdx.x % SH::W);
  py = tb.y0 + (int)(threadIdx.x / SH::W);
  return px < c.x1 && py < c.y1;
}

// ---------------------------------------------------------------------------
// in-block path compaction
//
// A wave steps its paths vertex by vertex for as long as its longest path
// lives, and most paths end at their first surface vertex.  Each block takes
// every path's first vertex in place (neighbouring pixels: coherent texture
// and scene accesses), then moves the surviving paths into its lowest lanes,
// kXchg at a time through LDS, and finishes them on as few waves as they
// fill.  Waves left without a path exit at once, which returns their
// registers to the CU for other blocks.  A moved path keeps the pixel
// identity of the lane it came from (src), so it draws the same random
// numbers and writes to the same pixel.
// ---------------------------------------------------------------------------
constexpr int kXchg = 32;  // paths per exchange round
// Survivors are packed only when that frees at least one wave (a one-wave
// block never packs).
template <class SH>
constexpr int compact_max() {
  return SH::N - 64;
}

// The hit records of the path of pixel `pix` in slot `slot` (recs null: none).
__device__ __forceinline__ HitRecs hit_recs(JSO_GMEM uint32_t* recs, int slot, uint32_t npix,
                                            uint32_t pix, uint32_t epoch) {
  return HitRecs{recs ? recs + ((size_t)slot * kHitRecs * npix + pix) * kRecWords : nullptr,
                 npix * (uint32_t)kRecWords, epoch};
}

// Identity of the paths of one block: tile origin and random stream.
template <class SH>
struct BlockPaths {
  uint64_t key;
  uint32_t sample;
  int x0, y0, width;
  uint32_t flags;
  __device__ __forceinline__ uint32_t pixel(int src) const {
    return (uint32_t)((y0 + src / SH::W) * width + (x0 + src % SH::W));
  }
  __device__ __forceinline__ Rng rng(int src) const { return make_rng(key, pixel(src), sample); }
};

template <class SH>
__device__ __forceinline__ BlockPaths<SH> block_paths(const TileBlock& tb, const DevScene& S,
                                                      uint64_t key, uint32_t sample,
                                                      uint32_t flags) {
  return BlockPaths<SH>{key, sample, tb.x0, tb.y0, S.width, flags};
}

// Rank of this lane among the lanes of the block with `flag` set, and their
// number (block-uniform).  Every lane of the block must call it.
template <class SH>
__device__ __forceinline__ int block_rank(bool flag, int& total, int* s_cnt) {
  const uint64_t m = __ballot(flag);
  const int lane = (int)__lane_id(), wv = (int)threadIdx.x >> 6;
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) s_cnt[wv] = __popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SH::WAVES; ++w) {
    const int c = s_cnt[w];
    off += w < wv ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return off + below;
}

// LDS exchange buffer, word-major (word i of slot k at i * kXchg + k), so a
// wave's accesses fall in distinct banks.
template <class T>
__device__ __forceinline__ void xchg_put(uint32_t* buf, int slot, const T& v) {
  static_assert(sizeof(T) % 4 == 0, "exchange item size");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) buf[i * kXchg + slot] = w[i];
}

template <class T>
__device__ __forceinline__ void xchg_get(const uint32_t* buf, int slot, T& v) {
  uint32_t w[sizeof(T) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = buf[i * kXchg + slot];
  __builtin_memcpy(&v, w, sizeof(T));
}

// Move the item of every lane with `live` set (rank r among n) to lane r.
// Lanes below n receive one item in `out`; the others keep theirs.
template <class T>
__device__ __forceinline__ void pack(uint32_t* buf, bool live, int r, int n, const T& in, T& out) {
  const int t = (int)threadIdx.x;
  for (int base = 0; base < n; base += kXchg) {
    if (live && r >= base && r < base + kXchg) xchg_put(buf, r - base, in);
    __syncthreads();
    if (t >= base && t < base + kXchg && t < n) xchg_get(buf, t - base, out);
    __syncthreads();
  }
}

__device__ __forceinline__ void store_radiance(double* __restrict__ out, uint32_t pix,
                                               const double led[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) out[3 * (size_t)pix + k] = led[k];
}

// Work counters: one 64-bit atomic per wave and counter.
__device__ __forceinline__ void count_work(unsigned long long* w, int paths, int verts) {
  if (!w) return;
  paths = wave_sum(paths);
  verts = wave_sum(verts);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(w, (unsigned long long)paths);
    atomicAdd(w + 1, (unsigned long long)verts);
  }
}

struct FwdItem {
  Path P;
  int src, pad_;
};

struct FwdItem2 {  // a shared-path pair: the path and its second ledger
  Path P;
  Ledger2 L2;
  int src, pad_;
};

constexpr int kFwdXchgWords = (int)(sizeof(FwdItem) / 4);
constexpr int kFwd2XchgWords = (int)(sizeof(FwdItem2) / 4);

// The second ledger of an exchange item (single paths have none: `none`).
__device__ __forceinline__ Ledger2& ledger2(FwdItem2& w, Ledger2&) { return w.L2; }
__device__ __forceinline__ Ledger2& ledger2(FwdItem&, Ledger2& none) { return none; }

// ---------------------------------------------------------------------------
// forward pass: one block = one tile of one slice; each path's radiance (its
// FP64 ledger total) goes to the slice's slot.
// ---------------------------------------------------------------------------
// The kernel bodies take the scene through a restrict-qualified parameter:
// nothing the kernels write aliases it, so its fields stay in registers.
// kTwo: the slice is a shared-path pair (params_b set): each path also
// carries the ledger of params_b, stored to slot_b.
// kRec: REC_WRITE where the slice's bit of rec_mask asks for hit records.
template <class SH, bool kMesh, bool kTwo, int kRec = REC_NONE>
__device__ __forceinline__ void forward_tile(const FwdArgs& A, const DevScene* __restrict__ Sp,
                                             const TileBlock& tb, uint32_t iter,
                                             uint32_t* s_xchg, int* s_cnt, const TravStack& st,
                                             unsigned long long* work) {
  using Item = typename std::conditional<kTwo, FwdItem2, FwdItem>::type;
  const DevScene& S = *Sp;
  const FwdSlice& sl = A.sl[tb.slice];
  int px, py;
  const bool inside = tile_pixel<SH>(A.crop, tb, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  const uint64_t key = stream_key(A.key.seed, iter, sl.tag);
  const BlockPaths<SH> B = block_paths<SH>(tb, S, key, sl.sample, A.flags);
  double* out = G(A.slots) + (size_t)sl.slot * A.npix * 3;
  double* out_b = kTwo ? G(A.slots) + (size_t)sl.slot_b * A.npix * 3 : nullptr;
  const float* params_b = kTwo ? G(sl.params_b) : nullptr;
  const float zero[3] = {0.0f, 0.0f, 0.0f};
  VertexGrad vg;
  int n_vert = 0;
  Item mine;
  Ledger2 none;
  Path& P = mine.P;
  Ledger2& L2 = ledger2(mine, none);
  P.alive = false;
  JSO_GMEM uint32_t* recs = nullptr;
  if constexpr (kRec != REC_NONE) recs = ((A.rec_mask >> tb.slice) & 1u) ? A.recs : nullptr;
  if (active) {
    const Rng rng = B.rng((int)threadIdx.x);
    const HitRecs hr = hit_recs(recs, sl.slot, A.npix, pix, A.rec_epoch);
    path_begin<kMesh, kRec>(S, st, rng, px, py, A.flags, P, hr);
    if (kTwo) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        L2.led[k] = P.led[k];  // what the camera ray sees does not depend on the material
        L2.beta[k] = 1.0f;
      }
    }
    if (P.alive) {
      ++n_vert;
      path_vertex2<false, kMesh, kTwo, kRec>(S, st, G(sl.params), params_b, rng, A.flags, P, L2,
                                             zero, zero, vg, hr);
    }
    if (!P.alive) {
      store_radiance(out, pix, P.led);
      if (kTwo) store_radiance(out_b, pix, L2.led);
    }
  }
  int n;
  const bool alive = P.alive;
  const int r = block_rank<SH>(alive, n, s_cnt);
  mine.src = (int)threadIdx.x;
  Item W;
  if (n > compact_max<SH>()) {
    W = mine;
  } else {
    W.P.alive = false;
    W.src = (int)threadIdx.x;
    if (n > 0) pack(s_xchg, alive, r, n, mine, W);
  }
  // no barrier below: waves without a path leave
  if (W.P.alive) {
    const Rng rng = B.rng(W.src);
    Ledger2& WL = ledger2(W, none);
    const HitRecs hr = hit_recs(recs, sl.slot, A.npix, B.pixel(W.src), A.rec_epoch);
    while (W.P.alive) {
      ++n_vert;
      path_vertex2<false, kMesh, kTwo, kRec>(S, st, G(sl.params), params_b, rng, A.flags, W.P,
                                             WL, zero, zero, vg, hr);
    }
    store_radiance(out, B.pixel(W.src), W.P.led);
    if (kTwo) store_radiance(out_b, B.pixel(W.src), WL.led);
  }
  count_work(work ? work + 2 : nullptr, active ? 1 : 0, n_vert);
}

// ---------------------------------------------------------------------------
// persistent launches
//
// With a work queue (queue != null) a path kernel runs a fixed grid whose
// blocks pull grid-block indices (tiles of units) from queue[0] until `total`
// are taken; the last block to finish resets queue[0] and queue[1] (the count
// of finished blocks) to zero for the next launch.  Without one, block b is
// blockIdx.x, renumbered by xcd_runs in the kernel instances that order their
// tiles in runs (tile_block).  The barriers of the pull also separate one tile's use
// of the block's LDS from the next tile's: waves that leave a tile early wait
// there for the others.
// ---------------------------------------------------------------------------
// The block numbers of a path launch in the order the XCDs take them.  The
// hardware deals a grid's blocks out to the 8 XCDs in turn (block i to XCD
// i mod 8), each XCD with an L2 of its own.  Renumbered, XCD x takes runs of
// kXcdRun consecutive blocks (a tile with all its slices, when a step has 8:
// paths through the same pixels) and the XCDs take turns run by run, so the
// slices of a tile share one L2 while the XCDs still take neighbouring tiles
// in turn (an object in the middle of the view spreads over all of them).  A
// bijection of [0, n): blocks past the last whole round of 8 runs keep their
// numbers.  Runs of 8 measured best: against 64 (8 tiles) the 200k-triangle
// sphere step took 5.2 instead of 7.4 ms, the terrain 23.4 instead of 23.6.
// A launch whose units hold one slice each (a one-sample replayed adjoint)
// has no slices to keep together and takes runs of 1: plain turns, tile by
// tile (runs of 8 tiles there load the XCDs unevenly).
constexpr uint32_t kXcdRun = 8;
__device__ __forceinline__ uint32_t xcd_runs(uint32_t i, uint32_t n, uint32_t run) {
  const uint32_t round = 8 * run, full = n - n % round;
  if (i >= full) return i;
  const uint32_t x = i & 7u, k = i >> 3;
  return ((k / run) * 8 + x) * run + k % run;
}

// The run length of a launch: `run` when its first or last unit holds more
// than one slice (the units of a launch share their slice layout, except
// that a replay launch puts its pair units, one slice, before its single
// units), else 1.  The replay takes runs of kXcdRunReplay blocks (its tiles
// hold one or two slices, so a run is 32-64 neighbouring tiles): measured
// against runs of 8, the terrain step 23.4 -> 23.1 ms and the 200k-triangle
// sphere 5.22 -> 5.09 ms.
constexpr uint32_t kXcdRunReplay = 64;
template <class U>
__device__ __forceinline__ uint32_t xcd_run_of(const U* __restrict__ u, int n, uint32_t run) {
  return (u[0].n_slices > 1 || u[n - 1].n_slices > 1) ? run : 1u;
}

template <bool kRuns>
__device__ __forceinline__ bool next_block(uint32_t* queue, uint32_t total, uint32_t* s_vb,
                                           bool first, uint32_t& vb, uint32_t run) {
  if (!queue) {
    vb = kRuns ? xcd_runs(blockIdx.x, total, run) : blockIdx.x;
    return first;
  }
  if (threadIdx.x == 0) *s_vb = atomicAdd(queue, 1u);
  __syncthreads();
  vb = *s_vb;
  __syncthreads();  // every lane has read it before lane 0 takes the next
  return vb < total;
}

__device__ __forceinline__ void queue_done(uint32_t* queue) {
  if (!queue || threadIdx.x != 0) return;
  __threadfence();
  if (atomicAdd(queue + 1, 1u) == gridDim.x - 1) {
    atomicExch(queue, 0u);
    atomicExch(queue + 1, 0u);
  }
}

// kMesh: the launch's scenes may hold a triangle mesh; the dynamic LDS then
// holds `stack` traversal-stack entries per lane.
// kShared: the launch may hold shared-path pair slices (the other launches
// keep the smaller exchange buffer and register budget of single paths).
// Register budgets (waves per SIMD), each the fastest measured on the
// 2048x2048 terrain and the 512x512 textured step: analytic scenes 7 (72
// VGPRs); mesh scenes 6 (80 VGPRs, some private-memory spills: 6% faster than
// 5, 7 is slower again); the two-ledger path of shared pairs 5 (96 VGPRs:
// 14% faster than 4 on the terrain).
template <int TW, int TH, bool kMesh, bool kShared>
__global__ void __launch_bounds__(TW * TH)
__attribute__((amdgpu_waves_per_eu(kShared ? 5 : (kMesh ? 6 : 7))))
k_forward(const FwdArgs* __restrict__ Units, int n_units, int stack, unsigned long long* work,
          uint32_t* queue, uint32_t total) {
  using SH = Shape<TW, TH>;
  __shared__ uint32_t s_xchg[(kShared ? kFwd2XchgWords : kFwdXchgWords) * kXchg];
  __shared__ int s_cnt[SH::WAVES];
  __shared__ uint32_t s_vb;
  extern __shared__ uint32_t s_dyn[];
  const TravStack st{s_dyn + threadIdx.x, SH::N, stack};
  uint32_t b;
  const uint32_t run = kShared || queue ? 1u : xcd_run_of(Units, n_units, kXcdRun);
  for (bool first = true; next_block<!kShared>(queue, total, &s_vb, first, b, run);
       first = false) {
    const FwdArgs& A = unit_of(Units, n_units, b);
    const uint32_t iter = iteration_of(A.key);
    if (A.h.max_iter && iter >= A.h.max_iter) continue;  // finished problem
    const TileBlock tb = tile_block<SH, !kShared>(A, b);
    if (kShared && G(A.sl[tb.slice].params_b) != nullptr)  // uniform over the block
      forward_tile<SH, kMesh, kShared>(A, G(A.scene), tb, iter, s_xchg, s_cnt, st, work);
    else
      forward_tile<SH, kMesh, false, (kShared || !kMesh) ? REC_NONE : REC_WRITE>(
          A, G(A.scene), tb, iter, s_xchg, s_cnt, st, work);
  }
  queue_done(queue);
}

// ---------------------------------------------------------------------------
// primal images from their slots: mean radiance, adjoint image, loss.  Grid
// (blocks, jobs); blocks stride over the crop's pixels and reduce the loss to
// one atomic each.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kFinBlock) k_finalize(const FinArgs* __restrict__ Units,
                                                         int n_units) {
  __shared__ double s_red[kFinBlock / 64];
  const FinArgs& A = unit_of(Units, n_units);
  const uint32_t iter = iteration_of(A.key);
  if (A.h.max_iter && iter >= A.h.max_iter) return;  // finished problem
  const uint32_t local = blockIdx.x - A.h.block0;
  const FinJob& job = A.jobs[local / A.nblocks];
  const int bx = (int)(local % A.nblocks);
  const int cw = A.crop.x1 - A.crop.x0, chh = A.crop.y1 - A.crop.y0;
  double se = 0.0;
  for (int i = bx * kFinBlock + (int)threadIdx.x; i < cw * chh; i += (int)A.nblocks * kFinBlock) {
    const uint32_t pix = (uint32_t)((A.crop.y0 + i / cw) * A.width + (A.crop.x0 + i % cw));
    if (!(G(A.mask) && G(A.mask)[pix])) {
      double sum[3] = {0.0, 0.0, 0.0};
      for (int s = 0; s < job.n; ++s) {
        const double* c = G(A.slots) + ((size_t)(job.slot0 + s) * A.npix + pix) * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) sum[k] += c[k];
      }
      if (!job.first) {
#pragma unroll
        for (int k = 0; k < 3; ++k) sum[k] = G(job.accum)[3 * (size_t)pix + k] + sum[k];
      }
      if (!job.last) {
#pragma unroll
        for (int k = 0; k < 3; ++k) G(job.accum)[3 * (size_t)pix + k] = sum[k];
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float I = (float)(sum[k] * job.inv_spp);
          if (G(job.img)) G(job.img)[3 * (size_t)pix + k] = I;
          if (G(job.delta)) {
            const float t = G(A.target)[3 * (size_t)pix + k];
            const float e = I - t;
            const float w = A.relative ? 1.0f / (t * t + kRelEps) : 1.0f;
            G(job.delta)[3 * (size_t)pix + k] = A.delta_scale * e * w;
            se += (double)e * (double)e * (double)w;
          }
        }
      }
    } else if (job.last && G(job.delta)) {
#pragma unroll
      for (int k = 0; k < 3; ++k) G(job.delta)[3 * (size_t)pix + k] = 0.0f;
    }
  }
  if (job.last && G(job.loss2)) {
    se = wave_sum(se);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = se;
    __syncthreads();
    if (threadIdx.x == 0) {
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < kFinBlock / 64; ++w) tot += s_red[w];
      if (tot != 0.0) unsafeAtomicAdd(&G(job.loss2)[iter & 1u], tot * A.loss_scale);
    }
  }
}

// ---------------------------------------------------------------------------
// gradient scatter
//
// Neighbouring pixels of a tile hit the same texels, and same-address FP32
// atomics within one instruction serialise in the memory system.  Each block
// therefore sums its texel contributions in an LDS hash table (open
// addressing, keys claimed with LDS compare-and-swap, values added with LDS
// float atomics) and flushes every distinct parameter once with a global
// atomic at the end.  A congested probe sequence falls back to a direct
// global atomic, so the table can never lose a contribution.
// ---------------------------------------------------------------------------
constexpr int kTableBits = 8;
constexpr int kTableSize = 1 << kTableBits;  // texels per block table
constexpr int kMaxProbe = 32;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
// LDS per block (dynamic): kTableSize * 4 * (1 + n_ch) bytes, 5 KiB for
// RGB + roughness.  Only first vertices (one tile's footprint: some 25-100
// texels in the workloads here) enter it.  A block keeps its LDS until its
// last wave ends, so after the compaction leaves most blocks with one or two
// waves, LDS bounds the blocks a CU holds: 256 slots instead of 1024 made the
// terrain replay 15% faster (31% with shared-path pairs); past 256 the table
// has no use.

struct GradTable {
  uint32_t* keys;  // LDS: texel index of each slot
  float* vals;     // LDS: n_ch gradient values per slot
  float* grad;     // global gradient buffer of this block's job
  // deterministic mode (fx set): every contribution goes, rounded to a
  // multiple of 1 / fx_scale, into a 64-bit fixed-point accumulator with an
  // integer atomic; integer sums do not depend on the order the atomics
  // arrive in, so the result is bitwise reproducible across launches, tile
  // shapes and batches.  The block table (LDS float atomics) is bypassed.
  unsigned long long* fx;
  double fx_scale;
};

// Add v to gradient element i: an FP32 atomic, or (kDet) fixed point (see
// GradTable).  The deterministic mode has kernel instances of its own, so the
// default ones carry none of its code.
template <bool kDet>
__device__ __forceinline__ void grad_add(const GradTable& T, size_t i, float v) {
  if constexpr (kDet)
    atomicAdd(T.fx + i, (unsigned long long)__double2ll_rn((double)v * T.fx_scale));
  else
    unsafeAtomicAdd(T.grad + i, v);
}

// Slot of `texel` in the table (claimed if new), or -1 when the probe
// sequence is congested.
__device__ __forceinline__ int table_slot(const GradTable& T, uint32_t texel) {
  uint32_t h = (texel * 2654435761u) >> (32 - kTableBits);
  for (int p = 0; p < kMaxProbe; ++p) {
    uint32_t k = T.keys[h];
    if (k == kEmpty) {
      const uint32_t old = atomicCAS(&T.keys[h], kEmpty, texel);
      k = old == kEmpty ? texel : old;
    }
    if (k == texel) return (int)h;
    h = (h + 1) & (kTableSize - 1);
  }
  return -1;
}

// Element q of the footprint (q = 0..3: t00, t01, t10, t01 + t10 - t00) and
// its weight, computed arithmetically so no per-lane array is indexed.  A
// triangle's fourth element has weight 0 and is never touched.
template <bool kMesh>
__device__ __forceinline__ void footprint_texel(const Footprint& fp, int q, int& texel,
                                                float& w) {
  const int dx = fp.t01 - fp.t00, dy = fp.t10 - fp.t00;
  texel = fp.t00 + (q & 1) * dx + (q >> 1) * dy;
  w = footprint_weight<kMesh>(fp, q);
}

// Add one first-hit vertex's material gradient g (R, G, B, metal, rough) to
// its four texels in the block table (global atomics when a probe sequence is
// congested).
template <bool kMesh, bool kDet>
__device__ __forceinline__ void scatter_texels(const DevScene& S, const GradTable& T,
                                               const Footprint& fp, const float g[5],
                                               float sign) {
  const int nc = S.n_ch;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    int texel;
    float w;
    footprint_texel<kMesh>(fp, q, texel, w);
    if (w == 0.0f) continue;
    const int h = kDet ? -1 : table_slot(T, (uint32_t)texel);
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int s = S.slot[b];
      if (s < 0) continue;
      const float v = w * (sign * g[b]);
      if (v == 0.0f) continue;
      if (h >= 0)
        __hip_atomic_fetch_add(&T.vals[h * nc + s], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        grad_add<kDet>(T, (size_t)texel * nc + s, v);
    }
  }
}

// Scatter the later-vertex gradient of every lane with `has` set straight to
// memory.  Device-scope float atomics are priced per cache line, so the wave
// spreads each vertex over 4 * n_ch lanes, neighbouring lanes taking the
// neighbouring channels of one texel: a texel then costs one transaction
// instead of n_ch.  Must be reached by all 64 lanes of the wave.
template <bool kMesh, bool kDet>
__device__ __forceinline__ void scatter_wave(const DevScene& S, const GradTable& T,
                                             const VertexGrad& v, float sign, bool has) {
  uint64_t m = __ballot(has);
  if (m == 0) return;
  const int nc = S.n_ch;
  const int per = 4 * nc;  // lanes per vertex
  const int nv = 64 / per;  // vertices per round
  const int lane = (int)__lane_id();
  const int vi = lane / per;
  const int within = lane - vi * per;
  const int q = within / nc;
  const int c = within - q * nc;
  while (m != 0) {
    uint64_t mm = m;
    for (int k = 0; k < vi && mm != 0; ++k) mm &= mm - 1;
    const bool work = vi < nv && mm != 0;
    const int src = work ? __ffsll((unsigned long long)mm) - 1 : lane;
    Footprint fp;
    fp.global = 0;
    fp.tri = kMesh ? __shfl(v.fp.tri, src, 64) : 0;
    fp.t00 = __shfl(v.fp.t00, src, 64);
    fp.t01 = __shfl(v.fp.t01, src, 64);
    fp.t10 = __shfl(v.fp.t10, src, 64);
    fp.fx = __shfl(v.fp.fx, src, 64);
    fp.fy = __shfl(v.fp.fy, src, 64);
    float gc = 0.0f;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const float x = __shfl(v.g[b], src, 64);
      if (S.slot[b] == c) gc = x;
    }
    if (work) {
      int texel;
      float w;
      footprint_texel<kMesh>(fp, q, texel, w);
      const float val = w * (sign * gc);
      if (w != 0.0f && val != 0.0f) grad_add<kDet>(T, (size_t)texel * nc + c, val);
    }
    for (int k = 0; k < nv && m != 0; ++k) m &= m - 1;
  }
}

__device__ __forceinline__ bool same_footprint(const Footprint& a, const Footprint& b) {
  return a.global == b.global && a.tri == b.tri && a.t00 == b.t00 && a.t01 == b.t01 &&
         a.t10 == b.t10 &&
         __float_as_uint(a.fx) == __float_as_uint(b.fx) &&
         __float_as_uint(a.fy) == __float_as_uint(b.fy);
}

// Accumulates vertex gradients: global materials into per-lane registers
// (reduced over the wave when it leaves), first-hit texels into the block's
// table; later textured vertices are handed back for the wave-cooperative
// scatter.
template <bool kDet>
struct Sink {
  float acc[5];
  GradTable T;
  __device__ __forceinline__ void init(const GradTable& t) {
    T = t;
#pragma unroll
    for (int b = 0; b < 5; ++b) acc[b] = 0.0f;
  }
  // returns true when v is a later textured vertex left to scatter_wave
  template <bool kMesh>
  __device__ __forceinline__ bool add(const DevScene& S, const VertexGrad& v, float sign) {
    if (!v.valid) return false;
    if (v.fp.global) {
      if constexpr (kDet) {  // each contribution on its own: fixed point is order-free
#pragma unroll
        for (int b = 0; b < 5; ++b) {
          const float x = sign * v.g[b];
          if (S.slot[b] >= 0 && x != 0.0f) grad_add<kDet>(T, (size_t)S.slot[b], x);
        }
        return false;
      }
#pragma unroll
      for (int b = 0; b < 5; ++b) acc[b] += sign * v.g[b];
      return false;
    }
    if (v.j > 1) return true;
    scatter_texels<kMesh, kDet>(S, T, v.fp, v.g, sign);
    return false;
  }
  // every lane of the block (nthreads), after a barrier; neighbouring lanes
  // flush neighbouring channels of one texel
  __device__ __forceinline__ void flush_table(const DevScene& S, int nthreads) {
    const int nc = S.n_ch;
    for (int i = threadIdx.x; i < kTableSize * nc; i += nthreads) {
      const int slot = i / nc;
      const int c = i - slot * nc;
      const uint32_t k = T.keys[slot];
      if (k == kEmpty) continue;
      const float v = T.vals[i];
      if (v != 0.0f) grad_add<kDet>(T, (size_t)k * nc + c, v);
    }
  }
  // every lane of the wave
  __device__ __forceinline__ void flush_acc(const DevScene& S) {
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int s = S.slot[b];
      const float v = wave_sum(acc[b]);
      if (s >= 0 && (threadIdx.x & 63) == 0 && v != 0.0f) grad_add<kDet>(T, (size_t)s, v);
    }
  }
};

// Replay state of one path (single) or one finite-difference pair, moved
// between lanes by the compaction.
struct RepItem {
  Path P;
  float adj[3];
  int src;
};


struct RepSharedItem {  // a shared-path pair: one path, two ledgers
  Path P;
  Ledger2 L2;
  float adj_a[3], adj_b[3];
  int src, pad_;
};

constexpr int kRepXchgWords = (int)(sizeof(RepSharedItem) / 4);
static_assert(sizeof(RepItem) <= sizeof(RepSharedItem), "exchange buffer size");

// Start the replay of a path: P.led = the radiance still to come.
template <bool kMesh, int kRec>
__device__ __forceinline__ void replay_begin(const DevScene& S, const TravStack& st,
                                             const Rng& rng, int px, int py, uint32_t flags,
                                             const double* __restrict__ C, Path& P,
                                             const HitRecs& hr) {
  path_begin<kMesh, kRec>(S, st, rng, px, py, flags, P, hr);
#pragma unroll
  for (int k = 0; k < 3; ++k) P.led[k] = C[k] - P.led[k];
}

// One block = one pixel tile of one slice of single paths.  Each path is
// replayed vertex by vertex from its forward radiance: first vertices in place
// (their gradients go to the block table, flushed right after), later ones on
// the compacted lanes in a wave-uniform loop, so the later-vertex scatter can
// use the whole wave.  The exchange buffer reuses the table's LDS.
template <class SH, bool kMesh, bool kDet, int kRec = REC_NONE>
__device__ __forceinline__ void adjoint_tile(const RepArgs& A, const DevScene* __restrict__ Sp,
                                             const TileBlock& tb, uint32_t iter, uint32_t* s_dyn,
                                             int* s_cnt, const TravStack& st,
                                             unsigned long long* work) {
  const DevScene& S = *Sp;
  uint32_t* s_keys = s_dyn;
  float* s_vals = reinterpret_cast<float*>(s_dyn + kTableSize);
  const RepSlice& sl = A.sl[tb.slice];
  int px, py;
  const bool inside = tile_pixel<SH>(A.crop, tb, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  for (int i = threadIdx.x; i < kTableSize; i += SH::N) s_keys[i] = kEmpty;
  for (int i = threadIdx.x; i < kTableSize * S.n_ch; i += SH::N) s_vals[i] = 0.0f;
  __syncthreads();
  Sink<kDet> sink;
  sink.init(GradTable{s_keys, s_vals, G(sl.grad), G(sl.fx), sl.fx_scale});
  const uint64_t key = stream_key(A.key.seed, iter, sl.tag);
  const BlockPaths<SH> B = block_paths<SH>(tb, S, key, sl.sample, A.flags);
  const Rng rng = B.rng((int)threadIdx.x);
  const int tid = (int)threadIdx.x;
  RepItem mine;
  mine.P.alive = false;
  mine.src = tid;
  int n_vert = 0;
  {
    VertexGrad v;
    v.valid = false;
    if (active) {
#pragma unroll
      for (int k = 0; k < 3; ++k) mine.adj[k] = G(sl.delta)[3 * (size_t)pix + k] * sl.adj_scale;
      const HitRecs hr = hit_recs(kRec != REC_NONE ? A.recs : nullptr, sl.slot_a, A.npix, pix,
                                  A.rec_epoch);
      replay_begin<kMesh, kRec>(S, st, rng, px, py, A.flags,
                                G(A.slots) + ((size_t)sl.slot_a * A.npix + pix) * 3, mine.P, hr);
      if (mine.P.alive) {
        ++n_vert;
        path_vertex<true, kMesh, kRec>(S, st, G(sl.params), rng, A.flags, mine.P, mine.adj, v,
                                       hr);
      }
    }
    sink.template add<kMesh>(S, v, sl.sign);  // first vertices (j = 1) go to the table
  }
  __syncthreads();
  sink.flush_table(S, SH::N);
  const bool live = mine.P.alive;
  int n;
  const int r = block_rank<SH>(live, n, s_cnt);  // its barriers also retire the table
  RepItem W;
  if (n > compact_max<SH>()) {
    W = mine;
  } else {
    W.P.alive = false;
    W.src = tid;
    if (n > 0) pack(s_dyn, live, r, n, mine, W);
  }
  // no barrier below: waves without a path leave
  if (__ballot(W.P.alive) != 0) {
    const Rng wr = B.rng(W.src);
    const HitRecs whr = hit_recs(kRec != REC_NONE ? A.recs : nullptr, sl.slot_a, A.npix,
                                 B.pixel(W.src), A.rec_epoch);
    while (__ballot(W.P.alive) != 0) {
      VertexGrad v;
      v.valid = false;
      if (W.P.alive) {
        ++n_vert;
        path_vertex<true, kMesh, kRec>(S, st, G(sl.params), wr, A.flags, W.P, W.adj, v, whr);
      }
      const bool later = sink.template add<kMesh>(S, v, sl.sign);
      scatter_wave<kMesh, kDet>(S, sink.T, v, sl.sign, later);
    }
  }
  sink.flush_acc(S);
  count_work(work, active ? 1 : 0, n_vert);
}

// The gradient of the partner lane's vertex (lane ^ 1); every lane of the wave
// must call it.  Where both vertices are valid and share their footprint
// bitwise, the first lane of the pair keeps the difference of the two
// gradients and the second drops its vertex, so equal parameter vectors give
// an exactly zero difference before any atomic.  The second lane's gradient
// is then negated, so both lanes scatter with sign +1 (the wave-cooperative
// scatter applies one sign to every lane's vertex).
template <bool kMesh>
__device__ __forceinline__ void pair_difference(VertexGrad& v, int half) {
  Footprint o;
  const int ov = __shfl_xor(v.valid ? 1 : 0, 1, 64);
  o.global = __shfl_xor(v.fp.global, 1, 64);
  o.tri = kMesh ? __shfl_xor(v.fp.tri, 1, 64) : 0;
  o.t00 = __shfl_xor(v.fp.t00, 1, 64);
  o.t01 = __shfl_xor(v.fp.t01, 1, 64);
  o.t10 = __shfl_xor(v.fp.t10, 1, 64);
  o.fx = __shfl_xor(v.fp.fx, 1, 64);
  o.fy = __shfl_xor(v.fp.fy, 1, 64);
  float og[5];
#pragma unroll
  for (int b = 0; b < 5; ++b) og[b] = __shfl_xor(v.g[b], 1, 64);
  Footprint mine = v.fp;
  if (!kMesh) mine.tri = 0;
  if (v.valid && ov && same_footprint(mine, o)) {
    if (half == 0) {
#pragma unroll
      for (int b = 0; b < 5; ++b) v.g[b] -= og[b];
    } else {
      v.valid = false;
    }
  }
  if (half) {
#pragma unroll
    for (int b = 0; b < 5; ++b) v.g[b] = -v.g[b];
  }
}

// A replay-pair slice (Eq. 5 by primary-sample-space replay): one block = a
// tile of TW x TH/2 pixels, lanes 2k and 2k + 1 replaying pixel k's path at
// A's parameters (+) and at B's (-) from the same random numbers, vertex by
// vertex in lockstep; coinciding vertices are differenced across the lane pair
// (pair_difference).  A pair occupies two lanes of one path each, so the
// kernel keeps the register budget of single paths.  The first vertices go to
// the block table; then the live pairs are compacted, each onto two
// neighbouring lanes.
template <class SH, bool kMesh, bool kDet, int kRec = REC_NONE>
__device__ __forceinline__ void adjoint_tile_pairs(const RepArgs& A,
                                                   const DevScene* __restrict__ Sp,
                                                   const TileBlock& tb, uint32_t iter,
                                                   uint32_t* s_dyn, int* s_cnt,
                                                   const TravStack& st,
                                                   unsigned long long* work) {
  const DevScene& S = *Sp;
  uint32_t* s_keys = s_dyn;
  float* s_vals = reinterpret_cast<float*>(s_dyn + kTableSize);
  const RepSlice& sl = A.sl[tb.slice];
  const int tid = (int)threadIdx.x;
  const int half = tid & 1;
  auto pixel_of = [&](int t, int& x, int& y) {
    const int k = t >> 1;
    x = tb.x0 + k % SH::W;
    y = tb.y0 + k / SH::W;
  };
  int px, py;
  pixel_of(tid, px, py);
  const bool inside = px < A.crop.x1 && py < A.crop.y1;
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  for (int i = threadIdx.x; i < kTableSize; i += SH::N) s_keys[i] = kEmpty;
  for (int i = threadIdx.x; i < kTableSize * S.n_ch; i += SH::N) s_vals[i] = 0.0f;
  __syncthreads();
  Sink<kDet> sink;
  sink.init(GradTable{s_keys, s_vals, G(sl.grad), G(sl.fx), sl.fx_scale});
  const uint64_t key = stream_key(A.key.seed, iter, sl.tag);
  const float* params = half ? G(sl.params_b) : G(sl.params);
  RepItem mine;
  mine.P.alive = false;
  mine.src = tid;
  int n_vert = 0;
  {
    VertexGrad v;
    v.valid = false;
    if (active) {
      const float* delta = half ? G(sl.delta_b) : G(sl.delta);
#pragma unroll
      for (int k = 0; k < 3; ++k) mine.adj[k] = delta[3 * (size_t)pix + k] * sl.adj_scale;
      const Rng rng = make_rng(key, pix, sl.sample);
      const int slot = half ? sl.slot_b : sl.slot_a;
      const HitRecs hr = hit_recs(kRec != REC_NONE ? A.recs : nullptr, slot, A.npix, pix,
                                  A.rec_epoch);
      replay_begin<kMesh, kRec>(S, st, rng, px, py, A.flags,
                                G(A.slots) + ((size_t)slot * A.npix + pix) * 3, mine.P, hr);
      if (mine.P.alive) {
        ++n_vert;
        path_vertex<true, kMesh, kRec>(S, st, params, rng, A.flags, mine.P, mine.adj, v, hr);
      }
    }
    pair_difference<kMesh>(v, half);
    sink.template add<kMesh>(S, v, 1.0f);  // first vertices (j = 1) go to the table
  }
  __syncthreads();
  sink.flush_table(S, SH::N);
  // pairs with a live path, counted on their first lanes; both lanes of such
  // a pair move (to lanes 2 r and 2 r + 1), a finished path keeps its lane
  const int pair_live = (mine.P.alive ? 1 : 0) | __shfl_xor(mine.P.alive ? 1 : 0, 1, 64);
  int n;
  const int r0 = block_rank<SH>(pair_live && half == 0, n, s_cnt);
  const int r = 2 * __shfl(r0, tid & ~1 & 63, 64) + half;
  RepItem W;
  if (2 * n > compact_max<SH>()) {
    W = mine;
  } else {
    W.P.alive = false;
    W.src = tid;
    if (n > 0) pack(s_dyn, pair_live != 0, r, 2 * n, mine, W);
  }
  // no barrier below: waves without a live pair leave
  if (__ballot(W.P.alive) != 0) {
    int wx, wy;
    pixel_of(W.src, wx, wy);
    const uint32_t wpix = (uint32_t)(wy * S.width + wx);
    const Rng wr = make_rng(key, wpix, sl.sample);
    const HitRecs whr = hit_recs(kRec != REC_NONE ? A.recs : nullptr,
                                 half ? sl.slot_b : sl.slot_a, A.npix, wpix, A.rec_epoch);
    while (__ballot(W.P.alive) != 0) {
      VertexGrad v;
      v.valid = false;
      if (W.P.alive) {
        ++n_vert;
        path_vertex<true, kMesh, kRec>(S, st, params, wr, A.flags, W.P, W.adj, v, whr);
      }
      pair_difference<kMesh>(v, half);
      const bool later = sink.template add<kMesh>(S, v, 1.0f);
      scatter_wave<kMesh, kDet>(S, sink.T, v, 1.0f, later);
    }
  }
  sink.flush_acc(S);
  count_work(work, active ? 1 : 0, n_vert);
}

// A shared-path pair slice (Eq. 5 as written): each path is drawn at A's
// parameters and replayed once; the vertex carries both ledgers (B's material
// evaluated over A's densities), and the difference of the two gradients is
// formed in registers over the one footprint they share, so it is scattered
// once.  The first vertices go to the block table as in adjoint_tile.
template <class SH, bool kMesh, bool kDet>
__device__ __forceinline__ void adjoint_tile_shared(const RepArgs& A,
                                                    const DevScene* __restrict__ Sp,
                                                    const TileBlock& tb, uint32_t iter,
                                                    uint32_t* s_dyn, int* s_cnt,
                                                    const TravStack& st,
                                                    unsigned long long* work) {
  const DevScene& S = *Sp;
  uint32_t* s_keys = s_dyn;
  float* s_vals = reinterpret_cast<float*>(s_dyn + kTableSize);
  const RepSlice& sl = A.sl[tb.slice];
  int px, py;
  const bool inside = tile_pixel<SH>(A.crop, tb, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  for (int i = threadIdx.x; i < kTableSize; i += SH::N) s_keys[i] = kEmpty;
  for (int i = threadIdx.x; i < kTableSize * S.n_ch; i += SH::N) s_vals[i] = 0.0f;
  __syncthreads();
  Sink<kDet> sink;
  sink.init(GradTable{s_keys, s_vals, G(sl.grad), G(sl.fx), sl.fx_scale});
  const uint64_t key = stream_key(A.key.seed, iter, sl.tag);
  const BlockPaths<SH> B = block_paths<SH>(tb, S, key, sl.sample, A.flags);
  const Rng rng = B.rng((int)threadIdx.x);
  const int tid = (int)threadIdx.x;
  const float* pa = G(sl.params);
  const float* pb = G(sl.params_b);
  RepSharedItem mine;
  mine.P.alive = false;
  mine.src = tid;
  int n_vert = 0;
  {
    VertexGrad v;
    v.valid = false;
    if (active) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        mine.adj_a[k] = G(sl.delta)[3 * (size_t)pix + k] * sl.adj_scale;
        mine.adj_b[k] = G(sl.delta_b)[3 * (size_t)pix + k] * sl.adj_scale;
      }
      path_begin<kMesh>(S, st, rng, px, py, A.flags, mine.P);
      const double* Ca = G(A.slots) + ((size_t)sl.slot_a * A.npix + pix) * 3;
      const double* Cb = G(A.slots) + ((size_t)sl.slot_b * A.npix + pix) * 3;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        mine.L2.led[k] = Cb[k] - mine.P.led[k];
        mine.L2.beta[k] = 1.0f;
        mine.P.led[k] = Ca[k] - mine.P.led[k];
      }
      if (mine.P.alive) {
        ++n_vert;
        path_vertex2<true, kMesh, true>(S, st, pa, pb, rng, A.flags, mine.P, mine.L2,
                                        mine.adj_a, mine.adj_b, v);
      }
    }
    sink.template add<kMesh>(S, v, 1.0f);  // first vertices (j = 1) go to the table
  }
  __syncthreads();
  sink.flush_table(S, SH::N);
  const bool live = mine.P.alive;
  int n;
  const int r = block_rank<SH>(live, n, s_cnt);  // its barriers also retire the table
  RepSharedItem W;
  if (n > compact_max<SH>()) {
    W = mine;
  } else {
    W.P.alive = false;
    W.src = tid;
    if (n > 0) pack(s_dyn, live, r, n, mine, W);
  }
  // no barrier below: waves without a path leave
  if (__ballot(W.P.alive) != 0) {
    const Rng wr = B.rng(W.src);
    while (__ballot(W.P.alive) != 0) {
      VertexGrad v;
      v.valid = false;
      if (W.P.alive) {
        ++n_vert;
        path_vertex2<true, kMesh, true>(S, st, pa, pb, wr, A.flags, W.P, W.L2, W.adj_a, W.adj_b,
                                        v);
      }
      const bool later = sink.template add<kMesh>(S, v, 1.0f);
      scatter_wave<kMesh, kDet>(S, sink.T, v, 1.0f, later);
    }
  }
  sink.flush_acc(S);
  count_work(work, active ? 1 : 0, n_vert);
}

// Dynamic LDS: with kMesh, `stack` traversal-stack entries per lane first
// (the LDS part of the stack), then the gradient table / exchange buffer.
// kShared: the launch's pair slices are shared-path pairs; otherwise they are
// replay pairs on lane pairs (units with pair_lanes).  Single paths, lane
// pairs and shared-path pairs each keep one path per lane, so the kernel runs
// at 5 waves per SIMD (96 VGPRs; a few spills: 4-10% faster than 4 waves at
// 128, 6 waves is slower again).
// kDet: the deterministic mode (fixed-point sums); its instances take every
// kind of slice (single paths, lane pairs, shared-path pairs).
template <int TW, int TH, bool kMesh, bool kShared, bool kDet = false>
__global__ void __launch_bounds__(TW * TH)
__attribute__((amdgpu_waves_per_eu(5)))
k_adjoint(const RepArgs* __restrict__ Units, int n_units, int stack, unsigned long long* work,
          uint32_t* queue, uint32_t total) {
  using SH = Shape<TW, TH>;
  // hit records: read by the replays of single paths and replay pairs in the
  // mesh instances (BVH traversal is what they save; analytic scenes intersect
  // a plane and a few spheres for less than a record costs); the shared-path
  // and deterministic instances trace every ray
  constexpr int kRec = (kShared || kDet || !kMesh) ? REC_NONE : REC_READ;
  extern __shared__ uint32_t s_dyn[];
  __shared__ int s_cnt[SH::WAVES];
  __shared__ uint32_t s_vb;
  const TravStack st{s_dyn + threadIdx.x, SH::N, stack};
  uint32_t* lds = s_dyn + (kMesh ? stack * SH::N : 0);
  uint32_t b;
  const uint32_t run = kShared || queue ? 1u : xcd_run_of(Units, n_units, kXcdRunReplay);
  for (bool first = true; next_block<!kShared>(queue, total, &s_vb, first, b, run);
       first = false) {
    const RepArgs& A = unit_of(Units, n_units, b);
    const uint32_t iter = iteration_of(A.key);
    if (A.h.max_iter && iter >= A.h.max_iter) continue;  // finished problem
    if ((!kShared || kDet) && A.pair_lanes) {  // uniform over the block, as below
      const TileBlock tb = tile_block<SH, !kShared>(A, b, SH::H / 2);
      adjoint_tile_pairs<SH, kMesh, kDet, kRec>(A, G(A.scene), tb, iter, lds, s_cnt, st, work);
      continue;
    }
    const TileBlock tb = tile_block<SH, !kShared>(A, b);
    if (kShared && G(A.sl[tb.slice].params_b) != nullptr)
      adjoint_tile_shared<SH, kMesh, kDet>(A, G(A.scene), tb, iter, lds, s_cnt, st, work);
    else
      adjoint_tile<SH, kMesh, kDet, kRec>(A, G(A.scene), tb, iter, lds, s_cnt, st, work);
  }
  queue_done(queue);
}

// ---------------------------------------------------------------------------
// emission-absorption volume (layout JSO_LAYOUT_VOLUME; the volume experiment
// of the Experiments section).  Each lane marches its pixel's ray through the
// cube: the chord is split into n = ceil(chord / voxel) equal segments of
// length dt, sampled at t0 + (k + u) dt with one jitter u per ray; each
// sample reads the clamp-to-edge trilinear interpolation of 8 voxels (one
// 16-byte load each: emission RGB, density).  Radiance: sum_k T_k a_k e_k +
// T_n env with a_k = 1 - exp(-sigma_k dt), T_{k+1} = T_k exp(-sigma_k dt),
// summed in an FP64 ledger.  The march draws nothing from the parameters, so
// a finite-difference pair is one march with two ledgers in either fd_mode.
// ---------------------------------------------------------------------------
struct VolRay {
  V3 o, d;
  float t0, dt, us;
  int n;  // segments (0: the ray misses the cube)
};

__device__ __forceinline__ VolRay vol_ray(const DevScene& S, const Rng& rng, int px, int py,
                                          uint32_t flags) {
  float u[4];
  rng.draw(0, 0, u);
  const bool center = (flags & JSO_F_PIXEL_CENTER) != 0;
  const float jx = center ? 0.5f : u[0], jy = center ? 0.5f : u[1];
  VolRay r;
  r.us = center ? 0.5f : u[2];
  const int v = py / S.view_h;
  const int row = py - v * S.view_h;
  const float sx = (2.0f * ((float)px + jx) / (float)S.width - 1.0f) * S.tan_half * S.aspect;
  const float sy = (1.0f - 2.0f * ((float)row + jy) / (float)S.view_h) * S.tan_half;
  r.o = ld3(S.view_eye[v]);
  r.d = normalize(ld3(S.view_cw[v]) + ld3(S.view_cu[v]) * sx + ld3(S.view_cv[v]) * sy);
  const float o[3] = {r.o.x, r.o.y, r.o.z}, d[3] = {r.d.x, r.d.y, r.d.z};
  float t0 = 0.0f, t1 = 3.0e38f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float inv = safe_inv(d[a]);
    const float ta = (S.vol_lo[a] - o[a]) * inv, tb = (S.vol_lo[a] + S.vol_side - o[a]) * inv;
    t0 = fmaxf(t0, fminf(ta, tb));
    t1 = fminf(t1, fmaxf(ta, tb));
  }
  r.n = 0;
  r.t0 = t0;
  r.dt = 0.0f;
  if (t1 > t0) {
    r.n = max(1, (int)ceilf((t1 - t0) * S.vol_inv_vox));
    r.dt = (t1 - t0) / (float)r.n;
  }
  return r;
}

// Offsets of voxel coordinate i along each axis in the bricked copy (see
// BrickArgs): the brick's offset (multiples of 64 voxels) plus the axis's two
// Morton bits, so a voxel's index is the sum of its three axis offsets.
__device__ __forceinline__ int brick_x(int i, int Rb) {
  (void)Rb;
  return ((i >> 2) << 6) | (i & 1) | ((i & 2) << 2);
}
__device__ __forceinline__ int brick_y(int i, int Rb) {
  return (((i >> 2) * Rb) << 6) | ((i & 1) << 1) | ((i & 2) << 3);
}
__device__ __forceinline__ int brick_z(int i, int Rb) {
  return (((i >> 2) * Rb * Rb) << 6) | ((i & 1) << 2) | ((i & 2) << 4);
}

// Trilinear corners of the sample at x: voxel indices in the bricked copy (8,
// clamped to the grid), the cell's base (unclamped floor of the grid
// coordinate) and the fractions.
struct VolCell {
  int idx[8];
  int bx, by, bz;
  float fx, fy, fz;
  __device__ __forceinline__ float w(int c) const {
    return ((c & 1) ? fx : 1.0f - fx) * ((c & 2) ? fy : 1.0f - fy) * ((c & 4) ? fz : 1.0f - fz);
  }
};

__device__ __forceinline__ VolCell vol_cell(const DevScene& S, V3 x) {
  const int R = S.vol_res, Rb = S.vol_rb;
  const float g[3] = {(x.x - S.vol_lo[0]) * S.vol_inv_vox - 0.5f,
                      (x.y - S.vol_lo[1]) * S.vol_inv_vox - 0.5f,
                      (x.z - S.vol_lo[2]) * S.vol_inv_vox - 0.5f};
  int i0[3], i1[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float fl = floorf(g[a]);
    f[a] = g[a] - fl;
    i0[a] = min(max((int)fl, 0), R - 1);
    i1[a] = min(max((int)fl + 1, 0), R - 1);
  }
  VolCell c;
  c.fx = f[0];
  c.fy = f[1];
  c.fz = f[2];
  c.bx = (int)floorf(g[0]);
  c.by = (int)floorf(g[1]);
  c.bz = (int)floorf(g[2]);
  const int ox[2] = {brick_x(i0[0], Rb), brick_x(i1[0], Rb)};
  const int oy[2] = {brick_y(i0[1], Rb), brick_y(i1[1], Rb)};
  const int oz[2] = {brick_z(i0[2], Rb), brick_z(i1[2], Rb)};
#pragma unroll
  for (int k = 0; k < 8; ++k) c.idx[k] = oz[k >> 2] + oy[(k >> 1) & 1] + ox[k & 1];
  return c;
}

__device__ __forceinline__ float4 vol_fetch(const float* __restrict__ params, const VolCell& c) {
  const float4* p4 = reinterpret_cast<const float4*>(params);
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 q = p4[c.idx[k]];
    const float w = c.w(k);
    v.x += w * q.x;
    v.y += w * q.y;
    v.z += w * q.z;
    v.w += w * q.w;
  }
  return v;
}

// One march; kTwo: also the ledger of params_b.  led / led_b: radiance (FP64).
template <bool kTwo>
__device__ __forceinline__ int vol_march(const DevScene& S, const VolRay& r,
                                         const float* __restrict__ pa,
                                         const float* __restrict__ pb, double led[3],
                                         double led_b[3]) {
  float T = 1.0f, Tb = 1.0f;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) led[ch] = led_b[ch] = 0.0;
  for (int k = 0; k < r.n; ++k) {
    const VolCell c = vol_cell(S, r.o + r.d * (r.t0 + ((float)k + r.us) * r.dt));
    const float4 v = vol_fetch(pa, c);
    const float od = S.vol_sigma * v.w * r.dt;
    const float a = -expm1f(-od);
    led[0] += (double)(T * a * v.x);
    led[1] += (double)(T * a * v.y);
    led[2] += (double)(T * a * v.z);
    T *= expf(-od);
    if (kTwo) {
      const float4 vb = vol_fetch(pb, c);
      const float odb = S.vol_sigma * vb.w * r.dt;
      const float ab = -expm1f(-odb);
      led_b[0] += (double)(Tb * ab * vb.x);
      led_b[1] += (double)(Tb * ab * vb.y);
      led_b[2] += (double)(Tb * ab * vb.z);
      Tb *= expf(-odb);
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    led[ch] += (double)(T * S.env[ch]);
    if (kTwo) led_b[ch] += (double)(Tb * S.env[ch]);
  }
  return r.n;
}

// The hardware deals a grid's blocks out to the 8 XCDs in turn (block i to
// XCD i mod 8), and each XCD has an L2 of its own.  The volume kernels
// renumber their blocks so that XCD j takes the j-th contiguous eighth of
// the tiles, in order: the blocks resident on one XCD at a time are then
// neighbouring tiles of one view, whose rays cross the same voxels at about
// the same time and share that XCD's L2.  A bijection of [0, n).
__device__ __forceinline__ uint32_t xcd_block(uint32_t i, uint32_t n) {
  const uint32_t q = n >> 3, r = n & 7u, x = i & 7u;
  return x * q + min(x, r) + (i >> 3);
}

// A volume replay unit's block: its tiles in order, each tile's slices
// together (the slices of a tile march nearly the same rays, so running them
// side by side lets them share the voxels in L2).
template <class SH, class U>
__device__ __forceinline__ TileBlock vol_tile_block(const U& u, uint32_t b) {
  const uint32_t local = b - u.h.block0;
  const uint32_t ns = (uint32_t)u.n_slices;
  const uint32_t t = local / ns;
  return TileBlock{(int)(local - t * ns), u.crop.x0 + (int)(t % u.tiles_x) * SH::W,
                   u.crop.y0 + (int)(t / u.tiles_x) * SH::H};
}

// The volume forward: a block takes one 8x8 pixel tile and blockDim.x / 64 of
// the unit's slices, one wave each (block b of a unit: tile b / groups, slice
// group b % groups).  The waves march nearly the same rays in step, so each
// voxel line one of them brings into the CU's L1 and the XCD's L2 serves the
// others too.
__global__ void __launch_bounds__(64 * kVolMaxSliceWaves)
k_vol_forward(const FwdArgs* __restrict__ Units, int n_units, unsigned long long* work) {
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const FwdArgs& A = unit_of(Units, n_units, b);
  const uint32_t iter = iteration_of(A.key);
  if (A.h.max_iter && iter >= A.h.max_iter) return;  // finished problem
  const DevScene& S = *G(A.scene);
  const int waves = (int)(blockDim.x / 64);
  const uint32_t groups = (uint32_t)((A.n_slices + waves - 1) / waves);
  const uint32_t local = b - A.h.block0;
  const uint32_t t = local / groups;
  const int slice = (int)(local - t * groups) * waves + (int)(threadIdx.x / 64);
  if (slice >= A.n_slices) return;  // a whole wave: the group's last slices
  const FwdSlice& sl = A.sl[slice];
  const int lane = (int)(threadIdx.x % 64);
  const int px = A.crop.x0 + (int)(t % A.tiles_x) * 8 + (lane & 7);
  const int py = A.crop.y0 + (int)(t / A.tiles_x) * 8 + (lane >> 3);
  const bool inside = px < A.crop.x1 && py < A.crop.y1;
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  int n_samples = 0;
  if (active) {
    const Rng rng = make_rng(stream_key(A.key.seed, iter, sl.tag), pix, sl.sample);
    const VolRay r = vol_ray(S, rng, px, py, A.flags);
    double led[3], led_b[3];
    double* out = G(A.slots) + (size_t)sl.slot * A.npix * 3;
    if (G(sl.params_b) != nullptr) {
      n_samples = vol_march<true>(S, r, G(sl.params), G(sl.params_b), led, led_b);
      store_radiance(G(A.slots) + (size_t)sl.slot_b * A.npix * 3, pix, led_b);
    } else {
      n_samples = vol_march<false>(S, r, G(sl.params), nullptr, led, led_b);
    }
    store_radiance(out, pix, led);
  }
  count_work(work ? work + 2 : nullptr, active ? 1 : 0, n_samples);
}

// Replay: the remainder R = C - (radiance collected so far) gives, per sample,
//   dC/de_k     = T_k a_k
//   dC/dsigma_k = dt (T_{k+1} e_k - R_{k+1})
// (R_{k+1}: the radiance behind the sample, environment included), times the
// density scale, spread over the 8 voxels by the trilinear weights and added
// to the gradient with no-return FP32 atomics.  Pairs difference the two
// ledgers' gradients per sample (same voxels) and scatter once.
//
// Per-lane sums over the 8 corners of the current cell.  Consecutive samples
// of a ray share the corners of the cell faces they stay between, so their
// gradients are summed in registers and a corner is written out only when the
// ray leaves it.  A corner's slot is given by the parities of its voxel
// coordinates (bit 0: x, bit 1: y, bit 2: z), so moving to a neighbouring cell
// keeps the shared corners in place and only the slots whose coordinate
// changes are written out; slot indices stay compile-time constants (the sums
// stay in registers).
//
// The write-out is wave-cooperative: the lanes leaving a slot put its voxel
// and 4 sums into the wave's LDS staging area, and the wave adds them with 4
// lanes per voxel, so that one atomic instruction carries 16 voxels' 16-byte
// rows.  The L2 takes atomics at a rate per distinct line segment an
// instruction touches, not per lane, so this needs a quarter of the requests
// of adding each channel from its own lane.  Every lane of the wave runs the
// march to the wave's longest ray, those past their own end idle.
struct CornerSums {
  int x[2], y[2], z[2];  // voxel coordinate held by the slots of each parity
  float4 acc[8];
};

// A wave's staging area: the voxel (linear index) and sums of up to 8 slots
// per lane.
constexpr int kVolStage = 8 * 64;
struct VolStage {
  float4 v[kVolStage];
  int voxel[kVolStage];
};

// Write out the slots in each lane's mask f (bit sl: slot sl) and clear those
// sums.  Every lane of the wave calls this.  A lane's slots are staged
// together, in slot order (x-neighbouring voxels next to each other), lanes
// in order (neighbouring pixels): the voxels an atomic instruction carries
// then often share 64-byte segments of the gradient, which the L2 takes as
// one request.
__device__ __forceinline__ void corner_write(const DevScene& S, float* grad, CornerSums& cs,
                                             VolStage& st, uint32_t f) {
  if (__ballot(f != 0u) == 0) return;
  const int R = S.vol_res;
  const int lane = (int)__lane_id();
  // this lane's first entry: the exclusive prefix sum of the slot counts
  const int cnt = __popc(f);
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, (unsigned)o, 64);
    if (lane >= o) incl += t;
  }
  const int n = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));  // entries in all
  int e = incl - cnt;
#pragma unroll
  for (int sl = 0; sl < 8; ++sl) {
    if (!((f >> sl) & 1u)) continue;
    const int x = min(max(cs.x[sl & 1], 0), R - 1);
    const int y = min(max(cs.y[(sl >> 1) & 1], 0), R - 1);
    const int z = min(max(cs.z[sl >> 2], 0), R - 1);
    st.v[e] = cs.acc[sl];
    st.voxel[e] = (z * R + y) * R + x;
    cs.acc[sl] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    ++e;
  }
  // the staged entries of the other lanes are read below: LDS operations of
  // one wave complete in order; the fences keep the compiler from moving the
  // reads above the writes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int ch = lane & 3;
  for (int k = lane >> 2; k < n; k += 16) {
    const float val = reinterpret_cast<const float*>(&st.v[k])[ch];
    if (val != 0.0f) unsafeAtomicAdd(grad + 4 * (size_t)st.voxel[k] + ch, val);
  }
  // the next write-out reuses the area
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Move the slots of axis AX (0, 1, 2; coordinates co) to a cell with base b
// on that axis: returns the slots to write out first, those whose coordinate
// changes (the slots of parity p on axis AX: bit AX of the index equal to p),
// and sets the new coordinates in `next`.
template <int AX>
__device__ __forceinline__ uint32_t corner_move(const int co[2], int b, int next[2]) {
  constexpr uint32_t kLow = AX == 0 ? 0x55u : (AX == 1 ? 0x33u : 0x0Fu);
  next[0] = (b & 1) == 0 ? b : b + 1;
  next[1] = (b & 1) == 1 ? b : b + 1;
  return (co[0] != next[0] ? kLow : 0u) | (co[1] != next[1] ? (kLow ^ 0xFFu) : 0u);
}

// The cell base (floor of the grid coordinate) of the sample at x.
__device__ __forceinline__ void vol_base(const DevScene& S, V3 x, int& bx, int& by, int& bz) {
  bx = (int)floorf((x.x - S.vol_lo[0]) * S.vol_inv_vox - 0.5f);
  by = (int)floorf((x.y - S.vol_lo[1]) * S.vol_inv_vox - 0.5f);
  bz = (int)floorf((x.z - S.vol_lo[2]) * S.vol_inv_vox - 0.5f);
}

// One pixel's replay of a volume slice (see above); every lane of the wave
// calls it, those with active unset trace nothing.
__device__ __forceinline__ void vol_replay(const DevScene& S, const RepArgs& A,
                                           const RepSlice& sl, VolStage& st, bool active,
                                           uint32_t pix, int px, int py, uint32_t iter,
                                           int& n_samples) {
  const bool pair = G(sl.params_b) != nullptr;
  const float* pa = G(sl.params);
  const float* pb = G(sl.params_b);
  float* grad = G(sl.grad);
  VolRay r{};
  float adj[3], adj_b[3];
  double rem[3], rem_b[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    adj[ch] = adj_b[ch] = 0.0f;
    rem[ch] = rem_b[ch] = 0.0;
  }
  if (active) {
    const Rng rng = make_rng(stream_key(A.key.seed, iter, sl.tag), pix, sl.sample);
    r = vol_ray(S, rng, px, py, A.flags);
    const double* Ca = G(A.slots) + ((size_t)sl.slot_a * A.npix + pix) * 3;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      adj[ch] = G(sl.delta)[3 * (size_t)pix + ch] * sl.adj_scale;
      rem[ch] = Ca[ch];
    }
    if (pair) {
      const double* Cb = G(A.slots) + ((size_t)sl.slot_b * A.npix + pix) * 3;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        adj_b[ch] = G(sl.delta_b)[3 * (size_t)pix + ch] * sl.adj_scale;
        rem_b[ch] = Cb[ch];
      }
    }
  }
  const float sign = pair ? 1.0f : sl.sign;
  float T = 1.0f, Tb = 1.0f;
  CornerSums cs;
#pragma unroll
  for (int q = 0; q < 8; ++q) cs.acc[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int p = 0; p < 2; ++p) cs.x[p] = cs.y[p] = cs.z[p] = INT_MIN;
  // the wave's longest march (a scalar bound keeps the loop's registers as
  // few as a per-lane bound would)
  int n_wave = r.n;
  for (int o = 32; o > 0; o >>= 1) n_wave = max(n_wave, __shfl_xor(n_wave, o, 64));
  n_wave = __builtin_amdgcn_readfirstlane(n_wave);
  for (int k = 0; k < n_wave; ++k) {
    const bool live = k < r.n;
    const V3 xs = r.o + r.d * (r.t0 + ((float)k + r.us) * r.dt);
    int bx = 0, by = 0, bz = 0;
    if (live) vol_base(S, xs, bx, by, bz);
    if (k == 0) {  // the slots start at the first cell's corners (sums zero)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        cs.x[p] = ((bx & 1) == p) ? bx : bx + 1;
        cs.y[p] = ((by & 1) == p) ? by : by + 1;
        cs.z[p] = ((bz & 1) == p) ? bz : bz + 1;
      }
    }
    int nx[2], ny[2], nz[2];
    uint32_t f = corner_move<0>(cs.x, bx, nx) | corner_move<1>(cs.y, by, ny) |
                 corner_move<2>(cs.z, bz, nz);
    corner_write(S, grad, cs, st, live ? f : 0u);
    if (!live) continue;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      cs.x[p] = nx[p];
      cs.y[p] = ny[p];
      cs.z[p] = nz[p];
    }
    const VolCell c = vol_cell(S, xs);
    float g[4];
    {
      const float4 v = vol_fetch(pa, c);
      const float od = S.vol_sigma * v.w * r.dt;
      const float a = -expm1f(-od), et = expf(-od);
      const float e[3] = {v.x, v.y, v.z};
      const float Tn = T * et;
      float gs = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        rem[ch] -= (double)(T * a * e[ch]);
        g[ch] = adj[ch] * T * a;
        gs += adj[ch] * (Tn * e[ch] - (float)rem[ch]);
      }
      g[3] = gs * r.dt * S.vol_sigma;
      T = Tn;
    }
    if (pair) {
      const float4 v = vol_fetch(pb, c);
      const float od = S.vol_sigma * v.w * r.dt;
      const float a = -expm1f(-od), et = expf(-od);
      const float e[3] = {v.x, v.y, v.z};
      const float Tn = Tb * et;
      float gb[4], gs = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        rem_b[ch] -= (double)(Tb * a * e[ch]);
        gb[ch] = adj_b[ch] * Tb * a;
        gs += adj_b[ch] * (Tn * e[ch] - (float)rem_b[ch]);
      }
      gb[3] = gs * r.dt * S.vol_sigma;
      Tb = Tn;
#pragma unroll
      for (int q = 0; q < 4; ++q) g[q] -= gb[q];
    }
    // slot sl holds the cell's low corner on an axis when its parity there is
    // the base's
    const float wx0 = ((c.bx & 1) == 0) ? 1.0f - c.fx : c.fx;
    const float wy0 = ((c.by & 1) == 0) ? 1.0f - c.fy : c.fy;
    const float wz0 = ((c.bz & 1) == 0) ? 1.0f - c.fz : c.fz;
#pragma unroll
    for (int sl = 0; sl < 8; ++sl) {
      const float w = ((sl & 1) ? 1.0f - wx0 : wx0) * ((sl & 2) ? 1.0f - wy0 : wy0) *
                      ((sl & 4) ? 1.0f - wz0 : wz0) * sign;
      cs.acc[sl].x += w * g[0];
      cs.acc[sl].y += w * g[1];
      cs.acc[sl].z += w * g[2];
      cs.acc[sl].w += w * g[3];
    }
  }
  corner_write(S, grad, cs, st, r.n > 0 ? 0xFFu : 0u);
  n_samples = r.n;
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
k_vol_adjoint(const RepArgs* __restrict__ Units, int n_units, unsigned long long* work) {
  using SH = Shape<TW, TH>;
  __shared__ VolStage s_stage[SH::N / 64];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const RepArgs& A = unit_of(Units, n_units, b);
  const uint32_t iter = iteration_of(A.key);
  if (A.h.max_iter && iter >= A.h.max_iter) return;  // finished problem
  const DevScene& S = *G(A.scene);
  const TileBlock tb = vol_tile_block<SH>(A, b);
  const RepSlice& sl = A.sl[tb.slice];
  int px, py;
  const bool inside = tile_pixel<SH>(A.crop, tb, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(G(A.mask) && G(A.mask)[pix]);
  int n_samples = 0;
  vol_replay(S, A, sl, s_stage[threadIdx.x / 64], active, pix, px, py, iter, n_samples);
  count_work(work, active ? 1 : 0, n_samples);
}

// The bricked copy of a volume parameter vector (BrickArgs), one destination
// voxel per thread (the writes are contiguous).
__global__ void __launch_bounds__(kBrickBlock) k_vol_brick(const BrickArgs* __restrict__ Units,
                                                           int n_units) {
  const BrickArgs& A = unit_of(Units, n_units);
  const uint32_t lb = blockIdx.x - A.h.block0;
  const int R = A.R, Rb = A.Rb;
  const size_t n = (size_t)Rb * Rb * Rb * 64;
  for (size_t d = (size_t)lb * kBrickBlock + threadIdx.x; d < n;
       d += (size_t)A.nblocks * kBrickBlock) {
    const uint32_t brick = (uint32_t)(d >> 6), m = (uint32_t)d & 63u;
    const int x = (int)(brick % (uint32_t)Rb) * 4 + (int)((m & 1u) | ((m >> 2) & 2u));
    const int y = (int)((brick / (uint32_t)Rb) % (uint32_t)Rb) * 4 +
                  (int)(((m >> 1) & 1u) | ((m >> 3) & 2u));
    const int z = (int)(brick / ((uint32_t)Rb * (uint32_t)Rb)) * 4 +
                  (int)(((m >> 2) & 1u) | ((m >> 4) & 2u));
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (x < R && y < R && z < R) v = G(A.src)[((size_t)z * R + y) * R + x];
    G(A.dst)[d] = v;
  }
}

// ---------------------------------------------------------------------------
// fused meta-estimator + stabilised step
// ---------------------------------------------------------------------------
// Each thread takes kMetaK elements, one block-width apart, with every load
// issued before the arithmetic so the HBM latency is paid once.  The squared
// step is reduced per block into the partials buffer; the last block to finish sums
// the partials in block order (a deterministic ||pi_{i+1} - pi_i||^2) and
// advances the iteration state.
__global__ void __launch_bounds__(kMetaBlock) k_meta(const MetaArgs* __restrict__ Units,
                                                     int n_units) {
  __shared__ double s_coef[4];
  __shared__ double s_red[kMetaBlock / 64];
  __shared__ bool s_last;
  const MetaArgs& A = unit_of(Units, n_units);
  Ctl* ctl = G(A.ctl);
  const uint32_t it = ctl->iteration;
  if (A.h.max_iter && it >= A.h.max_iter) return;  // finished problem
  const uint32_t lb = blockIdx.x - A.h.block0, nb = A.nblocks;
  if (threadIdx.x == 0) {
    const double n2 = ctl->norm2[it & 1u];
    const uint32_t cF = ctl->count_F + 1u;
    const bool takeD = it >= 1u && n2 > 0.0;
    const uint32_t cD = ctl->count_D + (takeD ? 1u : 0u);
    s_coef[0] = (1.0 - A.beta_F) / (1.0 - pow(A.beta_F, (double)cF));
    s_coef[1] = takeD ? (1.0 - A.beta_D) / (1.0 - pow(A.beta_D, (double)cD)) : 0.0;
    s_coef[2] = takeD ? n2 : 0.0;
    s_coef[3] = takeD ? 1.0 : 0.0;
  }
  __syncthreads();
  const double wF = s_coef[0], wD = s_coef[1], n2 = s_coef[2];
  const bool takeD = s_coef[3] != 0.0;
  const double sq_n2 = takeD ? sqrt(n2) : 1.0;
  const uint32_t n = (uint32_t)A.n, nc = (uint32_t)A.n_ch;
  double local = 0.0;
  const uint32_t span = kMetaBlock * kMetaK;
  const uint32_t ab = A.ablate;  // uniform
  const bool centred = (ab & JSO_ABLATE_CENTRED) != 0;
  const bool uncorr = (ab & JSO_ABLATE_UNCORRELATED) != 0;
  const bool clip = (ab & JSO_ABLATE_NO_CLIP) == 0;
  for (uint32_t base = lb * span + threadIdx.x; base < n; base += nb * span) {
    float F[kMetaK], dF[kMetaK], p[kMetaK];
    double m2F[kMetaK], m2D[kMetaK], mean[kMetaK], var[kMetaK], ap[kMetaK];
#pragma unroll
    for (int e = 0; e < kMetaK; ++e) {
      const uint32_t i = base + (uint32_t)e * kMetaBlock;
      if (i < n) {
        F[e] = G(A.F)[i];
        dF[e] = takeD ? G(A.dF)[i] : 0.0f;
        p[e] = G(A.params)[i];
        m2F[e] = G(A.m2F)[i];
        m2D[e] = G(A.m2D)[i];
        mean[e] = G(A.mean)[i];
        var[e] = G(A.var)[i];
        ap[e] = G(A.alpha_prev)[i];
      }
    }
#pragma unroll
    for (int e = 0; e < kMetaK; ++e) {
      const uint32_t i = base + (uint32_t)e * kMetaBlock;
      if (i >= n) continue;
      const double f = (double)F[e], df = (double)dF[e];
      // Var[F] (Eq. 9; bias-corrected Moment2)
      const double xF = uncorr ? (double)G(A.Fv)[i] : f;
      const double mF = m2F[e] + wF * (xF * xF - m2F[e]);
      double varF = mF;
      if (centred) {
        const double m1 = G(A.m1F)[i] + wF * (xF - G(A.m1F)[i]);
        G(A.m1F)[i] = m1;
        varF = fmax(mF - m1 * m1, 0.0);
      }
      // Var[dF] (Eq. 13-14)
      double mD = m2D[e];
      double varD = 0.0;
      if (takeD) {
        const double x = (uncorr ? (double)G(A.dFv)[i] : df) / sq_n2;
        mD = mD + wD * (x * x - mD);
        double vd = mD;
        if (centred) {
          const double m1 = G(A.m1D)[i] + wD * (x - G(A.m1D)[i]);
          G(A.m1D)[i] = m1;
          vd = fmax(mD - m1 * m1, 0.0);
        }
        varD = vd * n2;
      }
      // carry the previous estimate forward, weight (Eq. 8, 17), combine (Eq. 7, 15)
      double mu = mean[e] + df;
      double v = var[e] + varD;
      // Eq. 8; a parameter with every variance zero (untouched so far) gets alpha = 0
      const double den = varF + v;
      double a = den > 0.0 ? varF / den : 0.0;
      if (clip)
        a = fmin(a, 1.0 / (2.0 - ap[e]));
      else if (isinf(ap[e]))
        a = 0.0;  // the ablation drops Eq. 17 only: alpha_0 = 0 (Eq. 7's initialisation)
      mu = a * mu + (1.0 - a) * f;
      v = a * a * v + (1.0 - a) * (1.0 - a) * varF;
      // stabilised step (Eq. 21) and projection
      const double step = -(double)A.eta * mu / (sqrt(v) + 1e-8);
      const uint32_t ch = i % nc;
      const float pn = fminf(fmaxf((float)((double)p[e] + step), A.lo[ch]), A.hi[ch]);
      const double dp = (double)pn - (double)p[e];
      local += dp * dp;
      G(A.m2F)[i] = mF;
      G(A.m2D)[i] = mD;
      G(A.mean)[i] = mu;
      G(A.var)[i] = v;
      G(A.alpha_prev)[i] = a;
      G(A.params_prev)[i] = p[e];
      G(A.params)[i] = pn;
      if (A.zero_grads) {
        G(A.F)[i] = 0.0f;
        G(A.dF)[i] = 0.0f;
        if (uncorr) {
          G(A.Fv)[i] = 0.0f;
          G(A.dFv)[i] = 0.0f;
        }
      }
    }
  }
  // ||pi_{i+1} - pi_i||^2 for the next iteration
  local = wave_sum(local);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) s_red[wv] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kMetaBlock / 64; ++w) tot += s_red[w];
    G(A.partials)[lb] = tot;
    __threadfence();
    s_last = atomicAdd(&ctl->blocks_done, 1u) == nb - 1u;
  }
  __syncthreads();
  if (!s_last) return;
  // last block: every block's partial is visible and every block has read
  // this iteration's inputs
  __threadfence();
  double sum = 0.0;
  if (threadIdx.x < 64) {
    for (uint32_t b = threadIdx.x; b < nb; b += 64) sum += G(A.partials)[b];
    sum = wave_sum(sum);
  }
  if (threadIdx.x == 0) {
    ctl->norm2[(it + 1u) & 1u] = sum;
    ctl->count_F = ctl->count_F + 1u;
    if (takeD) ctl->count_D = ctl->count_D + 1u;
    ctl->norm2[it & 1u] = 0.0;
    ctl->loss[(it + 1u) & 1u] = 0.0;
    ctl->iteration = it + 1u;
    ctl->blocks_done = 0u;
    __threadfence();
  }
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kMetaBlock) k_adam(const AdamArgs* __restrict__ Units,
                                                     int n_units) {
  __shared__ uint32_t s_it, s_t;
  const AdamArgs& A = unit_of(Units, n_units);
  Ctl* ctl = G(A.ctl);
  // one read of the iteration state per block: the last block advances it
  // once every block has signalled, and every wave must have read it by then
  if (threadIdx.x == 0) {
    s_it = ctl->iteration;
    s_t = ctl->adam_t;
  }
  __syncthreads();
  if (A.h.max_iter && s_it >= A.h.max_iter) return;  // finished problem (block-uniform)
  const uint32_t lb = blockIdx.x - A.h.block0, nb = A.nblocks;
  const uint32_t t = s_t + 1u;
  const float bc1 = (float)(1.0 - pow((double)A.beta1, (double)t));
  const float bc2 = (float)(1.0 - pow((double)A.beta2, (double)t));
  const size_t stride = (size_t)nb * kMetaBlock;
  for (size_t i = (size_t)lb * kMetaBlock + threadIdx.x; i < A.n; i += stride) {
    const float g = G(A.g)[i];
    const float m = A.beta1 * G(A.m)[i] + (1.0f - A.beta1) * g;
    const float v = A.beta2 * G(A.v)[i] + (1.0f - A.beta2) * g * g;
    G(A.m)[i] = m;
    G(A.v)[i] = v;
    const float mh = m / bc1, vh = v / bc2;
    const float p = G(A.params)[i];
    const int ch = (int)(i % (size_t)A.n_ch);
    const float pn = fminf(fmaxf(p - A.eta * mh / (sqrtf(vh) + A.eps), A.lo[ch]), A.hi[ch]);
    G(A.params_prev)[i] = p;
    G(A.params)[i] = pn;
    if (A.zero_grads) G(A.g)[i] = 0.0f;
  }
  __syncthreads();  // every wave of the block is done before it signals
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&ctl->blocks_done, 1u);
    if (done == nb - 1u) {
      __threadfence();
      ctl->adam_t = t;
      ctl->iteration = s_it + 1u;
      ctl->loss[(s_it + 1u) & 1u] = 0.0;
      ctl->blocks_done = 0u;
      __threadfence();
    }
  }
}

// ---------------------------------------------------------------------------
// texture-gradient preconditioner: one cosine-transform pass
// ---------------------------------------------------------------------------
// 64 x 64 outputs per block, k in chunks of 16 staged through LDS; each
// thread accumulates a 4 x 4 patch (rows m, columns j) in FP32.
constexpr int kDctK = 16;

__device__ __forceinline__ size_t dct_addr(const DctArgs& U, int k, int j) {
  return (size_t)k * U.sk + (size_t)(j / U.jin) * U.sjo + (size_t)(j % U.jin);
}

__global__ void __launch_bounds__(kDctBlock) k_dct(const DctArgs* __restrict__ Units,
                                                   int n_units) {
  __shared__ float s_a[kDctK][kDctTile + 1];
  __shared__ float s_b[kDctK][kDctTile + 1];
  const DctArgs& U = unit_of(Units, n_units);
  const uint32_t local = blockIdx.x - U.h.block0;
  const int m0 = (int)(local / U.tiles_j) * kDctTile, j0 = (int)(local % U.tiles_j) * kDctTile;
  const int tid = (int)threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;  // outputs: rows m0 + ty + 16 r, columns j0 + tx + 16 q
  const float* A = G(U.A);
  const float* in = G(U.in);
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0f;
  for (int k0 = 0; k0 < U.n; k0 += kDctK) {
    // stage A[m0 .. m0+63][k0 .. k0+15] and in(k0 .. k0+15, j0 .. j0+63)
#pragma unroll
    for (int e = tid; e < kDctK * kDctTile; e += kDctBlock) {
      const int kk = e % kDctK, mm = e / kDctK;
      const int m = m0 + mm, k = k0 + kk;
      float a = 0.0f;
      if (m < U.n && k < U.n) a = U.transA ? A[(size_t)k * U.n + m] : A[(size_t)m * U.n + k];
      s_a[kk][mm] = a;
      const int jj = e % kDctTile, kb = e / kDctTile;
      const int j = j0 + jj, kr = k0 + kb;
      s_b[kb][jj] = (j < U.N && kr < U.n) ? in[dct_addr(U, kr, j)] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kDctK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = s_a[kk][ty + 16 * r];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = s_b[kk][tx + 16 * q];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fmaf(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
  float* out = G(U.out);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = m0 + ty + 16 * r;
    if (m >= U.n) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx + 16 * q;
      if (j >= U.N) continue;
      float v = acc[r][q];
      if (G(U.eig_m)) v /= 1.0f + U.lambda * (G(U.eig_m)[m] + G(U.eig_j)[j / U.jdiv]);
      out[dct_addr(U, m, j)] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// deterministic mode: fold the fixed-point accumulators into their gradients
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kFxBlock) k_fx_flush(const FxArgs* __restrict__ Units,
                                                        int n_units) {
  const FxArgs& A = unit_of(Units, n_units);
  const uint32_t lb = blockIdx.x - A.h.block0;
  for (size_t i = (size_t)lb * kFxBlock + threadIdx.x; i < A.n;
       i += (size_t)A.nblocks * kFxBlock) {
    const long long v = (long long)G(A.fx)[i];
    if (v != 0) {
      G(A.grad)[i] += (float)((double)v * A.inv_scale);
      G(A.fx)[i] = 0ull;
    }
  }
}

__global__ void k_fill_f64(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* p, size_t n, float v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_philox(const uint32_t* ctr, size_t n, uint64_t key, uint32_t* out,
                         hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(cdiv(n, 256)), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(ctr), (uint32_t)n, (uint32_t)key,
                     (uint32_t)(key >> 32), reinterpret_cast<uint4*>(out));
  return hipGetLastError();
}

// LDS entries of the traversal stack per lane for a launch whose deepest mesh
// needs `stack` entries (the rest spill to private memory).
static int lds_stack(int stack) { return stack < kLdsStack ? stack : kLdsStack; }

// Grid of a launch of `blocks` tiles: all of them, or with a work queue a
// persistent grid of at most `persist` blocks.
static uint32_t grid_of(uint32_t blocks, const uint32_t* queue, uint32_t persist) {
  return queue && persist < blocks ? persist : blocks;
}

template <int TW, int TH, bool kShared>
static void fwd_launch(const FwdArgs* U, int n, uint32_t blocks, int stack,
                       unsigned long long* work, uint32_t* queue, uint32_t persist,
                       hipStream_t st) {
  const int cap = lds_stack(stack);
  const size_t lds = (size_t)cap * TW * TH * 4;
  const dim3 grid(grid_of(blocks, queue, persist));
  if (stack > 0)
    hipLaunchKernelGGL((k_forward<TW, TH, true, kShared>), grid, dim3(TW * TH), lds, st,
                       U, n, cap, work, queue, blocks);
  else
    hipLaunchKernelGGL((k_forward<TW, TH, false, kShared>), grid, dim3(TW * TH), 0, st,
                       U, n, 0, work, queue, blocks);
}
template <int TW, int TH>
static void fwd_launch(const FwdArgs* U, int n, uint32_t blocks, int stack, bool shared,
                       unsigned long long* work, uint32_t* queue, uint32_t persist,
                       hipStream_t st) {
  if (shared)
    fwd_launch<TW, TH, true>(U, n, blocks, stack, work, queue, persist, st);
  else
    fwd_launch<TW, TH, false>(U, n, blocks, stack, work, queue, persist, st);
}
hipError_t launch_forward(const FwdArgs* U, int n, uint32_t blocks, int shape, int stack,
                          bool shared, unsigned long long* work, hipStream_t st,
                          uint32_t* queue, uint32_t persist) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  if (stack < 0 || stack > kBvhMaxStack) return hipErrorInvalidValue;
  if (queue && persist == 0) return hipErrorInvalidValue;
  switch (shape) {
    case 0: fwd_launch<16, 16>(U, n, blocks, stack, shared, work, queue, persist, st); break;
    case 1: fwd_launch<16, 8>(U, n, blocks, stack, shared, work, queue, persist, st); break;
    case 2: fwd_launch<8, 8>(U, n, blocks, stack, shared, work, queue, persist, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(blocks), dim3(kFinBlock), 0, st, U, n);
  return hipGetLastError();
}

size_t adjoint_lds_bytes(int n_ch) {
  const size_t table = (size_t)kTableSize * 4 * (1 + (size_t)n_ch);
  const size_t xchg = (size_t)kRepXchgWords * kXchg * 4;
  return table > xchg ? table : xchg;
}

template <int TW, int TH, bool kShared, bool kDet>
static void adj_launch(const RepArgs* U, int n, uint32_t blocks, size_t lds, int stack,
                       unsigned long long* work, uint32_t* queue, uint32_t persist,
                       hipStream_t st) {
  const int cap = lds_stack(stack);
  const dim3 grid(grid_of(blocks, queue, persist));
  if (stack > 0)
    hipLaunchKernelGGL((k_adjoint<TW, TH, true, kShared, kDet>), grid, dim3(TW * TH),
                       lds + (size_t)cap * TW * TH * 4, st, U, n, cap, work, queue, blocks);
  else
    hipLaunchKernelGGL((k_adjoint<TW, TH, false, kShared, kDet>), grid, dim3(TW * TH), lds, st,
                       U, n, 0, work, queue, blocks);
}
template <int TW, int TH>
static void adj_launch(const RepArgs* U, int n, uint32_t blocks, size_t lds, int stack,
                       bool shared, bool det, unsigned long long* work, uint32_t* queue,
                       uint32_t persist, hipStream_t st) {
  if (det)  // one instance takes every kind of slice
    adj_launch<TW, TH, true, true>(U, n, blocks, lds, stack, work, queue, persist, st);
  else if (shared)
    adj_launch<TW, TH, true, false>(U, n, blocks, lds, stack, work, queue, persist, st);
  else
    adj_launch<TW, TH, false, false>(U, n, blocks, lds, stack, work, queue, persist, st);
}

hipError_t launch_adjoint(const RepArgs* U, int n, uint32_t blocks, int shape, size_t lds,
                          int stack, bool shared, unsigned long long* work, hipStream_t st,
                          uint32_t* queue, uint32_t persist, bool det) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  if (lds < adjoint_lds_bytes(0) || lds > adjoint_lds_bytes(5)) return hipErrorInvalidValue;
  if (stack < 0 || stack > kBvhMaxStack) return hipErrorInvalidValue;
  if (queue && persist == 0) return hipErrorInvalidValue;
  switch (shape) {
    case 0: adj_launch<16, 16>(U, n, blocks, lds, stack, shared, det, work, queue, persist, st); break;
    case 1: adj_launch<16, 8>(U, n, blocks, lds, stack, shared, det, work, queue, persist, st); break;
    case 2: adj_launch<8, 8>(U, n, blocks, lds, stack, shared, det, work, queue, persist, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vol_forward(const FwdArgs* U, int n, uint32_t blocks, int waves,
                              unsigned long long* work, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  if (waves < 1 || waves > kVolMaxSliceWaves) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vol_forward, dim3(blocks), dim3(64 * waves), 0, st, U, n, work);
  return hipGetLastError();
}

hipError_t launch_vol_adjoint(const RepArgs* U, int n, uint32_t blocks, int shape,
                              unsigned long long* work, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  switch (shape) {
    case 0: hipLaunchKernelGGL((k_vol_adjoint<16, 16>), dim3(blocks), dim3(256), 0, st, U, n, work); break;
    case 1: hipLaunchKernelGGL((k_vol_adjoint<16, 8>), dim3(blocks), dim3(128), 0, st, U, n, work); break;
    case 2: hipLaunchKernelGGL((k_vol_adjoint<8, 8>), dim3(blocks), dim3(64), 0, st, U, n, work); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_vol_brick(const BrickArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_vol_brick, dim3(blocks), dim3(kBrickBlock), 0, st, U, n);
  return hipGetLastError();
}

hipError_t launch_dct(const DctArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dct, dim3(blocks), dim3(kDctBlock), 0, st, U, n);
  return hipGetLastError();
}

hipError_t launch_meta(const MetaArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_meta, dim3(blocks), dim3(kMetaBlock), 0, st, U, n);
  return hipGetLastError();
}

hipError_t launch_fx_flush(const FxArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fx_flush, dim3(blocks), dim3(kFxBlock), 0, st, U, n);
  return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs* U, int n, uint32_t blocks, hipStream_t st) {
  if (n <= 0 || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(kMetaBlock), 0, st, U, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(cdiv(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace jso

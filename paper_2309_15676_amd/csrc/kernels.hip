// HIP kernels of the jso hot path (gfx950).
//
//   k_philox   - Philox4x32-10 block function over a counter array
//   k_primal   - primal renders of one or more parameter sets; writes the
//                L2 adjoint image 2 (I - T) / (3 W H) and the loss
//   k_adjoint  - replayed adjoint: forward pass for each path's radiance, then
//                a second pass over the same random numbers that forms the
//                per-vertex material derivatives and scatters them; a
//                finite-difference job replays the paths at pi_i and pi_{i-1}
//                in lockstep and differences coinciding vertices in registers
//   k_meta     - fused meta-estimator + stabilised step (FP64 state)
//   k_adam     - Adam baseline
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace jso {

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

// Blocks are kTile x kTile pixel tiles (256 lanes = four wave64 rows of 16 x 4).
constexpr int kTile = 16;
constexpr int kBlock = kTile * kTile;

__device__ __forceinline__ bool tile_pixel(const Crop& c, int& px, int& py) {
  px = c.x0 + (int)blockIdx.x * kTile + (int)(threadIdx.x % kTile);
  py = c.y0 + (int)blockIdx.y * kTile + (int)(threadIdx.x / kTile);
  return px < c.x1 && py < c.y1;
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_primal(const DevScene* __restrict__ Sp,
                                                   PrimalArgs A) {
  const DevScene& S = *Sp;
  const PrimalJob& job = A.jobs[blockIdx.z];
  int px, py;
  const bool inside = tile_pixel(A.crop, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(A.mask && A.mask[pix]);
  double se = 0.0;
  if (active) {
    const uint64_t key = stream_key(A.key.seed, iteration_of(A.key), job.tag);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < job.spp; ++s) {
      double C[3];
      path_radiance(S, job.params, make_rng(key, pix, (uint32_t)s), px, py, A.flags, C);
      acc[0] += C[0];
      acc[1] += C[1];
      acc[2] += C[2];
    }
    const double inv = 1.0 / (double)job.spp;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float I = (float)(acc[k] * inv);
      if (job.img) job.img[3 * (size_t)pix + k] = I;
      if (job.delta) {
        const float T = A.target[3 * (size_t)pix + k];
        const float e = I - T;
        job.delta[3 * (size_t)pix + k] = A.delta_scale * e;
        se += (double)e * (double)e;
      }
    }
  } else if (inside && job.delta) {
#pragma unroll
    for (int k = 0; k < 3; ++k) job.delta[3 * (size_t)pix + k] = 0.0f;
  }
  if (job.loss2) {
    se = wave_sum(se);
    if ((threadIdx.x & 63) == 0 && se != 0.0)
      unsafeAtomicAdd(&job.loss2[iteration_of(A.key) & 1u], se * A.loss_scale);
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
constexpr int kTableBits = 11;
constexpr int kTableSize = 1 << kTableBits;  // texels per block table
constexpr int kTableCh = 5;                  // value slots per texel (max channels)
constexpr int kMaxProbe = 32;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
// LDS per block: kTableSize * (4 + 4 * kTableCh) bytes = 48 KiB

struct GradTable {
  uint32_t* keys;  // LDS: texel index of each slot
  float* vals;     // LDS: kTableCh gradient values per slot
  float* grad;     // global gradient buffer of this block's job
};

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

// Texel q of the footprint (q = 0..3: x-offset q & 1, y-offset q >> 1) and its
// bilinear weight, computed arithmetically so no per-lane array is indexed.
__device__ __forceinline__ void footprint_texel(const Footprint& fp, int q, int& texel,
                                                float& w) {
  const int dx = fp.t01 - fp.t00, dy = fp.t10 - fp.t00;
  texel = fp.t00 + (q & 1) * dx + (q >> 1) * dy;
  w = ((q & 1) ? fp.fx : 1.0f - fp.fx) * ((q & 2) ? fp.fy : 1.0f - fp.fy);
}

// Add one first-hit vertex's material gradient g (R, G, B, metal, rough) to
// its four texels in the block table (global atomics when a probe sequence is
// congested).
__device__ __forceinline__ void scatter_texels(const DevScene& S, const GradTable& T,
                                               const Footprint& fp, const float g[5],
                                               float sign) {
  const int nc = S.n_ch;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    int texel;
    float w;
    footprint_texel(fp, q, texel, w);
    if (w == 0.0f) continue;
    const int h = table_slot(T, (uint32_t)texel);
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int s = S.slot[b];
      if (s < 0) continue;
      const float v = w * (sign * g[b]);
      if (v == 0.0f) continue;
      if (h >= 0)
        __hip_atomic_fetch_add(&T.vals[h * kTableCh + s], v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        unsafeAtomicAdd(T.grad + (size_t)texel * nc + s, v);
    }
  }
}

// Scatter the later-vertex gradient of every lane with `has` set straight to
// memory.  Device-scope float atomics are priced per cache line, so the wave
// spreads each vertex over 4 * n_ch lanes, neighbouring lanes taking the
// neighbouring channels of one texel: a texel then costs one transaction
// instead of n_ch.  Must be reached by all 64 lanes of the wave.
__device__ __forceinline__ void scatter_wave(const DevScene& S, float* __restrict__ grad,
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
    const int t00 = __shfl(v.fp.t00, src, 64);
    const int t01 = __shfl(v.fp.t01, src, 64);
    const int t10 = __shfl(v.fp.t10, src, 64);
    const float fx = __shfl(v.fp.fx, src, 64);
    const float fy = __shfl(v.fp.fy, src, 64);
    float gc = 0.0f;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const float x = __shfl(v.g[b], src, 64);
      if (S.slot[b] == c) gc = x;
    }
    if (work) {
      const int texel = t00 + (q & 1) * (t01 - t00) + (q >> 1) * (t10 - t00);
      const float w = ((q & 1) ? fx : 1.0f - fx) * ((q & 2) ? fy : 1.0f - fy);
      const float val = w * (sign * gc);
      if (val != 0.0f) unsafeAtomicAdd(grad + (size_t)texel * nc + c, val);
    }
    for (int k = 0; k < nv && m != 0; ++k) m &= m - 1;
  }
}

__device__ __forceinline__ bool same_footprint(const Footprint& a, const Footprint& b) {
  return a.global == b.global && a.t00 == b.t00 && a.t01 == b.t01 && a.t10 == b.t10 &&
         a.t11 == b.t11 && __float_as_uint(a.fx) == __float_as_uint(b.fx) &&
         __float_as_uint(a.fy) == __float_as_uint(b.fy);
}

// Accumulates vertex gradients: global materials into per-lane registers
// (reduced over the wave at the end), first-hit texels into the block's table;
// later textured vertices are handed back for the wave-cooperative scatter.
struct Sink {
  float acc[5];
  GradTable T;
  __device__ __forceinline__ void init(const GradTable& t) {
    T = t;
#pragma unroll
    for (int b = 0; b < 5; ++b) acc[b] = 0.0f;
  }
  // returns true when v is a later textured vertex left to scatter_wave
  __device__ __forceinline__ bool add(const DevScene& S, const VertexGrad& v, float sign) {
    if (!v.valid) return false;
    if (v.fp.global) {
#pragma unroll
      for (int b = 0; b < 5; ++b) acc[b] += sign * v.g[b];
      return false;
    }
    if (v.j > 1) return true;
    scatter_texels(S, T, v.fp, v.g, sign);
    return false;
  }
  // every lane of the block reaches this point
  __device__ __forceinline__ void flush(const DevScene& S) {
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int s = S.slot[b];
      const float v = wave_sum(acc[b]);
      if (s >= 0 && (threadIdx.x & 63) == 0 && v != 0.0f) unsafeAtomicAdd(T.grad + s, v);
    }
    __syncthreads();
    // neighbouring lanes flush neighbouring channels of one texel
    const int nc = S.n_ch;
    for (int i = threadIdx.x; i < kTableSize * nc; i += kBlock) {
      const int slot = i / nc;
      const int c = i - slot * nc;
      const uint32_t k = T.keys[slot];
      if (k == kEmpty) continue;
      const float v = T.vals[slot * kTableCh + c];
      if (v != 0.0f) unsafeAtomicAdd(T.grad + (size_t)k * nc + c, v);
    }
  }
};

// One block = one kTile x kTile pixel tile of one job's sample.  Each path is
// traced forward for its radiance, then replayed vertex by vertex; the loop is
// wave-uniform so the later-vertex scatter can use the whole wave.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_adjoint(const DevScene* __restrict__ Sp, AdjointArgs A) {
  const DevScene& S = *Sp;
  __shared__ uint32_t s_keys[kTableSize];
  __shared__ float s_vals[kTableSize * kTableCh];
  // find the job of this grid slice
  int ji = 0;
  while (ji + 1 < A.n_jobs && (int)blockIdx.z >= A.jobs[ji + 1].z0) ++ji;
  const AdjointJob& job = A.jobs[ji];
  const uint32_t sample = (uint32_t)(job.sample0 + ((int)blockIdx.z - job.z0));
  int px, py;
  const bool inside = tile_pixel(A.crop, px, py);
  const uint32_t pix = (uint32_t)(py * S.width + px);
  const bool active = inside && !(A.mask && A.mask[pix]);
  for (int i = threadIdx.x; i < kTableSize; i += kBlock) s_keys[i] = kEmpty;
  for (int i = threadIdx.x; i < kTableSize * kTableCh; i += kBlock) s_vals[i] = 0.0f;
  __syncthreads();
  Sink sink;
  sink.init(GradTable{s_keys, s_vals, job.grad});
  const uint64_t key = stream_key(A.key.seed, iteration_of(A.key), job.tag);
  const Rng rng = make_rng(key, pix, sample);
  const bool pair = job.params_b != nullptr;  // uniform over the block
  float adj_a[3] = {0.0f, 0.0f, 0.0f}, adj_b[3] = {0.0f, 0.0f, 0.0f};
  double Ca[3] = {0.0, 0.0, 0.0}, Cb[3] = {0.0, 0.0, 0.0};
  Path Pa, Pb;
  Pa.alive = Pb.alive = false;
  if (active) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      adj_a[k] = job.delta[3 * (size_t)pix + k] * job.adj_scale;
      if (pair) adj_b[k] = job.delta_b[3 * (size_t)pix + k] * job.adj_scale;
    }
    path_radiance(S, job.params, rng, px, py, A.flags, Ca);
    path_begin(S, rng, px, py, A.flags, Pa);
    if (pair) {
      path_radiance(S, job.params_b, rng, px, py, A.flags, Cb);
      path_begin(S, rng, px, py, A.flags, Pb);
    }
  }
  int n_vert = 0;
  if (!pair) {
    while (__ballot(Pa.alive) != 0) {
      VertexGrad va;
      va.valid = false;
      n_vert += Pa.alive ? 1 : 0;
      if (Pa.alive) path_vertex<true>(S, job.params, rng, A.flags, Pa, adj_a, Ca, va);
      const bool later = sink.add(S, va, job.sign);
      scatter_wave(S, job.grad, va, job.sign, later);
    }
  } else {
    // the pair is replayed in lockstep; coinciding vertices are differenced
    // in registers (+A - B)
    while (__ballot(Pa.alive || Pb.alive) != 0) {
      VertexGrad va, vb;
      va.valid = vb.valid = false;
      n_vert += (Pa.alive ? 1 : 0) + (Pb.alive ? 1 : 0);
      if (Pa.alive) path_vertex<true>(S, job.params, rng, A.flags, Pa, adj_a, Ca, va);
      if (Pb.alive) path_vertex<true>(S, job.params_b, rng, A.flags, Pb, adj_b, Cb, vb);
      if (va.valid && vb.valid && same_footprint(va.fp, vb.fp)) {
#pragma unroll
        for (int q = 0; q < 5; ++q) va.g[q] -= vb.g[q];
        vb.valid = false;
      }
      const bool later_a = sink.add(S, va, 1.0f);
      const bool later_b = sink.add(S, vb, -1.0f);
      scatter_wave(S, job.grad, va, 1.0f, later_a);
      scatter_wave(S, job.grad, vb, -1.0f, later_b);
    }
  }
  if (A.work) {
    const int paths = wave_sum(active ? (pair ? 2 : 1) : 0);
    const int verts = wave_sum(n_vert);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(A.work, (unsigned long long)paths);
      atomicAdd(A.work + 1, (unsigned long long)verts);
    }
  }
  sink.flush(S);
}

// ---------------------------------------------------------------------------
// fused meta-estimator + stabilised step
// ---------------------------------------------------------------------------
// Each thread takes kMetaK elements, one block-width apart, with every load
// issued before the arithmetic so the HBM latency is paid once.  The squared
// step is reduced per block into A.partials; the last block to finish sums
// the partials in block order (a deterministic ||pi_{i+1} - pi_i||^2) and
// advances the iteration state.
constexpr int kMetaK = 4;
constexpr int kMetaBlock = 256;

__global__ void __launch_bounds__(kMetaBlock) k_meta(MetaArgs A) {
  __shared__ double s_coef[4];
  __shared__ double s_red[kMetaBlock / 64];
  __shared__ bool s_last;
  Ctl* ctl = A.ctl;
  const uint32_t it = ctl->iteration;
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
  for (uint32_t base = blockIdx.x * span + threadIdx.x; base < n; base += gridDim.x * span) {
    float F[kMetaK], dF[kMetaK], p[kMetaK];
    double m2F[kMetaK], m2D[kMetaK], mean[kMetaK], var[kMetaK], ap[kMetaK];
#pragma unroll
    for (int e = 0; e < kMetaK; ++e) {
      const uint32_t i = base + (uint32_t)e * kMetaBlock;
      if (i < n) {
        F[e] = A.F[i];
        dF[e] = takeD ? A.dF[i] : 0.0f;
        p[e] = A.params[i];
        m2F[e] = A.m2F[i];
        m2D[e] = A.m2D[i];
        mean[e] = A.mean[i];
        var[e] = A.var[i];
        ap[e] = A.alpha_prev[i];
      }
    }
#pragma unroll
    for (int e = 0; e < kMetaK; ++e) {
      const uint32_t i = base + (uint32_t)e * kMetaBlock;
      if (i >= n) continue;
      const double f = (double)F[e], df = (double)dF[e];
      // Var[F] (Eq. 9; bias-corrected Moment2)
      const double mF = m2F[e] + wF * (f * f - m2F[e]);
      // Var[dF] (Eq. 13-14)
      double mD = m2D[e];
      double varD = 0.0;
      if (takeD) {
        const double x = df / sq_n2;
        mD = mD + wD * (x * x - mD);
        varD = mD * n2;
      }
      // carry the previous estimate forward, weight (Eq. 8, 17), combine (Eq. 7, 15)
      double mu = mean[e] + df;
      double v = var[e] + varD;
      double a = mF / (mF + v + 1e-30);
      a = fmin(a, 1.0 / (2.0 - ap[e]));
      mu = a * mu + (1.0 - a) * f;
      v = a * a * v + (1.0 - a) * (1.0 - a) * mF;
      // stabilised step (Eq. 21) and projection
      const double step = -(double)A.eta * mu / (sqrt(v) + 1e-8);
      const uint32_t ch = i % nc;
      const float pn = fminf(fmaxf((float)((double)p[e] + step), A.lo[ch]), A.hi[ch]);
      const double dp = (double)pn - (double)p[e];
      local += dp * dp;
      A.m2F[i] = mF;
      A.m2D[i] = mD;
      A.mean[i] = mu;
      A.var[i] = v;
      A.alpha_prev[i] = a;
      A.params_prev[i] = p[e];
      A.params[i] = pn;
      if (A.zero_grads) {
        A.F[i] = 0.0f;
        A.dF[i] = 0.0f;
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
    A.partials[blockIdx.x] = tot;
    __threadfence();
    s_last = atomicAdd(&ctl->blocks_done, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (!s_last) return;
  // last block: every block's partial is visible and every block has read
  // this iteration's inputs
  __threadfence();
  double sum = 0.0;
  if (threadIdx.x < 64) {
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += 64) sum += A.partials[b];
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
__global__ void __launch_bounds__(256) k_adam(AdamArgs A) {
  Ctl* ctl = A.ctl;
  const uint32_t t = ctl->adam_t + 1u;
  const float bc1 = (float)(1.0 - pow((double)A.beta1, (double)t));
  const float bc2 = (float)(1.0 - pow((double)A.beta2, (double)t));
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
    const float g = A.g[i];
    const float m = A.beta1 * A.m[i] + (1.0f - A.beta1) * g;
    const float v = A.beta2 * A.v[i] + (1.0f - A.beta2) * g * g;
    A.m[i] = m;
    A.v[i] = v;
    const float mh = m / bc1, vh = v / bc2;
    const float p = A.params[i];
    const int ch = (int)(i % (size_t)A.n_ch);
    const float pn = fminf(fmaxf(p - A.eta * mh / (sqrtf(vh) + A.eps), A.lo[ch]), A.hi[ch]);
    A.params_prev[i] = p;
    A.params[i] = pn;
    if (A.zero_grads) A.g[i] = 0.0f;
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t done = atomicAdd(&ctl->blocks_done, 1u);
    if (done == gridDim.x - 1u) {
      __threadfence();
      ctl->adam_t = t;
      ctl->iteration = ctl->iteration + 1u;
      ctl->loss[ctl->iteration & 1u] = 0.0;
      ctl->blocks_done = 0u;
      __threadfence();
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

hipError_t launch_primal(const DevScene* S, const PrimalArgs& A, int n_jobs, hipStream_t st) {
  const int w = A.crop.x1 - A.crop.x0, h = A.crop.y1 - A.crop.y0;
  if (w <= 0 || h <= 0 || n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_primal, dim3(cdiv(w, kTile), cdiv(h, kTile), n_jobs), dim3(kBlock), 0, st,
                     S, A);
  return hipGetLastError();
}

hipError_t launch_adjoint(const DevScene* S, const AdjointArgs& A, int n_slices, hipStream_t st) {
  const int w = A.crop.x1 - A.crop.x0, h = A.crop.y1 - A.crop.y0;
  if (w <= 0 || h <= 0 || n_slices <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint, dim3(cdiv(w, kTile), cdiv(h, kTile), n_slices), dim3(kBlock), 0,
                     st, S, A);
  return hipGetLastError();
}

static unsigned elementwise_grid(size_t n) {
  // at most 8 blocks per CU of 256 CUs; grid-stride beyond that
  const size_t want = (n + 255) / 256;
  return (unsigned)(want < 2048 ? (want ? want : 1) : 2048);
}

hipError_t launch_meta(const MetaArgs& A, hipStream_t st) {
  if (A.n >= (size_t)1 << 31 || A.n_ch < 1 || !A.partials) return hipErrorInvalidValue;
  const size_t want = cdiv(A.n, (size_t)kMetaBlock * kMetaK);
  const unsigned grid = (unsigned)(want < 1 ? 1 : (want > kMetaMaxBlocks ? kMetaMaxBlocks : want));
  hipLaunchKernelGGL(k_meta, dim3(grid), dim3(kMetaBlock), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(elementwise_grid(A.n)), dim3(256), 0, st, A);
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

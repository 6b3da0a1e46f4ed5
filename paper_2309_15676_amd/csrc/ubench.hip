// Memory-system microbenchmarks: the denominators of the roofline fractions
// the benchmark reports (a plain copy for HBM bandwidth, no-return FP32
// atomic adds under the address patterns a gradient scatter produces).  Not
// part of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "jso.h"

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_ub_copy(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 32-bit integer hash (a multiply-xorshift finaliser) of an operation index.
__device__ __forceinline__ uint32_t mix32(uint64_t x) {
  uint32_t h = (uint32_t)x ^ (uint32_t)(x >> 32) * 0x9E3779B9u;
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  h ^= h >> 15;
  h *= 0x846CA68Bu;
  h ^= h >> 16;
  return h;
}

// Operation i of a launch adds 1 to buf[index(i)].  Each thread issues kPer
// operations a grid apart (i = k * threads + thread), so one instruction of a
// wave covers 64 consecutive operation indices.
constexpr int kPer = 16;

__global__ void __launch_bounds__(kBlock) k_ub_atomics(float* __restrict__ buf, uint32_t n_buf,
                                                       int pattern, uint64_t n_ops) {
  const uint64_t threads = (uint64_t)gridDim.x * kBlock;
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t n_seg = n_buf / 16u;
#pragma unroll 4
  for (int k = 0; k < kPer; ++k) {
    const uint64_t i = (uint64_t)k * threads + t;
    if (i >= n_ops) return;
    uint32_t idx;
    switch (pattern) {
      case JSO_UB_RANDOM:
        idx = mix32(i) % n_buf;
        break;
      case JSO_UB_LINES:  // 16 neighbouring lanes share one 64-byte segment
        idx = (mix32(i >> 4) % n_seg) * 16u + (uint32_t)(i & 15u);
        break;
      case JSO_UB_16:
        idx = (uint32_t)(i & 15u);
        break;
      case JSO_UB_ROWS:  // 4 neighbouring lanes share one 16-byte row
        idx = (mix32(i >> 2) % (n_buf / 4u)) * 4u + (uint32_t)(i & 3u);
        break;
      default:  // JSO_UB_SAME
        idx = 0;
        break;
    }
    unsafeAtomicAdd(buf + idx, 1.0f);
  }
}

// One single-thread block per launch, each adding 1 to the counter the last
// one wrote: a chain of dependent launches whose length in time is the
// launch-to-launch gap.
__global__ void k_ub_tick(uint32_t* counter) {
  if (threadIdx.x == 0) counter[0] += 1u;
}

}  // namespace

namespace jso {
hipStream_t ctx_stream(jso_ctx* c);  // api.hip
int ctx_device(jso_ctx* c);
}  // namespace jso

namespace {

template <class Launch>
int timed(jso_ctx* c, int reps, double* ms, Launch launch) {
  if (!c || reps < 1 || !ms) return JSO_E_INVALID;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(jso::ctx_device(c));
  const hipStream_t st = jso::ctx_stream(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = JSO_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = JSO_E_HIP;
  } else {
    launch(st);  // warm-up
    float t = 0.0f;
    if (hipEventRecord(e0, st) != hipSuccess) rc = JSO_E_HIP;
    for (int r = 0; r < reps && rc == JSO_OK; ++r) launch(st);
    if (rc == JSO_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = JSO_E_HIP;
    *ms = (double)t / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}

unsigned grid_for(size_t work) {
  const size_t g = (work + kBlock - 1) / kBlock;
  return (unsigned)(g < 65536 ? (g ? g : 1) : 65536);
}

}  // namespace

extern "C" {

int jso_ub_copy(jso_ctx* c, void* dst, const void* src, size_t bytes, int reps, double* ms) {
  if (!dst || !src || bytes == 0 || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16)
    return JSO_E_INVALID;
  const size_t n = bytes / 16;
  return timed(c, reps, ms, [&](hipStream_t st) {
    hipLaunchKernelGGL(k_ub_copy, dim3(grid_for(n)), dim3(kBlock), 0, st,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  });
}

int jso_ub_atomics(jso_ctx* c, float* buf, size_t n_buf, int pattern, size_t n_ops, int reps,
                   double* ms) {
  if (!buf || n_buf < 16 || n_buf > 0xFFFFFFFFull || n_ops == 0) return JSO_E_INVALID;
  if (pattern < JSO_UB_RANDOM || pattern > JSO_UB_ROWS) return JSO_E_INVALID;
  const size_t threads = (n_ops + kPer - 1) / kPer;
  const size_t nb = (threads + kBlock - 1) / kBlock;  // covers n_ops: nb * kBlock * kPer >= n_ops
  if (nb > 0x7FFFFFFFu) return JSO_E_INVALID;
  const unsigned blocks = (unsigned)nb;
  return timed(c, reps, ms, [&](hipStream_t st) {
    hipLaunchKernelGGL(k_ub_atomics, dim3(blocks), dim3(kBlock), 0, st, buf, (uint32_t)n_buf,
                       pattern, (uint64_t)n_ops);
  });
}

int jso_ub_launch(jso_ctx* c, uint32_t* counter, int n_kernels, int use_graph, int reps,
                  double* ms) {
  if (!c || !counter || n_kernels < 1 || n_kernels > 4096) return JSO_E_INVALID;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(jso::ctx_device(c));
  const hipStream_t st = jso::ctx_stream(c);
  auto chain = [&](hipStream_t s) {
    for (int k = 0; k < n_kernels; ++k)
      hipLaunchKernelGGL(k_ub_tick, dim3(1), dim3(64), 0, s, counter);
  };
  int rc = JSO_OK;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (use_graph) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      rc = JSO_E_HIP;
    } else {
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = JSO_E_HIP;
      } else {
        chain(cs);
        if (hipStreamEndCapture(cs, &g) != hipSuccess ||
            hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
          rc = JSO_E_HIP;
      }
      (void)hipStreamDestroy(cs);
    }
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc == JSO_OK)
    rc = timed(c, reps, ms, [&](hipStream_t s) {
      if (use_graph) (void)hipGraphLaunch(ge, s);
      else chain(s);
    });
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  return rc;
}

}  // extern "C"

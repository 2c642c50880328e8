// Streaming kernels that measure the HBM ceiling the leapfrog kernels are
// judged against: a copy (read + write), a read-only pass and a write-only
// fill, each with 16-byte accesses by consecutive lanes (one 1 KiB segment
// per wave access), several accesses in flight per lane, grid-stride over
// the buffer, non-temporal stores.  Instrumentation only: no step of the
// method uses them.
#include <hip/hip_runtime.h>

#include <string>

#include "fit.h"

namespace fit {
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
}  // namespace fit

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;   // 16-byte accesses in flight per lane

using V4 = float __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_stream_copy(V4* __restrict__ dst,
                                                          const V4* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; base < n;
       base += stride) {
    V4 v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

// Read-only pass: every lane folds its values into one float; one store per
// lane at the end keeps the loads alive (sink: gridDim * kThreads floats).
__global__ __launch_bounds__(kThreads) void k_stream_read(const V4* __restrict__ src, int64_t n,
                                                          float* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * kThreads * kUnroll;
  float acc = 0.f;
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; base < n;
       base += stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < n) {
        const V4 v = __builtin_nontemporal_load(src + i);
        acc += (v.x + v.y) + (v.z + v.w);
      }
    }
  }
  sink[(int64_t)blockIdx.x * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_stream_fill(V4* __restrict__ dst, int64_t n,
                                                          float value) {
  const int64_t stride = (int64_t)gridDim.x * kThreads * kUnroll;
  const V4 v = {value, value, value, value};
  for (int64_t base = (int64_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; base < n;
       base += stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kThreads;
      if (i < n) __builtin_nontemporal_store(v, dst + i);
    }
  }
}

}  // namespace

using namespace fit;

extern "C" {

int fit_stream_probe(int mode, void* dst, const void* src, int64_t bytes, int blocks,
                     void* stream) {
  if (mode < 0 || mode > 2) return fail(FIT_E_INVALID, "mode must be 0 (copy), 1 (read), 2 (fill)");
  if (bytes <= 0 || bytes % 16 != 0) return fail(FIT_E_INVALID, "bytes must be a positive multiple of 16");
  if (blocks < 1 || blocks > (1 << 20)) return fail(FIT_E_INVALID, "blocks must be in [1, 2^20]");
  if (!dst || (mode != 2 && !src)) return fail(FIT_E_INVALID, "null buffer");
  if ((dst && reinterpret_cast<uintptr_t>(dst) % 16) || (src && reinterpret_cast<uintptr_t>(src) % 16))
    return fail(FIT_E_INVALID, "buffers must be aligned to 16 bytes");
  const int64_t n = bytes / 16;
  if (mode == 0) {
    const char* s = static_cast<const char*>(src);
    const char* d = static_cast<const char*>(dst);
    if (s < d + bytes && d < s + bytes) return fail(FIT_E_INVALID, "source and destination overlap");
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grd((unsigned)blocks), blk(kThreads);
  if (mode == 0)
    hipLaunchKernelGGL(k_stream_copy, grd, blk, 0, s, static_cast<V4*>(dst),
                       static_cast<const V4*>(src), n);
  else if (mode == 1)
    hipLaunchKernelGGL(k_stream_read, grd, blk, 0, s, static_cast<const V4*>(src), n,
                       static_cast<float*>(dst));
  else
    hipLaunchKernelGGL(k_stream_fill, grd, blk, 0, s, static_cast<V4*>(dst), n, 1.0f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "stream probe launch");
  return FIT_OK;
}

}  // extern "C"

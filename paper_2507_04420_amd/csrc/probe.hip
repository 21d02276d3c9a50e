// Measurement: the rates of independent random 4-byte reads and of random
// 4-byte atomic adds this GPU sustains, the two ceilings that bind a pass of
// random state accesses. A plain kernel: every thread takes UNROLL indices
// from a counter-based hash (SplitMix64 of the index, Steele, Lea and Flood,
// OOPSLA 2014) and reads (or atomically adds to) those words, so nothing but
// the random accesses themselves goes to memory.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>

#include "internal.h"
#include "mm.h"

using mmi::fail;
#define HIP_TRY MMI_HIP_TRY

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

constexpr int kUnroll = 4;

__global__ void probe_reads(const uint32_t* __restrict__ data, uint64_t words, int64_t ops,
                            uint32_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kUnroll;
  uint32_t acc = 0;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kUnroll; i < ops; i += stride) {
    uint32_t v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      v[u] = i + u < ops ? data[mix64((uint64_t)(i + u)) % words] : 0u;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc += v[u];
  }
  if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; never true for the zero-filled array
}

__global__ void probe_atomics(uint32_t* __restrict__ data, uint64_t words, int64_t ops) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kUnroll;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kUnroll; i < ops; i += stride) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (i + u < ops)
        __hip_atomic_fetch_add(data + mix64((uint64_t)(i + u) ^ 0x5bd1e995ull) % words, 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

extern "C" {

mm_status mm_probe_ceilings(int64_t array_bytes, int64_t ops, void* stream, double* reads_per_s,
                            double* atomics_per_s) {
  if (array_bytes < 4096 || ops < 1 || !reads_per_s || !atomics_per_s)
    return fail(MM_ERR_INVALID_ARG, "mm_probe_ceilings: array_bytes >= 4096, ops >= 1, "
                "non-null outputs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t words = (uint64_t)array_bytes / 4;
  uint32_t* data = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&data), words * 4 + 256, s));
  hipError_t e = hipMemsetAsync(data, 0, words * 4 + 256, s);
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  const int blocks = 8192, threads = 256;
  float ms[2] = {0, 0};
  for (int which = 0; which < 2 && e == hipSuccess; ++which) {
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // a warm-up, then two timed
      if (rep > 0) e = hipEventRecord(a, s);
      if (e != hipSuccess) break;
      if (which == 0)
        hipLaunchKernelGGL(probe_reads, dim3(blocks), dim3(threads), 0, s, data, words, ops,
                           data + words);
      else
        hipLaunchKernelGGL(probe_atomics, dim3(blocks), dim3(threads), 0, s, data, words, ops);
      e = hipGetLastError();
      if (e == hipSuccess && rep > 0) e = hipEventRecord(b, s);
      if (e == hipSuccess && rep > 0) e = hipEventSynchronize(b);
      float t = 0;
      if (e == hipSuccess && rep > 0) e = hipEventElapsedTime(&t, a, b);
      if (rep > 0) ms[which] += t / 2;
    }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFreeAsync(data, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(MM_ERR_HIP, "mm_probe_ceilings: %s", hipGetErrorString(e));
  *reads_per_s = (double)ops / (ms[0] / 1e3);
  *atomics_per_s = (double)ops / (ms[1] / 1e3);
  return MM_OK;
}

}  // extern "C"

// Matched-pair list output (the `matches` array that Algorithm 1 fills and returns).
//
// The sweep records its result in the mate array; this pass turns a mate
// array into the list of matched pairs (u, v), u < v, each pair once. Every
// wavefront compacts 64 vertices per step with a ballot and reserves its
// slots with one atomic add on a shared cursor, the GPU form of the paper's
// per-thread buffers taken from one shared block. The order of the pairs is
// not specified.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "mm.h"

using mmi::fail;
#define HIP_TRY MMI_HIP_TRY

namespace {

constexpr size_t kPairsCursorOffset = mmi::kCheckOffset + 64;

__global__ void pairs_kernel(const int32_t* __restrict__ mate, int64_t n, int32_t* __restrict__ out,
                             int64_t cap, unsigned long long* cursor) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += waves * 64) {
    const int64_t x = base + lane;
    const int64_t y = x < n ? (int64_t)mate[x] : -1;
    const bool lead = y > x && y < n;  // the lower end of a pair writes it
    const uint64_t bm = __ballot(lead);
    if (!bm) continue;
    unsigned long long start = 0;
    if (lane == 0)
      start = __hip_atomic_fetch_add(cursor, (unsigned long long)__popcll(bm), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    start = (unsigned long long)__shfl((long long)start, 0, 64);
    if (lead) {
      const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
      const unsigned long long slot = start + r;
      if ((int64_t)slot < cap) {
        out[2 * slot] = (int32_t)x;
        out[2 * slot + 1] = (int32_t)y;
      }
    }
  }
}

}  // namespace

extern "C" {

mm_status mm_pairs(mm_handle h, void* stream, const int32_t* match, int32_t* pairs, int64_t cap,
                   int64_t* count) {
  if (!h || !count) return fail(MM_ERR_INVALID_ARG, "null argument");
  const int64_t n = mmi::handle_n(h);
  if (!match && n > 0) return fail(MM_ERR_INVALID_ARG, "match is null");
  if (cap < 0 || (!pairs && cap > 0)) return fail(MM_ERR_INVALID_ARG, "bad pairs buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* cursor = reinterpret_cast<unsigned long long*>(mmi::handle_ws(h) + kPairsCursorOffset);
  HIP_TRY(hipMemsetAsync(cursor, 0, sizeof(unsigned long long), s));
  if (n > 0) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, match, n, pairs, cap,
                       cursor);
    HIP_TRY(hipGetLastError());
  }
  unsigned long long c = 0;
  HIP_TRY(hipMemcpyAsync(&c, cursor, sizeof(c), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *count = (int64_t)c;
  if ((int64_t)c > cap)
    return fail(MM_ERR_OUT_OF_MEMORY, "%lld pairs, buffer holds %lld (only the first %lld written)",
                (long long)c, (long long)cap, (long long)cap);
  return MM_OK;
}

}  // extern "C"

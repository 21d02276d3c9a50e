// Device-side verification of a mate array (the product's own check; the
// test suite pins it against the independent CPU checker).
//
// Counts, per class, the ways a mate array can fail to be a maximal matching
// of the graph (Section II-B): a mate out of range, a vertex matched to
// itself, an asymmetric pair, a pair that is not an edge, and an edge whose
// two endpoints are both unmatched.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "batch.h"
#include "internal.h"
#include "mm.h"

using mmi::fail;
#define HIP_TRY MMI_HIP_TRY

namespace {

template <typename OffT>
__device__ __forceinline__ bool has_entry(const OffT* off, const int32_t* nbr, int64_t x, int64_t y) {
  for (int64_t i = (int64_t)off[x]; i < (int64_t)off[x + 1]; ++i)
    if (nbr[i] == y) return true;
  return false;
}

__device__ __forceinline__ void flush_counts(unsigned long long c[6], unsigned long long* out) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    unsigned long long s = c[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0 && s)
      __hip_atomic_fetch_add(out + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One vertex x of a graph whose arrays are based at its first vertex.
template <typename OffT>
__device__ __forceinline__ void check_vertex(const OffT* off, const int32_t* nbr, int64_t n,
                                             const int32_t* mate, int64_t x,
                                             unsigned long long c[6]) {
  const int64_t y = mate[x];
  if (y < -1 || y >= n) {
    ++c[0];
  } else if (y == x) {
    ++c[1];
    ++c[5];
  } else if (y >= 0) {
    ++c[5];
    if ((int64_t)mate[y] != x) ++c[2];
    if (!has_entry(off, nbr, x, y) && !has_entry(off, nbr, y, x)) ++c[3];
  } else {
    // x unmatched: every other endpoint of its entries must be matched
    for (int64_t i = (int64_t)off[x]; i < (int64_t)off[x + 1]; ++i) {
      const int64_t z = nbr[i];
      if (z >= 0 && z < n && z != x && mate[z] == -1) ++c[4];
    }
  }
}

template <typename OffT>
__global__ void check_kernel(const OffT* __restrict__ off, const int32_t* __restrict__ nbr,
                             int64_t n, const int32_t* __restrict__ mate,
                             unsigned long long* out) {
  unsigned long long c[6] = {0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    check_vertex(off, nbr, n, mate, x, c);
  flush_counts(c, out);
}

__global__ void check_batch_kernel(const mmb::GraphDesc* __restrict__ descs,
                                   const int64_t* __restrict__ vtx_off, int32_t num_graphs,
                                   const int32_t* __restrict__ mate, unsigned long long* out) {
  unsigned long long c[6] = {0, 0, 0, 0, 0, 0};
  const int64_t N = vtx_off[num_graphs];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    int lo = 0, hi = num_graphs;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (vtx_off[mid] <= v) lo = mid; else hi = mid;
    }
    const mmb::GraphDesc d = descs[lo];
    check_vertex(d.off, d.nbr, d.n, mate + d.v0, v - d.v0, c);
  }
  flush_counts(c, out);
}

mm_status finish(unsigned long long* dev, hipStream_t s, int64_t* counts) {
  unsigned long long h[6];
  HIP_TRY(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < 6; ++k) counts[k] = (int64_t)h[k];
  return MM_OK;
}

int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

}  // namespace

extern "C" {

mm_status mm_check(mm_handle h, void* stream, const int32_t* match, int64_t* counts) {
  if (!h || !counts || (!match && mmi::handle_n(h) > 0))
    return fail(MM_ERR_INVALID_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long* dev = reinterpret_cast<unsigned long long*>(mmi::handle_ws(h) + mmi::kCheckOffset);
  HIP_TRY(hipMemsetAsync(dev, 0, 6 * sizeof(unsigned long long), s));
  const int64_t n = mmi::handle_n(h);
  if (n > 0) {
    if (mmi::handle_off64(h))
      hipLaunchKernelGGL((check_kernel<int64_t>), dim3(blocks_for(n)), dim3(256), 0, s,
                         static_cast<const int64_t*>(mmi::handle_off(h)), mmi::handle_nbr(h), n,
                         match, dev);
    else
      hipLaunchKernelGGL((check_kernel<int32_t>), dim3(blocks_for(n)), dim3(256), 0, s,
                         static_cast<const int32_t*>(mmi::handle_off(h)), mmi::handle_nbr(h), n,
                         match, dev);
    HIP_TRY(hipGetLastError());
  }
  return finish(dev, s, counts);
}

mm_status mm_batch_check(mm_batch_handle b, void* stream, const int32_t* match, int64_t* counts) {
  if (!b || !counts) return fail(MM_ERR_INVALID_ARG, "null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mmb::BatchInfo info = mmb::batch_info(b);
  if (!match && info.N > 0) return fail(MM_ERR_INVALID_ARG, "match is null");
  unsigned long long* dev = reinterpret_cast<unsigned long long*>(info.ws + mmi::kCheckOffset);
  HIP_TRY(hipMemsetAsync(dev, 0, 6 * sizeof(unsigned long long), s));
  if (info.N > 0) {
    hipLaunchKernelGGL(check_batch_kernel, dim3(blocks_for(info.N)), dim3(256), 0, s, info.descs,
                       info.vtx_off, info.G, match, dev);
    HIP_TRY(hipGetLastError());
  }
  return finish(dev, s, counts);
}

}  // extern "C"

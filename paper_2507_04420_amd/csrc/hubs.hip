// Create-time table of the hub tier: every list longer than hub_degree is cut
// into pieces of hub_chunk entries; the chunk pass of a sweep gives each
// piece to its own lane, so a long scan no longer rests on one lane. (The
// paper's blocks have about equal numbers of edges, Section IV-C; this is the
// same balance for the few lists that a block of vertices cannot even out.)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include <rocprim/device/device_scan.hpp>

#include "internal.h"
#include "sweep.h"

namespace {

template <typename OffT>
__global__ void chunk_counts_kernel(const OffT* __restrict__ off, int64_t n, int64_t hub_degree,
                                    int64_t chunk, int64_t* __restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
    if (v == n) {
      counts[n] = 0;
      continue;
    }
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
    counts[v] = d > hub_degree ? (d + chunk - 1) / chunk : 0;
  }
}

template <typename OffT>
__global__ void chunk_fill_kernel(const OffT* __restrict__ off, int64_t n, int64_t hub_degree,
                                  int64_t chunk, const int64_t* __restrict__ first,
                                  mmk::HubChunk* __restrict__ table) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
    if (e - b <= hub_degree) continue;
    int64_t k = first[v];
    for (int64_t p = b; p < e; p += chunk, ++k) {
      mmk::HubChunk c;
      c.b = p;
      c.e = p + chunk < e ? p + chunk : e;
      c.x = (int32_t)v;
      c.pad = 0;
      table[k] = c;
    }
  }
}

int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (int)b;
}

template <typename OffT>
hipError_t build_typed(const OffT* off, int64_t n, int64_t hub_degree, int64_t chunk,
                       mmk::HubChunk** table, int64_t* count, hipStream_t s) {
  int64_t* counts = nullptr;
  int64_t* first = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, tmp_bytes, counts, first, (int64_t)0,
                                         (size_t)(n + 1), rocprim::plus<int64_t>(), s);
  if (e == hipSuccess) e = hipMalloc(&counts, sizeof(int64_t) * (size_t)(n + 1));
  if (e == hipSuccess) e = hipMalloc(&first, sizeof(int64_t) * (size_t)(n + 1));
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((chunk_counts_kernel<OffT>), dim3(blocks_for(n + 1)), dim3(256), 0, s, off, n,
                       hub_degree, chunk, counts);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(tmp, tmp_bytes, counts, first, (int64_t)0, (size_t)(n + 1),
                                rocprim::plus<int64_t>(), s);
  int64_t total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, first + n, sizeof(total), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *table = nullptr;
  *count = 0;
  if (e == hipSuccess && total > 0) {
    e = hipMalloc(table, sizeof(mmk::HubChunk) * (size_t)total);
    if (e == hipSuccess) {
      hipLaunchKernelGGL((chunk_fill_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, n,
                         hub_degree, chunk, first, *table);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      *count = total;
    } else if (*table) {
      hipFree(*table);
      *table = nullptr;
    }
  }
  hipFree(counts);
  hipFree(first);
  hipFree(tmp);
  return e;
}

}  // namespace

namespace mmi {

hipError_t build_hub_chunks(const void* off, int off64, int64_t n, int64_t hub_degree,
                            int64_t chunk, mmk::HubChunk** table, int64_t* count, hipStream_t s) {
  *table = nullptr;
  *count = 0;
  if (n == 0 || hub_degree <= 0) return hipSuccess;
  if (off64)
    return build_typed(static_cast<const int64_t*>(off), n, hub_degree, chunk, table, count, s);
  return build_typed(static_cast<const int32_t*>(off), n, hub_degree, chunk, table, count, s);
}

}  // namespace mmi

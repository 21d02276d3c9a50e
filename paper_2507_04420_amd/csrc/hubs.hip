// Create-time table of the hub tier: every list longer than hub_degree is cut
// into pieces of hub_chunk entries; the chunk pass of a sweep gives each
// piece to its own lane, so a long scan no longer rests on one lane. (The
// paper's blocks have about equal numbers of edges, Section IV-C; this is the
// same balance for the few lists that a block of vertices cannot even out.)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include <rocprim/device/device_scan.hpp>

#include "batch.h"
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

// Batch form: global vertex v belongs to the graph found by binary search over
// the vertex-offset table; graphs swept whole by one wavefront get no pieces.
__device__ __forceinline__ int graph_of(const int64_t* vtx_off, int32_t G, int64_t v) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (vtx_off[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void batch_counts_kernel(const mmb::GraphDesc* __restrict__ descs,
                                    const int64_t* __restrict__ vtx_off, int32_t G, int64_t N,
                                    int64_t hub_degree, int64_t chunk, int64_t* __restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= N; v += stride) {
    if (v == N) {
      counts[N] = 0;
      continue;
    }
    const int g = graph_of(vtx_off, G, v);
    const mmb::GraphDesc d = descs[g];
    const int64_t x = v - d.v0;
    const int64_t deg = d.off[x + 1] - d.off[x];
    counts[v] = (!(d.flags & mmb::kWholeGraph) && deg > hub_degree) ? (deg + chunk - 1) / chunk : 0;
  }
}

__global__ void batch_fill_kernel(const mmb::GraphDesc* __restrict__ descs,
                                  const int64_t* __restrict__ vtx_off, int32_t G, int64_t N,
                                  int64_t chunk, const int64_t* __restrict__ counts,
                                  const int64_t* __restrict__ first, mmk::HubChunk* __restrict__ table) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    if (counts[v] == 0) continue;
    const int g = graph_of(vtx_off, G, v);
    const mmb::GraphDesc d = descs[g];
    const int64_t x = v - d.v0;
    const int64_t b = d.off[x], e = d.off[x + 1];
    int64_t k = first[v];
    for (int64_t p = b; p < e; p += chunk, ++k) {
      mmk::HubChunk c;
      c.b = p;
      c.e = p + chunk < e ? p + chunk : e;
      c.x = (int32_t)x;
      c.pad = 0;
      table[k] = c;
    }
  }
}

// first[vtx_off[g]] for every g: where each graph's pieces start.
__global__ void gather_first_kernel(const int64_t* __restrict__ first,
                                    const int64_t* __restrict__ vtx_off, int32_t G,
                                    int64_t* __restrict__ out) {
  const int g = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (g <= G) out[g] = first[vtx_off[g]];
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

namespace mmb {

hipError_t build_batch_hubs(const GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                            int64_t hub_degree, int64_t chunk, mmk::HubChunk** table,
                            int64_t* count, int64_t* first_host, hipStream_t s) {
  *table = nullptr;
  *count = 0;
  for (int32_t g = 0; g <= G; ++g) first_host[g] = 0;
  if (N == 0 || G == 0 || hub_degree <= 0) return hipSuccess;
  int64_t* counts = nullptr;
  int64_t* first = nullptr;
  int64_t* gfirst = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  hipError_t e = rocprim::exclusive_scan(nullptr, tmp_bytes, counts, first, (int64_t)0,
                                         (size_t)(N + 1), rocprim::plus<int64_t>(), s);
  if (e == hipSuccess) e = hipMalloc(&counts, sizeof(int64_t) * (size_t)(N + 1));
  if (e == hipSuccess) e = hipMalloc(&first, sizeof(int64_t) * (size_t)(N + 1));
  if (e == hipSuccess) e = hipMalloc(&gfirst, sizeof(int64_t) * (size_t)(G + 1));
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(batch_counts_kernel, dim3(blocks_for(N + 1)), dim3(256), 0, s, descs_dev,
                       vtx_dev, G, N, hub_degree, chunk, counts);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(tmp, tmp_bytes, counts, first, (int64_t)0, (size_t)(N + 1),
                                rocprim::plus<int64_t>(), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gather_first_kernel, dim3((G + 1 + 255) / 256), dim3(256), 0, s, first,
                       vtx_dev, G, gfirst);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(first_host, gfirst, sizeof(int64_t) * (size_t)(G + 1), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const int64_t total = e == hipSuccess ? first_host[G] : 0;
  if (e == hipSuccess && total > 0) {
    e = hipMalloc(table, sizeof(mmk::HubChunk) * (size_t)total);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(batch_fill_kernel, dim3(blocks_for(N)), dim3(256), 0, s, descs_dev, vtx_dev,
                         G, N, chunk, counts, first, *table);
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
  if (e != hipSuccess)
    for (int32_t g = 0; g <= G; ++g) first_host[g] = 0;
  hipFree(counts);
  hipFree(first);
  hipFree(gfirst);
  hipFree(tmp);
  return e;
}

}  // namespace mmb

// Create-time table of the hub tier: every list longer than hub_degree is cut
// into pieces of hub_chunk entries; the chunk pass of a sweep gives each
// piece to its own lane, so a long scan no longer rests on one lane. (The
// paper's blocks have about equal numbers of edges, Section IV-C; this is the
// same balance for the few lists that a block of vertices cannot even out.)
//
// The build costs one counting kernel and one wait when no list is long
// enough (the usual case for small graphs); only then does it allocate, once,
// stream-ordered, so that a create or destroy never waits for the whole
// device (a serving loop creates and destroys handles while other launches
// run). Each list reserves its run of pieces with one atomic, so the order of
// lists in the table varies from build to build; the pieces of one list stay
// adjacent.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch.h"
#include "internal.h"
#include "sweep.h"

namespace {

using ull = unsigned long long;

int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 16384) b = 16384;
  return (int)b;
}

__device__ __forceinline__ void put_pieces(mmk::HubChunk* table, int64_t k, int64_t b, int64_t e,
                                           int64_t chunk, int32_t x) {
  for (int64_t p = b; p < e; p += chunk, ++k) {
    mmk::HubChunk c;
    c.b = p;
    c.e = p + chunk < e ? p + chunk : e;
    c.x = x;
    c.pad = 0;
    table[k] = c;
  }
}

// Pass 1: pieces of every long list, summed into *total.
template <typename OffT>
__global__ void count_kernel(const OffT* __restrict__ off, int64_t n, int64_t hub_degree,
                             int64_t chunk, ull* total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
    if (d > hub_degree)
      __hip_atomic_fetch_add(total, (ull)((d + chunk - 1) / chunk), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Pass 2: each long list takes its run of slots from *cursor (zero on entry).
template <typename OffT>
__global__ void fill_kernel(const OffT* __restrict__ off, int64_t n, int64_t hub_degree,
                            int64_t chunk, ull* cursor, mmk::HubChunk* __restrict__ table) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t b = (int64_t)off[v], e = (int64_t)off[v + 1];
    if (e - b <= hub_degree) continue;
    const int64_t k = (int64_t)__hip_atomic_fetch_add(cursor, (ull)((e - b + chunk - 1) / chunk),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    put_pieces(table, k, b, e, chunk, (int32_t)v);
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

// Pieces of vertex v of a batch (0 unless its list is long and its graph is
// not swept whole); *g and *x receive its graph and local id.
__device__ __forceinline__ int64_t batch_pieces(const mmb::GraphDesc* descs,
                                                const int64_t* vtx_off, int32_t G, int64_t v,
                                                int64_t hub_degree, int64_t chunk, int* g,
                                                int64_t* x, int64_t* b, int64_t* e) {
  *g = graph_of(vtx_off, G, v);
  const mmb::GraphDesc& d = descs[*g];
  if (d.flags & mmb::kWholeGraph) return 0;
  *x = v - d.v0;
  *b = d.off[*x];
  *e = d.off[*x + 1];
  return *e - *b > hub_degree ? (*e - *b + chunk - 1) / chunk : 0;
}

// Pass 1: pieces per graph (into descs[g].pieces) and in all (*total).
__global__ void batch_count_kernel(mmb::GraphDesc* descs, const int64_t* __restrict__ vtx_off,
                                   int32_t G, int64_t N, int64_t hub_degree, int64_t chunk,
                                   ull* total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    int g;
    int64_t x, b, e;
    const int64_t k = batch_pieces(descs, vtx_off, G, v, hub_degree, chunk, &g, &x, &b, &e);
    if (k == 0) continue;
    __hip_atomic_fetch_add(reinterpret_cast<ull*>(&descs[g].pieces), (ull)k, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(total, (ull)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Pass 2: descs[g].pieces holds where graph g's pieces start; each long list
// takes its run from there (the field ends at the start of graph g+1).
__global__ void batch_fill_kernel(mmb::GraphDesc* descs, const int64_t* __restrict__ vtx_off,
                                  int32_t G, int64_t N, int64_t hub_degree, int64_t chunk,
                                  mmk::HubChunk* __restrict__ table) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    int g;
    int64_t x, b, e;
    const int64_t k = batch_pieces(descs, vtx_off, G, v, hub_degree, chunk, &g, &x, &b, &e);
    if (k == 0) continue;
    const int64_t at = (int64_t)__hip_atomic_fetch_add(
        reinterpret_cast<ull*>(&descs[g].pieces), (ull)k, __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT);
    put_pieces(table, at, b, e, chunk, (int32_t)x);
  }
}

// Marks the graphs that are not meshes. Once a graph is marked, its other
// vertices see the mark with a plain load and write nothing.
__global__ void find_meshes_kernel(mmb::GraphDesc* descs, const int64_t* __restrict__ vtx_off,
                                   int32_t G, int64_t N) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    const int g = graph_of(vtx_off, G, v);
    mmb::GraphDesc& d = descs[g];
    const int64_t x = v - d.v0;
    if (d.off[x + 1] - d.off[x] > mmb::kMeshDegree &&
        __hip_atomic_load(&d.not_mesh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      __hip_atomic_store(&d.not_mesh, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename OffT>
hipError_t build_typed(const OffT* off, int64_t n, int64_t hub_degree, int64_t chunk, uint8_t* ctrl,
                       mmk::HubChunk** table, int64_t* count, hipStream_t s) {
  ull* total = reinterpret_cast<ull*>(ctrl + mmi::kHubOffset);
  ull* cursor = total + 1;
  hipError_t e = hipMemsetAsync(total, 0, 2 * sizeof(ull), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((count_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, n, hub_degree,
                     chunk, total);
  e = hipGetLastError();
  ull host_total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&host_total, total, sizeof(ull), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || host_total == 0) return e;
  e = hipMallocAsync(reinterpret_cast<void**>(table), sizeof(mmk::HubChunk) * (size_t)host_total, s);
  if (e != hipSuccess) {
    *table = nullptr;
    return e;
  }
  hipLaunchKernelGGL((fill_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, n, hub_degree,
                     chunk, cursor, *table);
  e = hipGetLastError();
  if (e != hipSuccess) {
    hipFreeAsync(*table, s);
    *table = nullptr;
    return e;
  }
  *count = (int64_t)host_total;
  return hipSuccess;
}

}  // namespace

namespace mmi {

hipError_t build_hub_chunks(const void* off, int off64, int64_t n, int64_t hub_degree,
                            int64_t chunk, uint8_t* ctrl, mmk::HubChunk** table, int64_t* count,
                            hipStream_t s) {
  *table = nullptr;
  *count = 0;
  if (n == 0 || hub_degree <= 0) return hipSuccess;
  if (off64)
    return build_typed(static_cast<const int64_t*>(off), n, hub_degree, chunk, ctrl, table, count, s);
  return build_typed(static_cast<const int32_t*>(off), n, hub_degree, chunk, ctrl, table, count, s);
}

hipError_t fill_hub_chunks(const void* off, int off64, int64_t n, int64_t hub_degree, int64_t chunk,
                           unsigned long long* cursor, mmk::HubChunk* table, hipStream_t s) {
  if (n == 0 || hub_degree <= 0) return hipSuccess;
  if (off64)
    hipLaunchKernelGGL((fill_kernel<int64_t>), dim3(blocks_for(n)), dim3(256), 0, s,
                       static_cast<const int64_t*>(off), n, hub_degree, chunk, cursor, table);
  else
    hipLaunchKernelGGL((fill_kernel<int32_t>), dim3(blocks_for(n)), dim3(256), 0, s,
                       static_cast<const int32_t*>(off), n, hub_degree, chunk, cursor, table);
  return hipGetLastError();
}

void free_owned(void* p) {
  // stream-ordered on the null stream: no wait for the whole device; the
  // owner first makes the null stream wait for the last pass that reads the
  // memory (an event recorded on that pass's stream)
  if (p) hipFreeAsync(p, nullptr);
}

}  // namespace mmi

namespace mmb {

hipError_t count_batch_hubs(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                            int64_t hub_degree, int64_t chunk, uint8_t* ctrl, hipStream_t s) {
  ull* total = reinterpret_cast<ull*>(ctrl + mmi::kHubOffset);
  hipError_t e = hipMemsetAsync(total, 0, sizeof(ull), s);
  if (e != hipSuccess || N == 0 || G == 0 || hub_degree <= 0) return e;
  hipLaunchKernelGGL(batch_count_kernel, dim3(blocks_for(N)), dim3(256), 0, s, descs_dev, vtx_dev,
                     G, N, hub_degree, chunk, total);
  return hipGetLastError();
}

hipError_t batch_find_meshes(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                             hipStream_t s) {
  if (N == 0 || G == 0) return hipSuccess;
  hipLaunchKernelGGL(find_meshes_kernel, dim3(blocks_for(N)), dim3(256), 0, s, descs_dev, vtx_dev,
                     G, N);
  return hipGetLastError();
}

hipError_t fill_batch_hubs(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                           int64_t hub_degree, int64_t chunk, mmk::HubChunk* table, hipStream_t s) {
  hipLaunchKernelGGL(batch_fill_kernel, dim3(blocks_for(N)), dim3(256), 0, s, descs_dev, vtx_dev, G,
                     N, hub_degree, chunk, table);
  return hipGetLastError();
}

}  // namespace mmb

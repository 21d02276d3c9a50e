// Create-time relabelling of a graph (tuning.relabel).
//
// Mode 1, by degree: new ids list the vertices by ascending log2-degree
// bucket (isolated vertices first), keeping the given order inside a bucket.
// Two effects:
//   * the sweep visits low-degree sources first, which shortens the scans
//     (a low-degree source reaches a free neighbour early, and hubs are
//     usually matched as neighbours before their own turn comes);
//   * the high-degree vertices, whose states most scans read, get the
//     highest ids, so their status words and hint bits share few cache lines
//     and stay in L2.
// Lists of up to 64 entries are sorted by new id (low-degree neighbours
// first).
//
// Mode 2, hot vertices last: isolated vertices first, then every vertex of
// at most `hot` entries in the given order, then the others (the hot ones),
// also in the given order; lists keep their given order. The sweep then
// visits sources almost as given, but the states of the hot vertices, which
// most scans of a skewed graph read, sit together at the top of the state
// array: a few hundred thousand vertices in a few MB, which the L2 keeps,
// where in the given ids each of them would hold a cache line of its own.
//
// The relabelled CSR (int64 offsets, neighbour lists with ids mapped) and the
// map from new to given ids live in the workspace; the sweep writes its
// output in the given ids. Temporary buffers of the sort are allocated and
// freed here (create time only).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "internal.h"

namespace {

__device__ __forceinline__ uint32_t bucket_of(int64_t d) {
  return d <= 0 ? 0u : 64u - (uint32_t)__clzll((unsigned long long)d);  // 1 + floor(log2 d)
}

// Sort keys: the log2-degree bucket (mode 1), or 0 isolated / 1 / 2 more than
// `hot` entries (mode 2).
template <typename OffT>
__global__ void degree_keys_kernel(const OffT* __restrict__ off, int64_t n, int mode, int64_t hot,
                                   uint32_t* __restrict__ keys) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v];
    keys[v] = mode == 1 ? bucket_of(d) : (d <= 0 ? 0u : (d > hot ? 2u : 1u));
  }
}

// inv[orig[v]] = v; rdeg[v] = degree of new vertex v; rdeg[n] = 0.
template <typename OffT>
__global__ void invert_kernel(const OffT* __restrict__ off, const int32_t* __restrict__ orig,
                              int64_t n, int32_t* __restrict__ inv, int64_t* __restrict__ rdeg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += stride) {
    if (v == n) {
      rdeg[n] = 0;
      continue;
    }
    const int64_t x = orig[v];
    inv[x] = (int32_t)v;
    rdeg[v] = (int64_t)off[x + 1] - (int64_t)off[x];
  }
}

// Number of isolated vertices: the sorted keys start with them.
__global__ void count_isolated_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                      unsigned long long* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (keys[v] == 0 && (v + 1 == n || keys[v + 1] != 0)) *out = (unsigned long long)(v + 1);
}

// Copies the lists. A wavefront takes 64 new vertices: each lane copies its
// own vertex's list when it has at most 64 entries, sorted by new id when
// `sort_short` (an insertion sort in LDS, element k of lane l at k * 64 + l
// so that the lanes use different banks); longer lists are then copied by the
// whole wavefront, one after the other, lanes spread over it, in their given
// order. Ascending new ids in the degree order put a list's low-degree
// neighbours first, and those are the ones still free when a low-degree
// source is swept: the sweep reads fewer ids.
template <typename OffT>
__global__ __launch_bounds__(256) void copy_lists_kernel(
    const OffT* __restrict__ off, const int32_t* __restrict__ nbr, const int32_t* __restrict__ orig,
    const int32_t* __restrict__ inv, const int64_t* __restrict__ roff, int32_t* __restrict__ rnbr,
    int64_t n, int sort_short) {
  __shared__ int32_t sort_s[4][64 * 64];
  int32_t* srt = sort_s[threadIdx.x >> 6];
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += waves * 64) {
    const int64_t v = base + lane;
    int64_t b = 0, e = 0, d = 0;
    if (v < n) {
      const int64_t x = orig[v];
      b = (int64_t)off[x];
      e = (int64_t)off[x + 1];
      d = roff[v] - b;
    }
    const bool longl = e - b > 64;
    if (!longl && !sort_short) {
      for (int64_t k = b; k < e; ++k) rnbr[d + k] = inv[nbr[k]];
    } else if (!longl) {
      const int len = (int)(e - b);
      for (int k = 0; k < len; ++k) {
        const int32_t key = inv[nbr[b + k]];
        int j = k - 1;
        while (j >= 0 && srt[j * 64 + lane] > key) {
          srt[(j + 1) * 64 + lane] = srt[j * 64 + lane];
          --j;
        }
        srt[(j + 1) * 64 + lane] = key;
      }
      for (int k = 0; k < len; ++k) rnbr[d + b + k] = srt[k * 64 + lane];
    }
    uint64_t lm = __ballot(longl);
    while (lm) {
      const int l = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t lb = __shfl(b, l, 64), le = __shfl(e, l, 64), ld = __shfl(d, l, 64);
      for (int64_t j = lb + lane; j < le; j += 64) rnbr[ld + j] = inv[nbr[j]];
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
hipError_t build_typed(const OffT* off, const int32_t* nbr, int64_t n, int mode, int64_t hot,
                       int64_t* roff, int32_t* rnbr, int32_t* orig, int64_t* n_isolated,
                       hipStream_t s) {
  // 7 key bits cover every bucket 0 .. 64 (mode 1); 2 bits the three groups
  const int key_bits = mode == 1 ? 7 : 2;
  uint32_t *keys = nullptr, *keys_sorted = nullptr;
  int32_t* inv = nullptr;
  int64_t* rdeg = nullptr;
  void* tmp = nullptr;
  unsigned long long* iso = nullptr;
  size_t tmp_bytes = 0, sort_bytes = 0, scan_bytes = 0;
  hipError_t e = hipSuccess;
  auto ids = rocprim::counting_iterator<int32_t>(0);
  e = rocprim::radix_sort_pairs(nullptr, sort_bytes, keys, keys_sorted, ids, orig, (size_t)n, 0,
                                key_bits, s);
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(nullptr, scan_bytes, rdeg, roff, (int64_t)0, (size_t)(n + 1),
                                rocprim::plus<int64_t>(), s);
  tmp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&keys),
                                          sizeof(uint32_t) * (size_t)n, s);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&keys_sorted),
                                          sizeof(uint32_t) * (size_t)n, s);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&inv),
                                          sizeof(int32_t) * (size_t)n, s);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&rdeg),
                                          sizeof(int64_t) * (size_t)(n + 1), s);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&tmp),
                                          tmp_bytes > 0 ? tmp_bytes : 1, s);
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&iso),
                                          sizeof(unsigned long long), s);
  if (e == hipSuccess) e = hipMemsetAsync(iso, 0, sizeof(unsigned long long), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((degree_keys_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, n,
                       mode, hot, keys);
    e = hipGetLastError();
  }
  // the sort is stable: the given order inside each key
  if (e == hipSuccess)
    e = rocprim::radix_sort_pairs(tmp, sort_bytes, keys, keys_sorted, ids, orig, (size_t)n, 0,
                                  key_bits, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((invert_kernel<OffT>), dim3(blocks_for(n + 1)), dim3(256), 0, s, off, orig, n,
                       inv, rdeg);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(tmp, scan_bytes, rdeg, roff, (int64_t)0, (size_t)(n + 1),
                                rocprim::plus<int64_t>(), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(count_isolated_kernel, dim3(blocks_for(n)), dim3(256), 0, s, keys_sorted, n, iso);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((copy_lists_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s,
                       off, nbr, orig, inv, roff, rnbr, n, mode == 1 ? 1 : 0);
    e = hipGetLastError();
  }
  unsigned long long h_iso = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h_iso, iso, sizeof(h_iso), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *n_isolated = (int64_t)h_iso;
  if (keys) hipFreeAsync(keys, s);
  if (keys_sorted) hipFreeAsync(keys_sorted, s);
  if (inv) hipFreeAsync(inv, s);
  if (rdeg) hipFreeAsync(rdeg, s);
  if (tmp) hipFreeAsync(tmp, s);
  if (iso) hipFreeAsync(iso, s);
  return e;
}

}  // namespace

namespace mmi {

size_t relabel_temp_bytes(int64_t n) {
  if (n <= 0) return 0;
  // the sort's and the scan's own scratch, as rocPRIM reports it for these
  // sizes; without a device to ask, twice the sorted pairs plus 64 MiB
  size_t sort_bytes = 0, scan_bytes = 0;
  uint32_t* k = nullptr;
  int32_t* o = nullptr;
  int64_t* d = nullptr;
  auto ids = rocprim::counting_iterator<int32_t>(0);
  hipError_t e = hipSuccess;
  for (int bits : {7, 2}) {  // both modes' sorts
    size_t b = 0;
    if (e == hipSuccess)
      e = rocprim::radix_sort_pairs(nullptr, b, k, k, ids, o, (size_t)n, 0, bits, (hipStream_t)0);
    if (b > sort_bytes) sort_bytes = b;
  }
  if (e == hipSuccess)
    e = rocprim::exclusive_scan(nullptr, scan_bytes, d, d, (int64_t)0, (size_t)(n + 1),
                                rocprim::plus<int64_t>(), (hipStream_t)0);
  const size_t tmp = e == hipSuccess ? (sort_bytes > scan_bytes ? sort_bytes : scan_bytes)
                                     : 16 * (size_t)n + ((size_t)64 << 20);
  // keys, sorted keys, inverse map, degrees in new ids, the isolated count,
  // and the scratch, each a separate stream-ordered allocation
  return round_up(4 * (size_t)n, 256) * 3 + round_up(8 * (size_t)(n + 1), 256) + 256 +
         round_up(tmp, 256);
}

size_t relabel_bytes(int64_t n, int64_t m) {
  return round_up(sizeof(int64_t) * (size_t)(n + 1), 256) + round_up(sizeof(int32_t) * (size_t)n, 256) +
         round_up(sizeof(int32_t) * (size_t)m, 256);
}

hipError_t build_relabel(const void* off, int off64, const int32_t* nbr, int64_t n, int64_t m,
                         int mode, int64_t hot, uint8_t* region, RelabelView* view, hipStream_t s) {
  view->off = reinterpret_cast<int64_t*>(region);
  view->orig = reinterpret_cast<int32_t*>(region + round_up(sizeof(int64_t) * (size_t)(n + 1), 256));
  view->nbr = reinterpret_cast<int32_t*>(reinterpret_cast<uint8_t*>(view->orig) +
                                         round_up(sizeof(int32_t) * (size_t)n, 256));
  view->n_isolated = 0;
  (void)m;
  if (n == 0) return hipSuccess;
  if (off64)
    return build_typed(static_cast<const int64_t*>(off), nbr, n, mode, hot, view->off, view->nbr,
                       view->orig, &view->n_isolated, s);
  return build_typed(static_cast<const int32_t*>(off), nbr, n, mode, hot, view->off, view->nbr,
                     view->orig, &view->n_isolated, s);
}

}  // namespace mmi

// Create-time reordering of short neighbour lists (tuning.order_lists).
//
// The sweep examines a source's list in stored order and stops at the first
// neighbour it can match (the early exit of Fig. 6g), so the order inside a
// list decides how many neighbour states a scan reads. On a skewed graph the
// high-degree neighbours are usually matched already when a scan reaches
// them, and low-degree ones are usually still free. This copy keeps every id
// and every list's place, and only reorders each list of at most 256 entries
// by ascending log2 degree of the neighbour (stable: the given order among
// neighbours of one bucket). Longer lists, which the hub tier cuts into
// pieces anyway, are copied as they are. The sweep then reads the copy with
// the caller's offsets; nothing else changes (same ids, same states, same
// output).
//
// Upper neighbours first (order_lists = 2): a sweep that examines each edge
// from its lower end skips every neighbour below the source. This order puts
// the neighbours above the source first, in the same degree order, and those
// below it after them, so a scan can stop at the first neighbour below its
// source instead of reading the rest of the list only to skip it.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

static_assert(mmi::kOrderedMax == 256, "the wavefront sort takes 4 keys per lane");

namespace {

__device__ __forceinline__ uint32_t bucket_of(int64_t d) {
  return d <= 0 ? 0u : 64u - (uint32_t)__clzll((unsigned long long)d);  // 1 + floor(log2 d)
}

template <typename OffT>
__global__ void bucket_kernel(const OffT* __restrict__ off, int64_t n, uint8_t* __restrict__ bk) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    bk[v] = (uint8_t)bucket_of((int64_t)off[v + 1] - (int64_t)off[v]);
}

// Sorts the 256 keys k[0..3] of a wavefront (element lane * 4 + q in k[q])
// ascending: a bitonic network, partners in the same lane for distances
// below 4 and across lanes (a shuffle) above.
__device__ __forceinline__ void bitonic256(uint32_t (&k)[4], int lane) {
#pragma unroll
  for (int size = 2; size <= 256; size <<= 1) {
#pragma unroll
    for (int d = size >> 1; d > 0; d >>= 1) {
      uint32_t other[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        other[q] = d < 4 ? k[q ^ d] : (uint32_t)__shfl_xor((int)k[q], d >> 2, 64);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane * 4 + q;
        const bool up = (i & size) == 0, low = (i & d) == 0;
        const uint32_t a = k[q], b = other[q];
        k[q] = (low == up) ? (a < b ? a : b) : (a < b ? b : a);
      }
    }
  }
}

// A wavefront takes 64 vertices at a time. A lane reorders its own vertex's
// list when it has at most 64 entries: an insertion sort of the keys
// bucket * 64 + position (distinct keys, so the order among equal buckets is
// the given one), element k of lane l at k * 64 + l so that the lanes use
// different banks; then it writes the ids in key order. Lists of 65 to 256
// entries are then reordered by the whole wavefront, one after the other:
// keys bucket * 256 + position, four per lane, sorted by a bitonic network in
// registers. Longer lists are copied as they are, coalesced. With
// upper_first, a neighbour below the list's vertex has a key above every
// other (a bit above the bucket's: a degree below 2^63 has a bucket below 64).
template <typename OffT>
__global__ __launch_bounds__(256) void order_lists_kernel(const OffT* __restrict__ off,
                                                          const int32_t* __restrict__ nbr,
                                                          const uint8_t* __restrict__ bk, int64_t n,
                                                          int upper_first,
                                                          int32_t* __restrict__ out) {
  __shared__ uint16_t keys_s[4][64 * 64];
  uint16_t* srt = keys_s[threadIdx.x >> 6];
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += waves * 64) {
    const int64_t v = base + lane;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = (int64_t)off[v];
      e = (int64_t)off[v + 1];
    }
    const bool midl = e - b > 64 && e - b <= mmi::kOrderedMax;
    const bool longl = e - b > mmi::kOrderedMax;
    if (!midl && !longl) {
      const int len = (int)(e - b);
      for (int k = 0; k < len; ++k) {
        const int32_t y = nbr[b + k];
        const uint32_t low = (upper_first && (int64_t)y < v) ? 1u : 0u;
        const uint16_t key = (uint16_t)((low << 12) | ((uint32_t)bk[y] << 6) | (uint32_t)k);
        int j = k - 1;
        while (j >= 0 && srt[j * 64 + lane] > key) {
          srt[(j + 1) * 64 + lane] = srt[j * 64 + lane];
          --j;
        }
        srt[(j + 1) * 64 + lane] = key;
      }
      for (int k = 0; k < len; ++k) out[b + k] = nbr[b + (srt[k * 64 + lane] & 63)];
    }
    uint64_t mm = __ballot(midl);
    while (mm) {
      const int l = __builtin_ctzll(mm);
      mm &= mm - 1;
      const int64_t lb = __shfl(b, l, 64);
      const int len = (int)(__shfl(e, l, 64) - lb);
      const int64_t lv = base + l;
      uint32_t k[4];
      for (int q = 0; q < 4; ++q) {
        const int i = lane * 4 + q;
        if (i < len) {
          const int32_t y = nbr[lb + i];
          const uint32_t low = (upper_first && (int64_t)y < lv) ? 1u : 0u;
          k[q] = (low << 14) | ((uint32_t)bk[y] << 8) | (uint32_t)i;
        } else {
          k[q] = 0xffffffffu;
        }
      }
      bitonic256(k, lane);
      for (int q = 0; q < 4; ++q) {
        const int r = lane * 4 + q;
        if (r < len) out[lb + r] = nbr[lb + (k[q] & 255u)];
      }
    }
    uint64_t lm = __ballot(longl);
    while (lm) {
      const int l = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t lb = __shfl(b, l, 64), le = __shfl(e, l, 64);
      for (int64_t j = lb + lane; j < le; j += 64) out[j] = nbr[j];
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
hipError_t build_typed(const OffT* off, const int32_t* nbr, int64_t n, int upper_first, int32_t* out,
                       hipStream_t s) {
  uint8_t* bk = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&bk), (size_t)n, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((bucket_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, n, bk);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((order_lists_kernel<OffT>), dim3(blocks_for(n)), dim3(256), 0, s, off, nbr, bk,
                       n, upper_first, out);
    e = hipGetLastError();
  }
  if (bk) hipFreeAsync(bk, s);
  // a run may come on another stream: the copy is complete when create returns
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace

namespace mmi {

size_t order_temp_bytes(int64_t n) { return n > 0 ? round_up((size_t)n, 256) : 0; }

hipError_t build_ordered_lists(const void* off, int off64, const int32_t* nbr, int64_t n,
                               int upper_first, int32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (off64) return build_typed(static_cast<const int64_t*>(off), nbr, n, upper_first, out, s);
  return build_typed(static_cast<const int32_t*>(off), nbr, n, upper_first, out, s);
}

}  // namespace mmi

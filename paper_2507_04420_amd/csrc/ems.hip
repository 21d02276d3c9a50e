// Iterated Endpoints Mutual Selection (Section II-C), the multi-pass scheme
// the paper contrasts Skipper with, as a GPU baseline.
//
// Every iteration has two steps over the vertices still unmatched:
//   * selection: each unmatched vertex scans its whole list and selects its
//     heaviest edge to an unmatched neighbour;
//   * refinement: an edge selected by both of its ends becomes a match.
// Edge weights are fixed pseudo-random values: SplitMix64 (Steele, Lea and
// Flood, OOPSLA 2014) of the seed, xor the key (min << 32 | max), mixed again.
// The heaviest free edge overall is always selected by both ends, so every
// iteration matches at least one pair, and the result is the greedy matching
// in descending weight order (ties: smaller key first). The pass ends when no
// unmatched vertex has an unmatched neighbour. Its work is a full scan of the
// unmatched vertices' lists per iteration, against Skipper's single scan that
// stops at a source's first match.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "internal.h"
#include "mm.h"

using mmi::fail;
#define HIP_TRY MMI_HIP_TRY

namespace {

constexpr size_t kEmsCountersOffset = mmi::kCheckOffset + 128;  // touched, selecting, pairs

__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void wave_add(unsigned long long v, unsigned long long* out) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0 && v)
    __hip_atomic_fetch_add(out, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void ems_fill_kernel(int32_t* __restrict__ mate, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) mate[v] = -1;
}

// Selection: sel[x] = the unmatched neighbour y of unmatched x whose edge is
// heaviest (weight descending, then key ascending), or -1. A wavefront takes
// 64 vertices, one per lane; a list of more than 64 entries is then scanned
// by the whole wavefront (lanes 64 entries apart, a shuffle reduction), so
// that a hub's list does not hold one lane for its whole length.
__device__ __forceinline__ bool heavier(uint64_t w, uint64_t key, uint64_t bw, uint64_t bkey) {
  return w > bw || (w == bw && key < bkey);
}

template <typename OffT>
__global__ void ems_select_kernel(const OffT* __restrict__ off, const int32_t* __restrict__ nbr,
                                  int64_t n, const int32_t* __restrict__ mate,
                                  int32_t* __restrict__ sel, uint64_t seed_mix,
                                  unsigned long long* counters) {
  unsigned long long touched = 0, selecting = 0;
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < n; base += waves * 64) {
    const int64_t x = base + lane;
    int32_t best = -1;
    int64_t b = 0, e = 0;
    bool longl = false;
    if (x < n && mate[x] == -1) {
      b = (int64_t)off[x];
      e = (int64_t)off[x + 1];
      touched += (unsigned long long)(e - b);
      longl = e - b > 64;
      uint64_t bw = 0, bkey = 0;
      for (int64_t i = b; i < e && !longl; ++i) {
        const int64_t y = nbr[i];
        if (y == x || mate[y] != -1) continue;
        const uint64_t key = x < y ? ((uint64_t)x << 32) | (uint64_t)y
                                   : ((uint64_t)y << 32) | (uint64_t)x;
        const uint64_t w = splitmix64(seed_mix ^ key);
        if (best < 0 || heavier(w, key, bw, bkey)) {
          best = (int32_t)y;
          bw = w;
          bkey = key;
        }
      }
    }
    if (x < n && !longl) {
      sel[x] = best;
      selecting += best >= 0;
    }
    uint64_t lm = __ballot(longl);
    while (lm) {
      const int l = __builtin_ctzll(lm);
      lm &= lm - 1;
      const int64_t xl = __shfl(x, l, 64), lb = __shfl(b, l, 64), le = __shfl(e, l, 64);
      int32_t by = -1;
      uint64_t bw = 0, bkey = ~0ull;
      for (int64_t i = lb + lane; i < le; i += 64) {
        const int64_t y = nbr[i];
        if (y == xl || mate[y] != -1) continue;
        const uint64_t key = xl < y ? ((uint64_t)xl << 32) | (uint64_t)y
                                    : ((uint64_t)y << 32) | (uint64_t)xl;
        const uint64_t w = splitmix64(seed_mix ^ key);
        if (by < 0 || heavier(w, key, bw, bkey)) {
          by = (int32_t)y;
          bw = w;
          bkey = key;
        }
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        const int32_t oy = __shfl_xor(by, d, 64);
        const uint64_t ow = __shfl_xor(bw, d, 64), okey = __shfl_xor(bkey, d, 64);
        if (oy >= 0 && (by < 0 || heavier(ow, okey, bw, bkey))) {
          by = oy;
          bw = ow;
          bkey = okey;
        }
      }
      if (lane == l) {
        sel[xl] = by;
        selecting += by >= 0;
      }
    }
  }
  wave_add(touched, counters + 0);
  wave_add(selecting, counters + 1);
}

// Refinement: mutually selected edges become matches (written once, by the
// lower end).
__global__ void ems_refine_kernel(const int32_t* __restrict__ sel, int64_t n,
                                  int32_t* __restrict__ mate, unsigned long long* counters) {
  unsigned long long pairs = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    const int64_t y = sel[x];
    if (y > x && sel[y] == x) {
      mate[x] = (int32_t)y;
      mate[y] = (int32_t)x;
      ++pairs;
    }
  }
  wave_add(pairs, counters + 2);
}

int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

}  // namespace

extern "C" {

size_t mm_ems_scratch_bytes(int64_t n) {
  if (n < 0 || n > INT32_MAX) return 0;
  return mmi::round_up((size_t)n * sizeof(int32_t), 256) + 256;
}

mm_status mm_ems_run(mm_handle h, void* stream, uint64_t seed, void* scratch,
                     size_t scratch_bytes, int32_t* match_out, mm_ems_stats* stats) {
  if (!h) return fail(MM_ERR_INVALID_ARG, "handle is null");
  const int64_t n = mmi::handle_n(h);
  if (!(mmi::handle_flags(h) & MM_SYMMETRIC))
    return fail(MM_ERR_UNSUPPORTED, "mutual selection needs a handle created with MM_SYMMETRIC");
  if (n > 0 && (!scratch || !match_out)) return fail(MM_ERR_INVALID_ARG, "null buffer");
  if (scratch_bytes < mm_ems_scratch_bytes(n))
    return fail(MM_ERR_OUT_OF_MEMORY, "scratch has %zu bytes, needs %zu", scratch_bytes,
                mm_ems_scratch_bytes(n));
  if (reinterpret_cast<uintptr_t>(scratch) % 256)
    return fail(MM_ERR_INVALID_ARG, "scratch must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t* sel = static_cast<int32_t*>(scratch);
  auto* ctr = reinterpret_cast<unsigned long long*>(mmi::handle_ws(h) + kEmsCountersOffset);
  const uint64_t seed_mix = splitmix64(seed);
  int64_t iters = 0, touched = 0, pairs = 0;
  if (n > 0) {
    hipLaunchKernelGGL(ems_fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, match_out, n);
    HIP_TRY(hipGetLastError());
    // every iteration matches at least one pair, so n/2 + 1 iterations always suffice
    for (int64_t it = 0; it <= n / 2 + 1; ++it) {
      HIP_TRY(hipMemsetAsync(ctr, 0, 3 * sizeof(unsigned long long), s));
      if (mmi::handle_off64(h))
        hipLaunchKernelGGL((ems_select_kernel<int64_t>), dim3(grid_for(n)), dim3(256), 0, s,
                           static_cast<const int64_t*>(mmi::handle_off(h)), mmi::handle_nbr(h), n,
                           match_out, sel, seed_mix, ctr);
      else
        hipLaunchKernelGGL((ems_select_kernel<int32_t>), dim3(grid_for(n)), dim3(256), 0, s,
                           static_cast<const int32_t*>(mmi::handle_off(h)), mmi::handle_nbr(h), n,
                           match_out, sel, seed_mix, ctr);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(ems_refine_kernel, dim3(grid_for(n)), dim3(256), 0, s, sel, n, match_out,
                         ctr);
      HIP_TRY(hipGetLastError());
      unsigned long long c[3];
      HIP_TRY(hipMemcpyAsync(c, ctr, sizeof(c), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      ++iters;
      touched += (int64_t)c[0];
      pairs += (int64_t)c[2];
      if (c[1] == 0) break;  // no unmatched vertex has an unmatched neighbour
      if (c[2] == 0) return fail(MM_ERR_NO_PROGRESS, "an iteration matched no pair");
    }
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iterations = iters;
    stats->touched = touched;
    stats->pairs = pairs;
  }
  return MM_OK;
}

}  // extern "C"

// Vertex-state layouts and the reservation protocol of Skipper (Algorithm 1,
// Section IV-C) on gfx950 atomics.
//
// States (Section IV-B, Fig. 4): ACC (accessible), RSVD (reserved), MCHD
// (matched). ACC -> RSVD and ACC -> MCHD are taken by atomics; RSVD -> ACC and
// RSVD -> MCHD are taken only by the lane that holds the reservation; MCHD is
// absorbing.
//
// Because MCHD is absorbing, a plain (cacheable, possibly stale) load that
// returns MCHD is always right; a stale load can only under-report MCHD, and
// the atomic that follows then returns the current state. Every decision that
// acts on ACC or RSVD is taken from an atomic's return value or from a
// device-coherent load.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmk {

enum : int { R_ACC = 0, R_RSVD = 1, R_MCHD = 2 };

__device__ __forceinline__ uint32_t ld_cached(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ int32_t ld_cached(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint32_t ld_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_coherent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_agent(uint32_t* p, uint32_t& expected, uint32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas_agent(int32_t* p, int32_t& expected, int32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Packed layout: one state byte per vertex, four vertices per 32-bit word.
// Encoding ACC = 0, RSVD = 1, MCHD = 3, so that
//   reserve  (ACC -> RSVD)  = fetch_or(1): leaves RSVD and MCHD unchanged, and
//                             its return value says which state it met; it
//                             cannot fail because a neighbouring byte changed;
//   commit   (RSVD -> MCHD) = fetch_or(2) by the holder;
//   release  (RSVD -> ACC)  = fetch_and(~1) by the holder;
//   match v  (ACC -> MCHD)  = 32-bit CAS on the containing word, retried while
//                             only other bytes of the word differ.
struct LayoutU8 {
  uint32_t* w;
  int32_t* mate;

  __device__ __forceinline__ static uint32_t shift(int64_t v) { return (uint32_t)(v & 3) * 8u; }

  // Cached read used to skip matched vertices; returns the whole word so that
  // the match CAS can start from it.
  __device__ __forceinline__ bool seen_matched(int64_t v, uint32_t& word) const {
    word = ld_cached(w + (v >> 2));
    return ((word >> shift(v)) & 2u) != 0;
  }
  __device__ __forceinline__ int state_coherent(int64_t v) const {
    uint32_t b = (ld_coherent(w + (v >> 2)) >> shift(v)) & 0xffu;
    return b == 0 ? R_ACC : (b & 2u) ? R_MCHD : R_RSVD;
  }
  __device__ __forceinline__ int reserve(int64_t u) const {
    uint32_t sh = shift(u);
    uint32_t old = __hip_atomic_fetch_or(w + (u >> 2), 1u << sh, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    uint32_t b = (old >> sh) & 0xffu;
    return b == 0 ? R_ACC : (b & 2u) ? R_MCHD : R_RSVD;
  }
  // guess: the last word value seen for v's word (a stale guess costs one CAS).
  // Returns R_ACC on success, R_MCHD / R_RSVD for the state met, or -1 when the
  // word kept changing in its other bytes (the caller retries next trip).
  __device__ __forceinline__ int match(int64_t v, int64_t u, uint32_t& guess,
                                       uint32_t& word_retries) const {
    (void)u;
    const uint32_t sh = shift(v);
    uint32_t* p = w + (v >> 2);
    uint32_t cur = guess & ~(0xffu << sh);
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
      uint32_t seen = cur;
      if (cas_agent(p, seen, cur | (3u << sh))) return R_ACC;
      const uint32_t b = (seen >> sh) & 0xffu;
      guess = seen;
      if (b != 0) return (b & 2u) ? R_MCHD : R_RSVD;
      cur = seen;
      ++word_retries;
    }
    return -1;
  }
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    __hip_atomic_fetch_or(w + (u >> 2), 2u << shift(u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mate[u] = (int32_t)v;
    mate[v] = (int32_t)u;
  }
  __device__ __forceinline__ void release(int64_t u) const {
    __hip_atomic_fetch_and(w + (u >> 2), ~(1u << shift(u)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Word layout: one int32 per vertex that is also the output mate array:
// -1 = ACC, -2 = RSVD, >= 0 = MCHD holding the mate.
struct LayoutU32 {
  int32_t* mate;

  __device__ __forceinline__ bool seen_matched(int64_t v, uint32_t& word) const {
    int32_t s = ld_cached(mate + v);
    word = (uint32_t)s;
    return s >= 0;
  }
  __device__ __forceinline__ int state_coherent(int64_t v) const {
    int32_t s = ld_coherent(mate + v);
    return s == -1 ? R_ACC : s >= 0 ? R_MCHD : R_RSVD;
  }
  __device__ __forceinline__ int reserve(int64_t u) const {
    int32_t seen = -1;
    if (cas_agent(mate + u, seen, -2)) return R_ACC;
    return seen >= 0 ? R_MCHD : R_RSVD;
  }
  __device__ __forceinline__ int match(int64_t v, int64_t u, uint32_t& guess,
                                       uint32_t& word_retries) const {
    (void)guess;
    (void)word_retries;
    int32_t seen = -1;
    if (cas_agent(mate + v, seen, (int32_t)u)) return R_ACC;
    return seen >= 0 ? R_MCHD : R_RSVD;
  }
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    __hip_atomic_store(mate + u, (int32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ void release(int64_t u) const {
    __hip_atomic_store(mate + u, (int32_t)-1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

}  // namespace mmk

// Vertex-state layouts and the reservation protocol of Skipper (Algorithm 1,
// Section IV-C) on gfx950 atomics.
//
// States (Section IV-B, Fig. 4): ACC (accessible), RSVD (reserved), MCHD
// (matched). ACC -> RSVD and ACC -> MCHD are taken by atomics; RSVD -> ACC and
// RSVD -> MCHD are taken only by the lane that holds the reservation; MCHD is
// absorbing.
//
// Two ways to take v (template parameter TWO_PHASE):
//   * as printed in Algorithm 1: one CAS moves v from ACC to MCHD;
//   * two-phase: v is reserved with the same operation as u (ACC -> RSVD),
//     and once both are held the holder marks both matched. The transitions
//     are still those of Fig. 4 (ACC -> RSVD -> MCHD). The linearisation
//     point of a successful match moves from the CAS on v to the reservation
//     of v, after which the pair is certain. It avoids CAS, whose throughput on
//     gfx950 is several times lower than that of fetch_or / atomic_min.
//   Ids are still taken in order (u < v), so every wait chain climbs in id and
//   ends at a vertex that is ACC or MCHD: no deadlock.
//
// Because MCHD is absorbing, a plain (cacheable, possibly stale) load that
// returns MCHD is always right; a stale load can only under-report MCHD, and
// the atomic that follows then returns the current state. Every decision that
// acts on ACC or RSVD is taken from an atomic's return value or from a
// device-coherent load.
//
// Each layout exposes raw operations that return the word they observed, and
// a decoder, so that the sweep can issue an operation on one loop trip and
// act on its result on the next.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmk {

enum : int { R_ACC = 0, R_RSVD = 1, R_MCHD = 2 };

__device__ __forceinline__ uint32_t ld_cached(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint32_t ld_coherent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t cas_agent(uint32_t* p, uint32_t expected, uint32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value observed
}
__device__ __forceinline__ void or_agent(uint32_t* p, uint32_t bits) {
  __hip_atomic_fetch_or(p, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Matched-vertex hint, set after a vertex becomes MCHD: one bit per vertex
// (lg = 5: 32 vertices per word, set with an atomic or) or one byte per
// vertex (lg = 2: set with a plain byte store, no atomic). Read with cached
// loads to skip matched neighbours; a clear entry proves nothing (the state
// word decides), so a late or lost update is harmless.
struct Hint {
  uint32_t* bits;  // null: no hint, the state word itself is read
  uint32_t lg;     // log2 of vertices per 32-bit word: 5 (bits) or 2 (bytes)
  __device__ __forceinline__ const uint32_t* word(int64_t v) const { return bits + (v >> lg); }
  __device__ __forceinline__ uint32_t shift(int64_t v) const {
    return (uint32_t)(v & ((1 << lg) - 1)) << (5 - lg);
  }
  __device__ __forceinline__ void set(int64_t v) const {
    if (lg == 2)
      reinterpret_cast<uint8_t*>(bits)[v] = 1;
    else
      or_agent(bits + (v >> 5), 1u << (uint32_t)(v & 31));
  }
};

// 32-bit words of a hint of mode `mode` (1: bits, 2: bytes) for n vertices.
__host__ __device__ __forceinline__ int64_t hint_words(int64_t n, int mode) {
  return mode == 2 ? (n + 3) / 4 : mode == 1 ? (n + 31) / 32 : 0;
}
__host__ __device__ __forceinline__ uint32_t hint_lg(int mode) { return mode == 2 ? 2u : 5u; }

// Packed layouts: BITS = 8 (one state byte per vertex, four per 32-bit word)
// or BITS = 2 (sixteen vertices per word). Field encoding ACC = 0, RSVD = 1,
// MCHD = 3, so that
//   reserve  (ACC -> RSVD)  = fetch_or(1): leaves RSVD and MCHD unchanged, and
//                             its return value says which state it met; it
//                             cannot fail because a neighbouring field changed;
//   commit   (RSVD -> MCHD) = fetch_or(2) by the holder;
//   release  (RSVD -> ACC)  = fetch_and(~1) by the holder;
//   match v  (ACC -> MCHD)  = 32-bit CAS on the containing word, expecting the
//                             field ACC and the other fields as last seen; when
//                             only the other fields differ, it is retried
//                             (CAS protocol only).
// The mate array is separate (written once per vertex).
template <int BITS, bool TWO_PHASE>
struct LayoutPacked {
  static_assert(BITS == 8 || BITS == 2, "packed state fields are 8 or 2 bits");
  uint32_t* w;
  int32_t* mate;
  Hint hint;
  static constexpr bool kTwoPhase = TWO_PHASE;
  static constexpr bool kStateIsMate = false;
  static constexpr bool kRelabelled = false;
  static constexpr int kPerWord = 32 / BITS;
  static constexpr int kLog = BITS == 8 ? 2 : 4;
  static constexpr uint32_t kMask = BITS == 8 ? 0xffu : 0x3u;

  __device__ __forceinline__ static uint32_t shift(int64_t v) {
    return (uint32_t)(v & (kPerWord - 1)) * (uint32_t)BITS;
  }
  __device__ __forceinline__ uint32_t* wp(int64_t v) const { return w + (v >> kLog); }
  __device__ __forceinline__ uint32_t word_cached(int64_t v) const { return ld_cached(wp(v)); }
  __device__ __forceinline__ uint32_t word_coherent(int64_t v) const { return ld_coherent(wp(v)); }
  __device__ __forceinline__ static int decode(uint32_t word, int64_t v) {
    const uint32_t b = (word >> shift(v)) & kMask;
    return b == 0 ? R_ACC : (b & 2u) ? R_MCHD : R_RSVD;
  }
  __device__ __forceinline__ static bool matched(uint32_t word, int64_t v) {
    return ((word >> shift(v)) & 2u) != 0;
  }
  // Returns the word before the fetch_or; decode() == R_ACC means u is now held.
  __device__ __forceinline__ uint32_t reserve(int64_t u) const {
    return __hip_atomic_fetch_or(wp(u), 1u << shift(u), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ static uint32_t match_expected(uint32_t guess, int64_t v) {
    return guess & ~(kMask << shift(v));
  }
  // One CAS attempt; returns the word observed. Success iff it equals
  // match_expected(guess, v).
  __device__ __forceinline__ uint32_t match(int64_t v, int64_t u, uint32_t guess) const {
    (void)u;
    const uint32_t exp = match_expected(guess, v);
    return cas_agent(wp(v), exp, exp | (3u << shift(v)));
  }
  __device__ __forceinline__ static bool match_ok(uint32_t seen, uint32_t guess, int64_t v) {
    return seen == match_expected(guess, v);
  }
  // u held (and v held too in the two-phase protocol, else already MCHD).
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    or_agent(wp(u), 2u << shift(u));
    if (TWO_PHASE) or_agent(wp(v), 2u << shift(v));
    mate[u] = (int32_t)v;
    mate[v] = (int32_t)u;
    if (hint.bits) {
      hint.set(u);
      hint.set(v);
    }
  }
  __device__ __forceinline__ void release(int64_t u) const {
    __hip_atomic_fetch_and(wp(u), ~(1u << shift(u)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Lazy output. fin_probe reads x's state once its list is exhausted with
  // every neighbour matched; if that read is ACC, x can never be matched and
  // finalize_after_read writes its output.
  __device__ __forceinline__ uint32_t fin_probe(int64_t x) const { return word_coherent(x); }
  __device__ __forceinline__ void finalize_after_read(int64_t x) const { mate[x] = -1; }
  __device__ __forceinline__ void write_unmatched(int64_t x) const { mate[x] = -1; }
};

// Word layout: one int32 per vertex that is also the output mate array.
// With the CAS protocol: ACC = -1, RSVD = -2, MCHD = the mate (>= 0), so an
// unmatched vertex already holds the output value -1.
// With the two-phase protocol: ACC = INT32_MAX, RSVD = INT32_MAX - 1, MCHD =
// the mate, and reserve = atomic_min(RSVD), which moves ACC to RSVD and leaves
// RSVD and every mate (< RSVD) unchanged. A vertex found final-unmatched is
// moved from ACC to -1 by a CAS (lazy output); without lazy output a last
// pass rewrites ACC as -1. -1 reads as "cannot be matched" (every neighbour of
// such a vertex is MCHD).
template <bool TWO_PHASE>
struct LayoutU32 {
  int32_t* mate;
  Hint hint;
  static constexpr bool kTwoPhase = TWO_PHASE;
  static constexpr bool kStateIsMate = true;
  static constexpr bool kRelabelled = false;
  static constexpr uint32_t kAcc = TWO_PHASE ? 0x7fffffffu : 0xffffffffu;
  static constexpr uint32_t kRsvd = TWO_PHASE ? 0x7ffffffeu : 0xfffffffeu;

  __device__ __forceinline__ uint32_t* p(int64_t v) const {
    return reinterpret_cast<uint32_t*>(mate + v);
  }
  __device__ __forceinline__ uint32_t word_cached(int64_t v) const { return ld_cached(p(v)); }
  __device__ __forceinline__ uint32_t word_coherent(int64_t v) const { return ld_coherent(p(v)); }
  __device__ __forceinline__ static int decode(uint32_t word, int64_t) {
    return word == kAcc ? R_ACC : word == kRsvd ? R_RSVD : R_MCHD;
  }
  __device__ __forceinline__ static bool matched(uint32_t word, int64_t) {
    return word != kAcc && word != kRsvd;
  }
  __device__ __forceinline__ uint32_t reserve(int64_t u) const {
    if (TWO_PHASE)
      return (uint32_t)__hip_atomic_fetch_min(reinterpret_cast<int32_t*>(p(u)), (int32_t)kRsvd,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return cas_agent(p(u), kAcc, kRsvd);
  }
  __device__ __forceinline__ static uint32_t match_expected(uint32_t, int64_t) { return kAcc; }
  __device__ __forceinline__ uint32_t match(int64_t v, int64_t u, uint32_t) const {
    return cas_agent(p(v), kAcc, (uint32_t)u);
  }
  __device__ __forceinline__ static bool match_ok(uint32_t seen, uint32_t, int64_t) {
    return seen == kAcc;
  }
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    __hip_atomic_store(mate + u, (int32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (TWO_PHASE)
      __hip_atomic_store(mate + v, (int32_t)u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hint.bits) {
      hint.set(u);
      hint.set(v);
    }
  }
  __device__ __forceinline__ void release(int64_t u) const {
    __hip_atomic_store(mate + u, (int32_t)kAcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Lazy output (two-phase encoding only; with the CAS encoding ACC is
  // already -1). fin_probe moves x from ACC to -1 with one CAS and returns the
  // state it met: ACC means done; RSVD means poll again; MCHD means matched.
  __device__ __forceinline__ uint32_t fin_probe(int64_t x) const {
    if (!TWO_PHASE) return word_coherent(x);
    return cas_agent(p(x), kAcc, 0xffffffffu);
  }
  __device__ __forceinline__ void finalize_after_read(int64_t) const {}
  __device__ __forceinline__ void write_unmatched(int64_t x) const {
    if (TWO_PHASE)
      __hip_atomic_store(mate + x, (int32_t)-1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// A layout over relabelled vertex ids whose output is in the caller's ids:
// the base layout keeps the states (and, for the word layout, the mates) in
// the new ids; each committed pair is also written to `out` through the map
// from new to given ids. `out` is filled with -1 before the sweep, so the
// lazy output paths are not used with it.
// The source's given id is read with its block (coalesced) and passed to the
// commit, so that only the neighbour's is looked up there.
template <class Base>
struct Relabelled : Base {
  int32_t* out;
  const int32_t* orig;
  static constexpr bool kRelabelled = true;
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    Base::commit(u, v);
    const int32_t ou = orig[u], ov = orig[v];
    out[ou] = ov;
    out[ov] = ou;
  }
  // x is u or v, and ox its given id
  __device__ __forceinline__ void commit_src(int64_t u, int64_t v, int64_t x, int32_t ox) const {
    Base::commit(u, v);
    const int32_t oy = orig[u == x ? v : u];
    out[ox] = oy;
    out[oy] = ox;
  }
};

}  // namespace mmk

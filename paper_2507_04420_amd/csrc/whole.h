// A graph small enough for one wavefront, swept with its states in that
// wavefront's LDS.
//
// When one wavefront sweeps a whole graph (a small batch member, or a small
// graph alone), no other wavefront ever reads or writes that graph's states.
// They can then live in LDS instead of device memory: Algorithm 1's reserve,
// CAS and commit become LDS atomics, whose latency is a small fraction of a
// device-scope atomic's (those pass L2 and go to memory). The protocol is the
// same (Section IV-B, Fig. 4) in its two-phase form (v is reserved like u,
// then both are marked matched): the states are packed 2 bits per vertex
// (LayoutPacked<2>, 4 KB for 16384 vertices), and a CAS on a packed word
// would fail whenever another lane changed a neighbouring field, while a
// fetch_or reservation never does. The mates are kept in LDS as well (16-bit
// ids), and a last pass writes the whole output, coalesced: inside the sweep
// the only device-memory operations left are the loads of offsets and ids,
// so a loop trip never waits for a store.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mm.h"
#include "protocol.h"
#include "sweep.h"

namespace mmk {

// LDS words a wavefront needs for n vertices: the states (2 bits each), then
// the mates (16 bits each), each part a whole number of 16-byte quads.
__host__ __device__ __forceinline__ int64_t whole_state_words(int64_t n) {
  return ((n + 15) / 16 + 3) / 4 * 4;
}
__host__ __device__ __forceinline__ int64_t whole_lds_words(int64_t n) {
  return whole_state_words(n) + ((n + 1) / 2 + 3) / 4 * 4;
}

// The two-phase packed layout with its mates in LDS (16-bit ids: every
// vertex id of such a graph is below MM_LDS_WHOLE_MAX <= 32768).
struct LayoutLds : LayoutPacked<2, true> {
  int16_t* mate16;
  __device__ __forceinline__ void commit(int64_t u, int64_t v) const {
    or_agent(wp(u), 2u << shift(u));
    or_agent(wp(v), 2u << shift(v));
    mate16[u] = (int16_t)v;
    mate16[v] = (int16_t)u;
  }
};
static_assert(MM_LDS_WHOLE_MAX <= 32768, "16-bit mates");

// Sweeps the sources 0 .. n-1 of one graph with this wavefront, using lds
// (at least whole_lds_words(n) words of LDS). mate: the graph's output (n
// entries, device memory), written for every vertex at the end.
template <typename OffT, bool STATS>
__device__ __forceinline__ void sweep_whole_lds(SweepParams p, const OffT* __restrict__ off,
                                                const int32_t* __restrict__ nbr, int64_t n,
                                                int32_t* mate, uint32_t* lds, QSlot* q,
                                                Counters<STATS>& cnt) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t words = whole_state_words(n);
  for (int64_t i = lane; i < words; i += 64) lds[i] = 0u;  // every vertex ACC
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  p.wave_vertices = (n + 63) / 64 * 64;
  p.disperse = 1;  // lanes stride apart (see the whole-graph case of mm_run)
  p.hub_degree = 0;
  p.chunks = nullptr;
  LayoutLds lay;
  lay.w = lds;
  lay.mate = nullptr;
  lay.hint = Hint{nullptr, 0};
  lay.mate16 = reinterpret_cast<int16_t*>(lds + words);
  // the graph is in device memory: global loads, which the waits for LDS
  // results do not include (flat loads would be counted with them)
  using GOff = const __attribute__((address_space(1))) OffT*;
  using GNbr = const __attribute__((address_space(1))) int32_t*;
  sweep_block<OffT, LayoutLds, false, false, STATS, GOff, GNbr>(p, (GOff)off, (GNbr)nbr, lay, 0, n,
                                                                q, cnt);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // every lane is done, so no vertex is still reserved: a state is ACC or MCHD
  for (int64_t v = lane; v < n; v += 64)
    mate[v] = LayoutLds::matched(lds[v >> 4], v) ? (int32_t)lay.mate16[v] : -1;
}

}  // namespace mmk

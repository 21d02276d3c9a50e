// The single-pass sweep of Skipper (Algorithm 1) as a gfx950 kernel.
//
// Work decomposition. Each wavefront owns a block of consecutive source
// vertices (the GPU form of the paper's blocks of consecutive vertices with
// about equal work, Section IV-C). Every lane works on one source at a time;
// a lane that finishes takes the next source of the block (ballot + mbcnt
// hand-out), so lanes stay busy whatever the spread of scan lengths. The
// hardware dispatcher hands blocks to the 256 CUs as earlier ones retire.
//
// Per lane, one source x at a time (Section II-B, CSR form):
//   * skip x if it is already matched (Fig. 6g);
//   * walk N_x in stored order; skip self-loops (Alg. 1 L6-7) and neighbours
//     seen matched; for a candidate y take u = min(x,y), v = max(x,y)
//     (Alg. 1 L8-9, which rules out reservation cycles) and run the
//     reservation: reserve u (L11), move v from ACC to MCHD (L13-14), then
//     mark u matched (L15) or release it (L17-18);
//   * stop at the first matched pair: x is matched and the rest of N_x is
//     never read.
//
// Waiting without intra-wavefront spin. Lanes of a wavefront share one
// instruction stream, so a lane may not loop waiting for a reservation that
// another lane of the same wavefront holds. Every wait of Algorithm 1 (L11's
// "continue" on a reserved u, L13's loop on a reserved v) therefore becomes
// "stay in this phase and retry on the next trip of the wavefront's loop":
// each trip, every lane advances by at most one protocol step. Reservation
// chains only wait on higher ids (u < v), so the lane at the top of any chain
// meets ACC or MCHD and finishes; no trip can block all lanes.
//
// Long scans. When a lane has scanned `assist_after` neighbours and still has
// more than a few left, the whole wavefront reads the next 64 ids of that list
// at once, finds the first one not seen matched with a ballot, and moves the
// lane's cursor there (or 64 ahead). It also re-reads the source's state so a
// source matched by another lane stops early.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "protocol.h"

namespace mmk {

enum : int { P_IDLE = 0, P_SCAN = 1, P_TRYU = 2, P_TRYV = 3, P_FINAL = 4, P_DONE = 5 };

// Launch parameters shared by every block of a sweep. Vertex ids inside a
// block are local to its graph; the layout object and the offsets pointer
// are already based at the graph's first vertex.
struct SweepParams {
  int64_t wave_vertices;   // multiple of 64
  int32_t disperse;
  int32_t assist_after;
  int64_t iter_cap;        // 0: per-block default budget
  uint32_t* err;           // bit 0: loop-trip budget exceeded
};

enum : int {
  S_SOURCES = 0, S_SKIPPED, S_TOUCHED, S_ASSIST, S_RES_ATT, S_RES_CONF, S_RES_MCHD, S_MAT_ATT,
  S_MAT_CONF, S_MAT_MCHD, S_WORD_RETRY, S_PAIRS, S_TRIPS, S_NUM
};

template <bool ON>
struct Counters {
  __device__ __forceinline__ void add(int, uint32_t) {}
  __device__ __forceinline__ void flush(unsigned long long*) {}
  uint32_t word_retries = 0;
};
template <>
struct Counters<true> {
  uint32_t c[S_NUM] = {};
  uint32_t word_retries = 0;
  __device__ __forceinline__ void add(int k, uint32_t v) { c[k] += v; }
  __device__ __forceinline__ void flush(unsigned long long* out) {
    c[S_WORD_RETRY] += word_retries;
#pragma unroll
    for (int k = 0; k < S_NUM; ++k) {
      unsigned long long s = c[k];
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
      if ((threadIdx.x & 63) == 0 && s)
        __hip_atomic_fetch_add(out + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
};

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Sweeps the sources vb .. vb+nv-1 of one graph with one wavefront.
// off: the graph's offsets (entries index `nbr`); L: its state layout;
// mate: its mate array (local ids).
template <typename OffT, class Layout, bool LAZY, bool STATS>
__device__ __forceinline__ void sweep_block(const SweepParams& a, const OffT* __restrict__ off,
                                            const int32_t* __restrict__ nbr, const Layout& L,
                                            int32_t* __restrict__ mate, int64_t vb, int64_t nv,
                                            Counters<STATS>& cnt) {
  const int lane = (int)(threadIdx.x & 63);
  const bool disperse = a.disperse && nv == a.wave_vertices;
  const int64_t stride = a.wave_vertices >> 6;

  // Loop-trip budget: explicit, or by default 65536 plus 8 per neighbour entry
  // of the block (a pass needs at most about one trip per entry plus short
  // waits), so even an unforeseen livelock ends with an error flag.
  const int64_t cap = a.iter_cap > 0 ? a.iter_cap
                                     : 65536 + 8 * ((int64_t)off[vb + nv] - (int64_t)off[vb]);
  int64_t handed = 0;  // wavefront-uniform hand-out cursor
  int phase = P_IDLE;
  int64_t x = 0, i = 0, e = 0, u = 0, v = 0;
  uint32_t xword = 0, vguess = 0;
  int32_t steps = 0;
  int64_t trips = 0;

  while (true) {
    // ---- hand the block's next sources to idle lanes
    const uint64_t idle = __ballot(phase == P_IDLE);
    if (idle) {
      if (phase == P_IDLE) {
        const int64_t k = handed + lanes_below(idle);
        if (k < nv) {
          x = vb + (disperse ? (k & 63) * stride + (k >> 6) : k);
          const int64_t b = (int64_t)off[x], en = (int64_t)off[x + 1];
          i = b;
          e = en;
          steps = 0;
          if (STATS) cnt.add(S_SOURCES, 1);
          if (b == en) {
            if (LAZY) mate[x] = -1;  // no incident entry: never matched (symmetric input)
          } else if (L.seen_matched(x, xword)) {
            if (STATS) cnt.add(S_SKIPPED, 1);
          } else {
            phase = P_SCAN;
          }
        } else {
          phase = P_DONE;
        }
      }
      handed += __popcll(idle);
    }
    const uint64_t busy = __ballot(phase != P_IDLE && phase != P_DONE);
    if (!busy) {
      if (handed >= nv) break;
      continue;
    }
    if (++trips > cap) {
      if (phase == P_TRYV) L.release(u);
      if (lane == 0) atomicOr(a.err, 1u);
      break;
    }

    // ---- wavefront assist for one long scan
    if (a.assist_after > 0) {
      const uint64_t lm = __ballot(phase == P_SCAN && steps >= a.assist_after && (e - i) > 4);
      if (lm) {
        const int ld = __builtin_ctzll(lm);
        const int64_t xl = readlane64(x, ld), il = readlane64(i, ld), el = readlane64(e, ld);
        const int64_t p = il + lane;
        bool cand = false;
        if (p < el) {
          const int32_t yy = nbr[p];
          uint32_t wd;
          cand = (yy != xl) && !L.seen_matched(yy, wd);
          if (STATS) cnt.add(S_ASSIST, 1);
        }
        const uint64_t cm = __ballot(cand);
        if (lane == ld) {
          i = cm ? il + __builtin_ctzll(cm) : (el - il > 64 ? il + 64 : el);
          uint32_t wd;
          if (L.seen_matched(x, wd)) phase = P_IDLE;  // source matched elsewhere
        }
      }
    }

    // ---- one scan step: find the next candidate edge (x, y)
    if (phase == P_SCAN) {
      if (i >= e) {
        phase = LAZY ? P_FINAL : P_IDLE;
      } else {
        const int64_t y = (int64_t)nbr[i];
        ++i;
        ++steps;
        if (STATS) cnt.add(S_TOUCHED, 1);
        uint32_t yword;
        if (y != x && !L.seen_matched(y, yword)) {
          u = (x < y ? x : y);
          v = (x < y ? y : x);
          vguess = (x < y) ? yword : xword;
          phase = P_TRYU;
        }
      }
    }
    // ---- reserve u (Alg. 1 L11-12)
    if (phase == P_TRYU) {
      if (STATS) cnt.add(S_RES_ATT, 1);
      const int r = L.reserve(u);
      if (r == R_ACC) {
        phase = P_TRYV;
      } else if (r == R_MCHD) {
        if (STATS) cnt.add(S_RES_MCHD, 1);
        phase = (u == x) ? P_IDLE : P_SCAN;
      } else {
        if (STATS) cnt.add(S_RES_CONF, 1);
        // L10 re-check of v while u is held by another lane; retry next trip
        if (L.state_coherent(v) == R_MCHD) phase = (v == x) ? P_IDLE : P_SCAN;
      }
    }
    // ---- match v (Alg. 1 L13-16), then mark u or release it (L17-18)
    if (phase == P_TRYV) {
      if (STATS) cnt.add(S_MAT_ATT, 1);
      const int r = L.match(v, u, vguess, cnt.word_retries);
      if (r == R_ACC) {
        L.commit(u, v);
        if (STATS) cnt.add(S_PAIRS, 1);
        phase = P_IDLE;
      } else if (r == R_MCHD) {
        if (STATS) cnt.add(S_MAT_MCHD, 1);
        L.release(u);
        phase = (v == x) ? P_IDLE : P_SCAN;
      } else if (r == R_RSVD) {
        if (STATS) cnt.add(S_MAT_CONF, 1);
      }
    }
    // ---- lazy output: x's list is exhausted, every neighbour is matched, so
    // x can only be matched by a reservation already in flight on x
    if (LAZY && phase == P_FINAL) {
      const int s = L.state_coherent(x);
      if (s == R_ACC) {
        mate[x] = -1;
        phase = P_IDLE;
      } else if (s == R_MCHD) {
        phase = P_IDLE;
      }
    }
  }
  if (STATS) cnt.add(S_TRIPS, lane == 0 ? (uint32_t)trips : 0u);
}

}  // namespace mmk

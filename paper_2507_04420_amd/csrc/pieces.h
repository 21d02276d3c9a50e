// The wavefront tier of long lists (tuning.hub_wave): a wavefront takes 64
// pieces of long lists (the hub tier's table entries: entries b .. e-1 of
// source x), like the lane tier, but sweeps each live one with all its lanes.
//
// First every lane reads the state of one piece's source, so pieces whose
// source is already matched (most of them, since hubs are usually matched as
// neighbours before their pieces run) cost one parallel load, as in the lane
// tier. Then, for each live piece in table order, the 64 lanes read 64
// consecutive ids per step (256 bytes, coalesced) and the states of those
// neighbours, and every lane re-reads the source's own state, so the piece
// stops as soon as the source is matched elsewhere (the early exit of Fig. 6g,
// per step instead of per id). A ballot finds the candidates in list order;
// for the first one, lane 0 runs the reservation of Algorithm 1 (take
// u = min(x, y), take v = max(x, y), commit or give u back) while the other
// lanes wait. Only lane 0 ever holds a vertex, and only while it runs one
// edge, so no lane of the wavefront waits on another lane of the same
// wavefront: lane 0 may poll a reservation another wavefront holds until it
// is released or committed (every such wait is on a higher id, as in the
// per-lane sweep). A live list is read once, coalesced, with the source
// checked before every 64 ids: the GPU form of a thread walking a hub's list.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "protocol.h"
#include "sweep.h"

namespace mmk {

enum : int { E_MATCHED = 0, E_X_DEAD, E_Y_DEAD, E_BUDGET };

// Pieces a wavefront takes per launch slot (single graphs) or work item
// (batches), in either tier: one per lane.
constexpr int kPiecesPerWave = 64;

__device__ __forceinline__ uint32_t bcast(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// One edge (x, y) by lane 0 for the whole wavefront (every lane runs the
// same uniform loop; only lane 0 touches memory). guess: the word the filter
// read for v (packed layouts' CAS guess). Returns E_MATCHED, E_X_DEAD (the
// source is matched: the piece is done), E_Y_DEAD (the edge is dead), or
// E_BUDGET (the loop budget ran out; nothing is held).
template <class Layout, bool STATS>
__device__ __forceinline__ int run_edge(const SweepParams& a, const Layout& L, int32_t x, int32_t y,
                                        uint32_t guess, uint32_t xorig, int64_t& budget,
                                        Counters<STATS>& cnt) {
  const bool l0 = (threadIdx.x & 63) == 0;
  const int32_t u = x < y ? x : y, v = x < y ? y : x;
  uint32_t vguess = guess;
  uint32_t econf = 0;
  enum { RES, CHK, MAT, MATW, VW } ph = RES;
  auto dead = [&](int32_t w) {
    if (STATS && l0) cnt.edge_done(econf);
    return w == x ? E_X_DEAD : E_Y_DEAD;
  };
  while (true) {
    if (--budget < 0) {
      if (l0 && (ph == MAT || ph == MATW)) L.release(u);  // held: give it back
      return E_BUDGET;
    }
    if (ph == RES) {
      uint32_t r = 0;
      if (l0) {
        r = L.reserve(u);
        if (STATS) cnt.add(S_RES_ATT, 1);
      }
      r = bcast(r);
      const int s = Layout::decode(r, u);
      if (s == R_ACC) {
        ph = MAT;
      } else {
        ++econf;
        if (STATS && l0) cnt.add(s == R_MCHD ? S_RES_MCHD : S_RES_CONF, 1);
        if (s == R_MCHD) return dead(u);
        ph = CHK;
      }
    } else if (ph == CHK) {
      uint32_t ru = 0, rv = 0;
      if (l0) {
        ru = L.word_coherent(u);
        rv = L.word_coherent(v);
      }
      ru = bcast(ru);
      rv = bcast(rv);
      if (Layout::decode(rv, v) == R_MCHD) return dead(v);
      const int su = Layout::decode(ru, u);
      if (su == R_MCHD) return dead(u);
      if (su == R_ACC) ph = RES;
    } else if (ph == MAT) {
      uint32_t r = 0;
      if (l0) {
        r = Layout::kTwoPhase ? L.reserve(v) : L.match(v, u, vguess);
        if (STATS) cnt.add(S_MAT_ATT, 1);
      }
      r = bcast(r);
      bool won;
      int s;
      if (Layout::kTwoPhase) {
        s = Layout::decode(r, v);
        won = s == R_ACC;
      } else {
        won = Layout::match_ok(r, vguess, v);
        s = won ? R_ACC : Layout::decode(r, v);
      }
      if (won) {
        if (l0) {
          if constexpr (Layout::kRelabelled)
            L.commit_src(u, v, x, (int32_t)xorig);
          else
            L.commit(u, v);
          if (STATS) {
            cnt.add(S_PAIRS, 1);
            cnt.edge_done(econf);
          }
        }
        return E_MATCHED;
      }
      if (s == R_ACC) {  // another field of v's word changed: try again
        if (STATS && l0) cnt.add(S_WORD_RETRY, 1);
        vguess = r;
      } else if (s == R_RSVD) {
        ++econf;
        if (STATS && l0) cnt.add(S_MAT_CONF, 1);
        if (a.wait_release) {
          if (l0) L.release(u);
          ph = VW;
        } else {
          ph = MATW;
        }
      } else {
        ++econf;
        if (STATS && l0) cnt.add(S_MAT_MCHD, 1);
        if (l0) L.release(u);
        return dead(v);
      }
    } else {  // MATW (holding u) or VW (holding nothing): wait for v
      uint32_t r = 0;
      if (l0) r = L.word_coherent(v);
      r = bcast(r);
      const int s = Layout::decode(r, v);
      if (s == R_ACC) {
        vguess = r;
        ph = ph == MATW ? MAT : RES;
      } else if (s == R_MCHD) {
        if (ph == MATW && l0) L.release(u);
        return dead(v);
      }
    }
  }
}

// Sweeps pieces p0 .. p0+np-1 (np <= 64) of the hub table a.chunks with this
// wavefront.
//
// seen (LDS, or null): the workgroup tier (hub_wave = 2, single graphs). The
// nseen wavefronts of a workgroup take consecutive runs of pieces, most of
// them pieces of the same long lists, and each keeps in seen[its wavefront]
// the last source it found matched. Every wavefront checks those slots as
// well as the source's state before each step, so once one wavefront matches
// a hub the others stop its pieces at their next step, without waiting for
// the state word to reach them through a cache. A slot only ever holds a
// matched vertex (matched is final), so a slot read late or overwritten
// costs only a step.
template <class Layout, bool HINT, bool STATS, class NbrP = const int32_t*>
__device__ __forceinline__ void sweep_pieces_wave(const SweepParams& a, NbrP __restrict__ nbr,
                                                  const Layout& L, int64_t p0, int64_t np,
                                                  Counters<STATS>& cnt, int32_t* seen = nullptr,
                                                  int nseen = 0) {
  const int lane = (int)(threadIdx.x & 63);
  auto seen_matched = [&](int32_t v) -> bool {
    bool hit = false;
    if (seen)
      for (int k = 0; k < nseen; ++k)
        hit |= __hip_atomic_load(seen + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == v;
    return hit;
  };
  auto mark = [&](int32_t v) {
    if (seen && lane == 0)
      __hip_atomic_store(seen + (threadIdx.x >> 6), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  };
  const bool upper = a.upper_only != 0;
  const bool nt = a.stream_loads != 0;
  auto filter_word = [&](int64_t y) -> uint32_t {
    if (HINT) return ld_cached(L.hint.word(y));
    return L.word_cached(y);
  };
  auto filter_matched = [&](uint32_t word, int64_t y) -> bool {
    if (HINT) return ((word >> L.hint.shift(y)) & 1u) != 0;
    return Layout::matched(word, y);
  };
  // one piece per lane: its source's state decides whether the piece is live
  HubChunk mine{0, 0, 0, 0};
  bool live = false;
  if (lane < np) {
    mine = a.chunks[p0 + lane];
    live = !filter_matched(filter_word(mine.x), mine.x) && !seen_matched(mine.x);
  }
  uint64_t todo = __ballot(live);
  // loop budget: one step per 64 entries of every piece and the polls of its
  // edges, with the per-block default's slack
  int64_t budget = a.iter_cap > 0 ? a.iter_cap : 65536 + 8 * np * a.hub_chunk;
  int64_t steps = 1;
  while (todo) {
    const int pl = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int32_t x = __builtin_amdgcn_readlane(mine.x, pl);
    const int64_t cb = ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine.b, pl)) |
                       ((int64_t)__builtin_amdgcn_readlane((int)(mine.b >> 32), pl) << 32);
    const int64_t ce = ((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mine.e, pl)) |
                       ((int64_t)__builtin_amdgcn_readlane((int)(mine.e >> 32), pl) << 32);
    uint32_t xorig = 0;
    if constexpr (Layout::kRelabelled) xorig = (uint32_t)L.orig[x];
    bool done = false;
    for (int64_t i = cb; i < ce && !done; i += 64) {
      ++steps;
      if (--budget < 0) {
        if (lane == 0) atomicOr(a.err, 1u);
        return;
      }
      const bool have = i + lane < ce;
      const int32_t y = have ? ld_stream(nbr + i + lane, nt) : x;
      const bool ok = have && y != x && (!upper || y > x);
      const uint32_t yw = ok ? filter_word(y) : 0u;
      const uint32_t xw = bcast(filter_word(x));
      if (STATS && lane == 0) cnt.add(S_TOUCHED, (uint32_t)(ce - i < 64 ? ce - i : 64));
      if (filter_matched(xw, x) || seen_matched(x)) {  // the source is matched: the rest is skipped
        mark(x);
        break;
      }
      uint64_t cand = __ballot(ok && !filter_matched(yw, y));
      while (cand) {
        const int l = __builtin_ctzll(cand);
        cand &= cand - 1;
        const int32_t yy = __builtin_amdgcn_readlane(y, l);
        const uint32_t yyw = (uint32_t)__builtin_amdgcn_readlane((int)yw, l);
        // the CAS guess for v: the word read for it (the hint carries none)
        const uint32_t guess = HINT ? 0u : (x < yy ? yyw : xw);
        const int r = run_edge<Layout, STATS>(a, L, x, yy, guess, xorig, budget, cnt);
        if (r == E_BUDGET) {
          if (lane == 0) atomicOr(a.err, 1u);
          return;
        }
        if (r != E_Y_DEAD) {  // x is matched, by this edge or elsewhere
          mark(x);
          done = true;
          break;
        }
      }
    }
  }
  if (STATS) cnt.add(S_TRIPS, lane == 0 ? (uint32_t)steps : 0u);
}

}  // namespace mmk

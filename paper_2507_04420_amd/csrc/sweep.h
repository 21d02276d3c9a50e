// The single-pass sweep of Skipper (Algorithm 1) as a gfx950 kernel.
//
// Work decomposition. Each wavefront owns a block of consecutive source
// vertices (the GPU form of the paper's blocks of consecutive vertices,
// Section IV-C). A wavefront-level front end reads the block 64 sources at a
// time (offsets and state, one coalesced load per lane), drops the sources
// that need no scan (no entries, or already matched: Fig. 6g) and queues the
// rest in LDS. Every lane works on one source at a time and takes the next
// queued source when it finishes, so lanes stay busy whatever the spread of
// scan lengths, and skipped sources cost no lane any loop trip. The hardware
// dispatcher hands blocks to the CUs as earlier ones retire.
//
// Per lane, one source x at a time (Section II-B, CSR form):
//   * skip x if it is already matched (Fig. 6g);
//   * walk N_x in stored order, W ids at a time; skip self-loops (Algorithm 1)
//     and neighbours seen matched; for a candidate y take u = min(x,y),
//     v = max(x,y) (the id order of Algorithm 1, which rules out reservation
//     cycles) and run the reservation: reserve u, take v, then mark u matched
//     or release it;
//   * stop at the first matched pair: the rest of N_x is never read.
//
// Pipelining. A lane's work is a chain of dependent memory operations
// (offsets -> ids -> states -> reserve -> take v). Each trip of the loop
// first consumes the results of the operations issued on the previous trip
// (ALU only), then issues one operation per lane, so the operations of all
// lanes, whatever their phase, are in flight together.
//
// Waiting without intra-wavefront spin. Lanes of a wavefront share one
// instruction stream, so no lane may loop waiting for a reservation that
// another lane of its wavefront holds. Every wait of Algorithm 1 (the retry
// on a reserved u, the loop on a reserved v) is "stay in this
// phase and poll again next trip". Reservation chains only wait on higher ids
// (u < v), so the lane at the top of any chain meets ACC or MCHD and finishes.
// With wait_release a lane releases u before it waits for v, so no lane waits
// on a lane that is itself waiting and no chain of holders forms.
//
// Long scans (the wavefront tier). When a lane has read `assist_after` ids of
// its list and more than 2W remain, the whole wavefront reads the next 64 ids
// of that list and their states in two trips, finds the first candidate with
// a ballot and moves the lane's cursor there (or 64 ahead); the other lanes
// keep working meanwhile.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "protocol.h"

namespace mmk {

constexpr int kMaxW = 4;

enum : int {
  P_IDLE = 0,  // needs a source
  P_IDS,       // next W neighbour ids requested
  P_STS,       // states of the buffered ids requested
  P_RES,       // reserve(u) issued (Algorithm 1's take of u)
  P_CHK,       // u was reserved by another lane: coherent re-read of u and v
  P_MAT,       // v requested: CAS ACC -> MCHD, or reserve(v) (two-phase)
  P_MATW,      // v was reserved by another lane: coherent re-read of v
  P_VW,        // the same wait with u released first (wait_release): then u again
  P_FIN,       // list exhausted: final check of the source's own state
  P_ASST,      // paused while the wavefront scans ahead for this lane
  P_DONE
};

// Launch parameters shared by every block of a sweep. Vertex ids inside a
// block are local to its graph; the layout object and the offsets pointer
// are already based at the graph's first vertex.
// A piece of a long list (the hub tier): entries b .. e-1 of source x.
struct HubChunk {
  int64_t b, e;
  int32_t x;
  int32_t pad;
};

struct SweepParams {
  int64_t wave_vertices;   // multiple of 64
  int32_t disperse;
  int32_t assist_after;
  int32_t scan_width;      // 1..kMaxW
  int32_t stream_loads;    // 1: offsets and ids through non-temporal loads
  int32_t wait_release;    // 1: release u while waiting for a reserved v
  int32_t upper_only;      // 1 (symmetric input): examine only neighbours above the source
  int32_t hub_wave;        // 1, 2: hub pieces swept by a wavefront each (pieces.h), else a lane each
  int32_t lower_stop;      // > 0 (with upper_only): every list of at most this many entries
                           // holds its neighbours above the source first, so its scan ends at
                           // the first neighbour below the source; 0: no such order
  int32_t probe_first;     // 1: a source's first state read takes only its first candidate;
                           // 2: every state read takes one candidate
  int64_t iter_cap;        // 0: per-block default budget
  uint32_t* err;           // bit 0: loop-trip budget exceeded
  // Hub tier. Main pass: sources with more than hub_degree entries are left
  // to the chunk pass (0: none are). Chunk pass (chunks != null): the block
  // indexes this table instead of the vertices, each entry one piece of at
  // most hub_chunk entries of one long list.
  int64_t hub_degree;
  int64_t hub_chunk;
  const HubChunk* chunks;
};

// Counters of the instrumented build. S_H0 .. S_H0+9: edges by the number of
// conflicts they met, in Table II's bins (1, 2, 3-4, ..., 129-256, >256);
// S_CMAX: the most conflicts one edge met.
enum : int {
  S_SOURCES = 0, S_SKIPPED, S_TOUCHED, S_ASSIST, S_RES_ATT, S_RES_CONF, S_RES_MCHD, S_MAT_ATT,
  S_MAT_CONF, S_MAT_MCHD, S_WORD_RETRY, S_PAIRS, S_TRIPS, S_H0, S_CMAX = S_H0 + 10, S_NUM
};

template <bool ON>
struct Counters {
  __device__ __forceinline__ void add(int, uint32_t) {}
  __device__ __forceinline__ void edge_done(uint32_t) {}
  __device__ __forceinline__ void flush(unsigned long long*) {}
};
template <>
struct Counters<true> {
  uint32_t c[S_NUM] = {};
  __device__ __forceinline__ void add(int k, uint32_t v) { c[k] += v; }
  // An edge's processing ended after `conf` conflicts.
  __device__ __forceinline__ void edge_done(uint32_t conf) {
    if (!conf) return;
    const int bin = conf == 1 ? 0 : min(9, 32 - __clz((int)(conf - 1)));  // ceil(log2 conf)
#pragma unroll
    for (int b = 0; b < 10; ++b)
      if (b == bin) c[S_H0 + b] += 1;  // unrolled: the array stays in registers
    c[S_CMAX] = conf > c[S_CMAX] ? conf : c[S_CMAX];
  }
  __device__ __forceinline__ void flush(unsigned long long* out) {
#pragma unroll
    for (int k = 0; k < S_NUM; ++k) {
      unsigned long long s = c[k];
      if (k == S_CMAX) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
          const unsigned long long o = __shfl_xor(s, d, 64);
          s = o > s ? o : s;
        }
        if ((threadIdx.x & 63) == 0 && s)
          __hip_atomic_fetch_max(out + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        continue;
      }
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

// One queued source of a wavefront's front end (kept in LDS).
struct QSlot {
  int64_t b, e;
  int32_t x;
  uint32_t word;  // the filter word read for x (a first guess for a CAS on x)
  uint32_t orig;  // relabelled graphs: x's given id
  uint32_t pad;
};
constexpr int kQueue = 128;  // ring entries per wavefront (power of two)

// Loads of offsets and neighbour ids: non-temporal when streaming, so that
// these once-read lines leave L2 before the state lines that are read again.
// P: a pointer, generic or to global memory (address space 1).
template <typename P>
__device__ __forceinline__ auto ld_stream(P p, bool nt) ->
    typename std::remove_cv<typename std::remove_reference<decltype(p[0] + 0)>::type>::type {
  return nt ? __builtin_nontemporal_load(p) : *p;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Sweeps the sources vb .. vb+nv-1 of one graph with one wavefront.
// off: the graph's offsets (entries index `nbr`); L: its state layout (with
// its mate array and hint, all based at the graph's first vertex).
// HINT: skip matched neighbours by the matched hint (a bit or byte per vertex) instead of the
// state word.
// q: this wavefront's LDS ring of kQueue slots.
// OffP / NbrP: the pointer types of off and nbr (generic by default; a caller
// that knows the graph is in device memory may pass global pointers).
template <typename OffT, class Layout, bool HINT, bool LAZY, bool STATS,
          class OffP = const OffT*, class NbrP = const int32_t*>
__device__ __forceinline__ void sweep_block(const SweepParams& a, OffP __restrict__ off,
                                            NbrP __restrict__ nbr, const Layout& L,
                                            int64_t vb, int64_t nv, QSlot* q,
                                            Counters<STATS>& cnt) {
  const int lane = (int)(threadIdx.x & 63);
  const int W = a.scan_width;
  const bool nt = a.stream_loads != 0;
  // Each undirected edge once (Algorithm 1 iterates over E): on symmetric
  // input the edge {x, y} is also in y's list, and the lane of min(x, y)
  // examines it whenever that endpoint is unmatched, so a lane may skip the
  // neighbours below its source without reading their states.
  const bool upper = a.upper_only != 0;
  // Dispersed lanes: hand-out index kk goes to source (kk & 63) * stride +
  // (kk >> 6), so that the lanes of a wavefront work stride sources apart;
  // indices whose source lies past the block are skipped.
  const bool disperse = a.disperse != 0 && !a.chunks;
  const int64_t stride = (nv + 63) >> 6;
  const int64_t span = disperse ? stride << 6 : nv;  // hand-out indices
  // Loop-trip budget: explicit, or by default 65536 plus 8 per neighbour entry
  // of the block (a pass needs at most about one trip per entry plus short
  // waits), so even an unforeseen livelock ends with an error flag.
  const int64_t cap = a.iter_cap > 0 ? a.iter_cap
                     : a.chunks ? 65536 + 8 * nv * a.hub_chunk
                                : 65536 + 8 * ((int64_t)off[vb + nv] - (int64_t)off[vb]);

  // Filter reads: the hint bit, or the vertex's own state word.
  auto filter_word = [&](int64_t y) -> uint32_t {
    if (HINT) return ld_cached(L.hint.word(y));
    return L.word_cached(y);
  };
  auto filter_matched = [&](uint32_t word, int64_t y) -> bool {
    if (HINT) return ((word >> L.hint.shift(y)) & 1u) != 0;
    return Layout::matched(word, y);
  };

  auto source_of = [&](int64_t kk) -> int64_t {
    return vb + (disperse ? (kk & 63) * stride + (kk >> 6) : kk);
  };
  auto in_block = [&](int64_t kk) -> bool {
    return disperse ? kk < span && (kk & 63) * stride + (kk >> 6) < nv : kk < nv;
  };
  // front end (wavefront-uniform): next hand-out index to read, the chunk
  // whose offsets and states are in flight, and the LDS ring's cursors
  int64_t chunk_next = 0, chunk_base = 0;
  bool chunk_pending = false;
  uint32_t q_head = 0, q_tail = 0;
  int64_t cb_b = 0, cb_e = 0;  // this lane's source of the pending chunk
  int32_t cb_x = 0;
  uint32_t cb_w = 0, cb_o = 0;  // its filter word and (relabelled graphs) given id
  int64_t trips = 0;
  int phase = P_IDLE;
  bool cut = false;  // the current list is ordered upper neighbours first
  bool probe1 = false;  // the next state read is the source's first: one candidate only
  int kr = 0;           // the buffered ids [k, kr) have their states read
  // vertex ids (local to the graph, < 2^31) in 32 bits, list positions in 64
  int32_t x = 0, u = 0, v = 0;
  int64_t i = 0, e = 0;
  int32_t ids[kMaxW];
  uint32_t rw[kMaxW];
#pragma unroll
  for (int j = 0; j < kMaxW; ++j) {
    ids[j] = 0;
    rw[j] = 0;
  }
  int k = 0, nids = 0, steps = 0;
  uint32_t xword = 0, vguess = 0;
  uint32_t xorig = 0;  // relabelled graphs: the source's given id
  uint32_t econf = 0;  // conflicts met by the current edge (instrumented build)
  // Results of the operations issued on a trip, one register per phase:
  // different lanes issue different phases on the same trip, and a shared
  // destination register would force a wait between them.
  uint32_t res_w = 0, chk_u = 0, chk_v = 0, mat_w = 0, matw_w = 0, fin_w = 0;
  // wavefront assist (uniform state)
  int asst = 0, al = 0;
  int64_t ai = 0, ae = 0;
  int32_t ax = 0;
  int32_t aid = -1;
  uint32_t aw = 0, axw = 0;

  // Next candidate among the buffered ids whose states were read, [k, kr);
  // else the states of the rest of the step's ids; else read on.
  auto advance = [&]() {
    int found = -1;
    int32_t fy = 0;
    uint32_t fw = 0;
#pragma unroll
    for (int j = kMaxW - 1; j >= 0; --j) {
      if (j >= k && j < kr && (int64_t)ids[j] != x && (!upper || ids[j] > x) &&
          !filter_matched(rw[j], ids[j])) {
        found = j;
        fy = ids[j];
        fw = rw[j];
      }
    }
    if (found >= 0) {
      const int32_t y = fy;
      k = found + 1;
      u = x < y ? x : y;
      v = x < y ? y : x;
      vguess = HINT ? 0u : ((x < y) ? fw : xword);
      phase = P_RES;
    } else if (kr < nids) {  // the rest of the step's ids: their states next
      k = kr;
      phase = P_STS;
    } else {
      k = nids;
      phase = (i < e) ? P_IDS : (LAZY ? P_FIN : P_IDLE);
    }
  };
  // The current edge cannot be matched because w (u or v) is matched.
  auto edge_dead = [&](int32_t w) {
    if (STATS) {
      cnt.edge_done(econf);
      econf = 0;
    }
    if (w == x) phase = P_IDLE; else advance();
  };

  // Consumes the result of the operation this lane issued last.
  auto consume = [&]() {
    switch (phase) {
      case P_IDS: {
        const int64_t rem = e - i;
        nids = rem < W ? (int)rem : W;
        i += nids;
        steps += nids;
        k = 0;
        if (STATS) cnt.add(S_TOUCHED, (uint32_t)nids);
        if (cut) {
          // past the neighbours above x: the rest of the list is below it
          bool low = false;
#pragma unroll
          for (int j = 0; j < kMaxW; ++j) low = low || (j < nids && ids[j] < x);
          if (low) e = i;
        }
        bool any = !upper;
#pragma unroll
        for (int j = 0; j < kMaxW; ++j) any = any || (j < nids && ids[j] > x);
        if (any) {
          phase = P_STS;
        } else {  // every id read is below the source: read on, no states
          k = nids;
          phase = (i < e) ? P_IDS : (LAZY ? P_FIN : P_IDLE);
        }
        break;
      }
      case P_STS:
        advance();
        break;
      case P_RES: {
        const int s = Layout::decode(res_w, u);
        if (s == R_ACC) {
          phase = P_MAT;
        } else if (s == R_MCHD) {
          if (STATS) {  // a failed take of u: a conflict too (Table II)
            cnt.add(S_RES_MCHD, 1);
            ++econf;
          }
          edge_dead(u);
        } else {
          if (STATS) {
            cnt.add(S_RES_CONF, 1);
            ++econf;
          }
          phase = P_CHK;
        }
        break;
      }
      case P_CHK: {
        const int su = Layout::decode(chk_u, u), sv = Layout::decode(chk_v, v);
        if (sv == R_MCHD) {
          edge_dead(v);
        } else if (su == R_MCHD) {
          edge_dead(u);
        } else if (su == R_ACC) {
          phase = P_RES;
        }
        break;
      }
      case P_MAT: {
        bool won;
        int s;
        if (Layout::kTwoPhase) {
          s = Layout::decode(mat_w, v);
          won = s == R_ACC;
        } else {
          won = Layout::match_ok(mat_w, vguess, v);
          s = won ? R_ACC : Layout::decode(mat_w, v);
        }
        if (won) {
          if constexpr (Layout::kRelabelled)
            L.commit_src(u, v, x, (int32_t)xorig);
          else
            L.commit(u, v);
          if (STATS) {
            cnt.add(S_PAIRS, 1);
            cnt.edge_done(econf);
            econf = 0;
          }
          phase = P_IDLE;
        } else if (s == R_ACC) {  // CAS lost to a change in another byte of the word
          if (STATS) cnt.add(S_WORD_RETRY, 1);
          vguess = mat_w;
        } else if (s == R_RSVD) {
          if (STATS) {
            cnt.add(S_MAT_CONF, 1);
            ++econf;
          }
          if (a.wait_release) {
            // hold nothing while waiting: a lane waiting on u then need not
            // wait for this lane's wait too, so no chain of holders forms
            L.release(u);
            phase = P_VW;
          } else {
            phase = P_MATW;
          }
        } else {
          if (STATS) {  // a failed take of v: a conflict too (Table II)
            cnt.add(S_MAT_MCHD, 1);
            ++econf;
          }
          L.release(u);
          edge_dead(v);
        }
        break;
      }
      case P_MATW: {
        const int s = Layout::decode(matw_w, v);
        if (s == R_ACC) {
          vguess = matw_w;
          phase = P_MAT;
        } else if (s == R_MCHD) {
          L.release(u);
          edge_dead(v);
        }
        break;
      }
      case P_VW: {
        const int s = Layout::decode(matw_w, v);
        if (s == R_ACC) {
          vguess = matw_w;
          phase = P_RES;  // take u again, then v
        } else if (s == R_MCHD) {
          edge_dead(v);
        }
        break;
      }
      case P_FIN: {
        // x's list is exhausted and every neighbour was seen matched, so only
        // a reservation already in flight on x can still match it. fin_w is
        // the state read (or, for the word layout with the two-phase protocol,
        // the state a CAS ACC -> -1 met).
        const int s = Layout::decode(fin_w, x);
        if (s == R_ACC) {
          L.finalize_after_read(x);
          phase = P_IDLE;
        } else if (s == R_MCHD) {
          phase = P_IDLE;
        }
        break;
      }
      default:
        break;
    }
  };
  // Issues this lane's next operation: one per lane and phase.
  auto issue = [&]() {
    switch (phase) {
      case P_IDS:
#pragma unroll
        for (int j = 0; j < kMaxW; ++j)
          if (j < W) ids[j] = (i + j < e) ? ld_stream(nbr + i + j, nt) : (int32_t)x;
        break;
      case P_STS: {
        // the candidates among [k, nids); with probe1 the first one only
        int lim = nids;
#pragma unroll
        for (int j = 0; j < kMaxW; ++j) {
          if (j >= k && j < lim && (int64_t)ids[j] != x && (!upper || ids[j] > x)) {
            rw[j] = filter_word(ids[j]);
            if (probe1 || a.probe_first == 2) lim = j + 1;
          }
        }
        kr = lim;
        probe1 = false;
        break;
      }
      case P_RES:
        if (STATS) cnt.add(S_RES_ATT, 1);
        res_w = L.reserve(u);
        break;
      case P_CHK:
        chk_u = L.word_coherent(u);
        chk_v = L.word_coherent(v);
        break;
      case P_MAT:
        if (STATS) cnt.add(S_MAT_ATT, 1);
        mat_w = Layout::kTwoPhase ? L.reserve(v) : L.match(v, u, vguess);
        break;
      case P_MATW:
      case P_VW:
        matw_w = L.word_coherent(v);
        break;
      case P_FIN:
        fin_w = L.fin_probe(x);
        break;
      default:
        break;
    }
  };

#pragma unroll 1
  while (true) {
    // ---------------- consume the results of last trip's operations
    // One wait for everything issued on the previous trip (s_waitcnt vmcnt(0);
    // expcnt and lgkmcnt left at their maxima), so that no issue branch below
    // waits for a register written on an earlier trip.
    __builtin_amdgcn_s_waitcnt(0x0f70);
    consume();

    // ---------------- wavefront assist: consume
    if (asst == 2) {
      const bool cand = aid >= 0 && (int64_t)aid != ax && (!upper || aid > ax) &&
                        !filter_matched(aw, aid);
      const uint64_t cm = __ballot(cand);
      const uint64_t lowm = a.lower_stop > 0 ? __ballot(aid >= 0 && aid < ax) : 0;
      if (lane == al) {
        if (filter_matched(axw, x)) {
          phase = P_IDLE;  // the source was matched by another lane meanwhile
        } else {
          // an ordered list ends at its first neighbour below x; every
          // candidate comes before it
          if (cut && lowm) e = ai + __builtin_ctzll(lowm);
          i = cm ? ai + __builtin_ctzll(cm) : (ae - ai > 64 ? ai + 64 : ae);
          steps = 0;
          nids = 0;
          k = 0;
          phase = (i < e) ? P_IDS : (LAZY ? P_FIN : P_IDLE);
        }
      }
      asst = 0;
    }

    // ---------------- front end: consume the chunk read on the previous trip
    if (chunk_pending) {
      const int64_t kk = chunk_base + lane;
      bool need = false;
      int64_t xs = 0;
      if (in_block(kk)) {
        xs = cb_x;
        if (STATS && !a.chunks) cnt.add(S_SOURCES, 1);
        if (cb_b == cb_e) {
          if (LAZY) L.write_unmatched(xs);  // no incident entry: never matched (symmetric input)
        } else if (a.hub_degree > 0 && cb_e - cb_b > a.hub_degree) {
          // a long list: the chunk pass sweeps it, spread over many lanes
        } else if (filter_matched(cb_w, xs)) {
          if (STATS) cnt.add(S_SKIPPED, 1);
        } else {
          need = true;
        }
      }
      const uint64_t nm = __ballot(need);
      if (need) {
        QSlot& slot = q[(q_tail + lanes_below(nm)) & (kQueue - 1)];
        slot.x = (int32_t)xs;
        slot.b = cb_b;
        slot.e = cb_e;
        slot.word = cb_w;
        slot.orig = cb_o;
      }
      q_tail += (uint32_t)__popcll(nm);
      chunk_pending = false;
    }

    // ---------------- hand queued sources to idle lanes
    const uint64_t idle = __ballot(phase == P_IDLE);
    const uint32_t avail = q_tail - q_head;
    if (idle && avail) {
      __builtin_amdgcn_wave_barrier();
      if (phase == P_IDLE) {
        const uint32_t r = lanes_below(idle);
        if (r < avail) {
          const QSlot slot = q[(q_head + r) & (kQueue - 1)];
          x = slot.x;
          i = slot.b;
          e = slot.e;
          cut = upper && a.lower_stop > 0 && !a.chunks && e - i <= a.lower_stop;
          probe1 = a.probe_first != 0;
          xword = HINT ? 0u : slot.word;
          xorig = slot.orig;
          steps = 0;
          phase = P_IDS;
        }
      }
      const uint32_t ni = (uint32_t)__popcll(idle);
      q_head += ni < avail ? ni : avail;
    }
    const bool front_done = chunk_next >= span && !chunk_pending && q_head == q_tail;
    if (front_done && !__ballot(phase != P_IDLE) && asst == 0) break;
    if (++trips > cap) {
      if (phase == P_MAT || phase == P_MATW) L.release(u);  // holding u
      if (lane == 0) atomicOr(a.err, 1u);
      break;
    }

    // ---------------- front end: read the next 64 sources when the queue runs low
    if (!chunk_pending && chunk_next < span && q_tail - q_head < 64) {
      chunk_base = chunk_next;
      chunk_next += 64;
      const int64_t kk = chunk_base + lane;
      if (in_block(kk)) {
        int64_t xs;
        if (a.chunks) {
          const HubChunk c = a.chunks[vb + kk];
          xs = c.x;
          cb_b = c.b;
          cb_e = c.e;
        } else {
          xs = source_of(kk);
          cb_b = (int64_t)ld_stream(off + xs, nt);
          cb_e = (int64_t)ld_stream(off + xs + 1, nt);
        }
        cb_x = (int32_t)xs;
        cb_w = filter_word(xs);
        if constexpr (Layout::kRelabelled) cb_o = (uint32_t)L.orig[xs];
      }
      chunk_pending = true;
    }

    // ---------------- wavefront assist: issue
    if (asst == 1) {
      aw = (aid >= 0 && (int64_t)aid != ax && (!upper || aid > ax)) ? filter_word(aid) : 0u;
      if (lane == al) axw = filter_word(x);
      if (STATS && aid >= 0) cnt.add(S_ASSIST, 1);
      asst = 2;
    } else if (asst == 0 && a.assist_after > 0) {
      const uint64_t lm =
          __ballot(phase == P_IDS && steps >= a.assist_after && (e - i) > 2 * W);
      if (lm) {
        al = __builtin_ctzll(lm);
        ai = readlane64(i, al);
        ae = readlane64(e, al);
        ax = __builtin_amdgcn_readlane(x, al);
        if (lane == al) phase = P_ASST;
        aid = (ai + lane < ae) ? ld_stream(nbr + ai + lane, nt) : -1;
        asst = 1;
      }
    }

    // ---------------- issue one operation per lane
    issue();
  }
  if (STATS) cnt.add(S_TRIPS, lane == 0 ? (uint32_t)trips : 0u);
}

}  // namespace mmk

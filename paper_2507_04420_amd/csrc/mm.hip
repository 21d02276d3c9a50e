// C ABI of the gfx950 maximal-matching library (declared in include/mm.h):
// handles, workspace layout, argument checks, and the kernel launches of one
// pass (state initialisation, then the sweep of Algorithm 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"
#include "mm.h"
#include "pieces.h"
#include "sweep.h"
#include "whole.h"

using namespace mmk;
using mmi::fail;
using mmi::kCtrlBytes;
using mmi::kStatsOffset;
using mmi::kStatWords;
using mmi::round_up;
#define HIP_TRY MMI_HIP_TRY

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace mmi {

mm_status fail(mm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

mm_status check_tuning(const mm_tuning& t) {
  if (t.layout != MM_LAYOUT_U8 && t.layout != MM_LAYOUT_U32 && t.layout != MM_LAYOUT_U2)
    return fail(MM_ERR_INVALID_ARG, "tuning.layout must be MM_LAYOUT_U8, MM_LAYOUT_U32 or MM_LAYOUT_U2");
  if (t.protocol != MM_PROTOCOL_CAS && t.protocol != MM_PROTOCOL_TWO_PHASE)
    return fail(MM_ERR_INVALID_ARG, "tuning.protocol must be MM_PROTOCOL_CAS or MM_PROTOCOL_TWO_PHASE");
  if (t.hint < 0 || t.hint > 2) return fail(MM_ERR_INVALID_ARG, "tuning.hint must be 0, 1 or 2");
  if (t.wg_size < 64 || t.wg_size > 256 || t.wg_size % 64)
    return fail(MM_ERR_INVALID_ARG, "tuning.wg_size must be 64, 128, 192 or 256 (got %d)",
                t.wg_size);
  if (t.wave_vertices < 64 || t.wave_vertices % 64)
    return fail(MM_ERR_INVALID_ARG, "tuning.wave_vertices must be a positive multiple of 64");
  if (t.disperse != 0 && t.disperse != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.disperse must be 0 or 1");
  if (t.lazy_init != 0 && t.lazy_init != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.lazy_init must be 0 or 1");
  if (t.scan_width < 1 || t.scan_width > kMaxW)
    return fail(MM_ERR_INVALID_ARG, "tuning.scan_width must be in [1, %d]", kMaxW);
  if (t.stream_loads != 0 && t.stream_loads != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.stream_loads must be 0 or 1");
  if (t.whole_graph_vertices < 0)
    return fail(MM_ERR_INVALID_ARG, "tuning.whole_graph_vertices must be >= 0");
  if (t.relabel < 0 || t.relabel > 2)
    return fail(MM_ERR_INVALID_ARG, "tuning.relabel must be 0, 1 or 2");
  if (t.relabel == 2 && t.hot_degree < 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.hot_degree must be >= 1 with relabel = 2");
  if (t.order_lists < 0 || t.order_lists > 2)
    return fail(MM_ERR_INVALID_ARG, "tuning.order_lists must be 0, 1 or 2");
  if (t.order_lists == 2 && !t.upper_only)
    return fail(MM_ERR_INVALID_ARG, "tuning.order_lists = 2 (upper neighbours first) needs "
                "upper_only = 1");
  if (t.order_lists && t.relabel)
    return fail(MM_ERR_INVALID_ARG, "tuning.order_lists does not apply with relabel (the "
                "relabelled copy orders its short lists itself)");
  if (t.hub_degree < 0) return fail(MM_ERR_INVALID_ARG, "tuning.hub_degree must be >= 0");
  if (t.hub_degree > 0 && t.hub_chunk < 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.hub_chunk must be >= 1 when hub_degree > 0");
  if (t.probe_first < 0 || t.probe_first > 2)
    return fail(MM_ERR_INVALID_ARG, "tuning.probe_first must be 0, 1 or 2");
  if (t.occupancy != 0 && t.occupancy != 6)
    return fail(MM_ERR_INVALID_ARG, "tuning.occupancy must be 0 or 6");
  if (t.iter_cap < 0) return fail(MM_ERR_INVALID_ARG, "tuning.iter_cap must be >= 0");
  if (t.whole_graph_lds != 0 && t.whole_graph_lds != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.whole_graph_lds must be 0 or 1");
  if (t.wait_release != 0 && t.wait_release != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.wait_release must be 0 or 1");
  if (t.min_waves < 0) return fail(MM_ERR_INVALID_ARG, "tuning.min_waves must be >= 0");
  if (t.upper_only != 0 && t.upper_only != 1)
    return fail(MM_ERR_INVALID_ARG, "tuning.upper_only must be 0 or 1");
  if (t.hub_wave < 0 || t.hub_wave > 2)
    return fail(MM_ERR_INVALID_ARG, "tuning.hub_wave must be 0, 1 or 2");
  if (t.mesh_wave_vertices < 0 || t.mesh_wave_vertices % 64)
    return fail(MM_ERR_INVALID_ARG, "tuning.mesh_wave_vertices must be 0 or a positive multiple of 64");
  return MM_OK;
}

size_t state_bytes(int64_t n, const mm_tuning& t) {
  if (t.layout == MM_LAYOUT_U8) return round_up((size_t)((n + 3) / 4) * 4, 256);
  if (t.layout == MM_LAYOUT_U2) return round_up((size_t)((n + 15) / 16) * 4, 256);
  return 0;
}

size_t hint_bytes(int64_t n, const mm_tuning& t) {
  return round_up((size_t)hint_words(n, t.hint) * 4, 256);
}

void stats_from_counters(const unsigned long long* c, mm_stats* out) {
  std::memset(out, 0, sizeof(*out));
  out->sources = c[S_SOURCES];
  out->sources_skipped = c[S_SKIPPED];
  out->touched = c[S_TOUCHED];
  out->assist_reads = c[S_ASSIST];
  out->reserve_attempts = c[S_RES_ATT];
  out->reserve_conflicts = c[S_RES_CONF];
  out->reserve_matched = c[S_RES_MCHD];
  out->match_attempts = c[S_MAT_ATT];
  out->match_conflicts = c[S_MAT_CONF];
  out->match_matched = c[S_MAT_MCHD];
  out->word_retries = c[S_WORD_RETRY];
  out->pairs = c[S_PAIRS];
  out->loop_trips = c[S_TRIPS];
  out->conflict_max = c[S_CMAX];
  for (int b = 0; b < 10; ++b) out->conflict_hist[b] = c[S_H0 + b];
}

}  // namespace mmi

using mmi::check_tuning;

namespace {

// ---------------------------------------------------------------- kernels

// A region to fill, split into a scalar head up to 16-byte alignment, whole
// 16-byte quads, and a scalar tail.
struct FillRegion {
  uint32_t* head;
  int64_t head_words;
  uint4* quads;
  int64_t n_quads;
  uint32_t* tail;
  int64_t tail_words;
  uint32_t value;
};

__host__ __device__ inline FillRegion fill_region(uint32_t* p, int64_t words, uint32_t value) {
  FillRegion r;
  const int64_t mis = (int64_t)((reinterpret_cast<uintptr_t>(p) >> 2) & 3);
  r.head = p;
  r.head_words = mis ? (4 - mis < words ? 4 - mis : words) : 0;
  r.quads = reinterpret_cast<uint4*>(p + r.head_words);
  r.n_quads = (words - r.head_words) >> 2;
  r.tail = p + r.head_words + 4 * r.n_quads;
  r.tail_words = words - r.head_words - 4 * r.n_quads;
  r.value = value;
  return r;
}

// Fills `words` 32-bit words with `value` (the initialisation of states and
// mates that opens Algorithm 1). Any 4-byte alignment.
__global__ void fill_u32_kernel(FillRegion r) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint4 vv = make_uint4(r.value, r.value, r.value, r.value);
  for (int64_t j = t; j < r.n_quads; j += stride) r.quads[j] = vv;
  if (t < r.head_words) r.head[t] = r.value;
  if (t < r.tail_words) r.tail[t] = r.value;
}

// Two fills in one launch: the output and the states of a relabelled pass.
__global__ void fill2_u32_kernel(FillRegion a, FillRegion b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint4 va = make_uint4(a.value, a.value, a.value, a.value);
  const uint4 vb = make_uint4(b.value, b.value, b.value, b.value);
  for (int64_t j = t; j < a.n_quads + b.n_quads; j += stride) {
    if (j < a.n_quads)
      a.quads[j] = va;
    else
      b.quads[j - a.n_quads] = vb;
  }
  if (t < a.head_words) a.head[t] = a.value;
  if (t < a.tail_words) a.tail[t] = a.value;
  if (t < b.head_words) b.head[t] = b.value;
  if (t < b.tail_words) b.tail[t] = b.value;
}

// Rewrites every word equal to `from` as `to` (word layout, two-phase
// encoding, without lazy output: vertices left accessible become -1).
__global__ void replace_u32_kernel(uint32_t* __restrict__ p, int64_t words, uint32_t from,
                                   uint32_t to) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < words; j += stride)
    if (p[j] == from) p[j] = to;
}

// CSR well-formedness (checked at create with MM_VALIDATE). Bits of *flags:
// 1 offsets[0] != 0 or offsets[n] != m; 2 offsets decrease; 4 neighbour out
// of range.
template <typename OffT>
__global__ void validate_kernel(const OffT* __restrict__ off, const int32_t* __restrict__ nbr,
                                int64_t n, int64_t m, uint32_t* flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t f = 0;
  if (t == 0 && ((int64_t)off[0] != 0 || (int64_t)off[n] != m)) f |= 1u;
  for (int64_t v = t; v < n; v += stride)
    if (off[v + 1] < off[v]) f |= 2u;
  for (int64_t j = t; j < m; j += stride) {
    const int32_t y = nbr[j];
    if (y < 0 || (int64_t)y >= n) f |= 4u;
  }
  if (f) atomicOr(flags, f);
}

// One graph: wavefront w < main_waves sweeps sources [v_begin + w *
// wave_vertices, ...); the wavefronts after them (dispatched last) take the
// hub tier's pieces, as one launch with the main pass: 64 to a wavefront, each
// swept by one lane, or (hub_wave) each live one by the whole wavefront.
// chunk_count (device, or null): the number of pieces when only the device
// knows it (the table was filled by this pass's own stream); n_chunks is then
// the table's capacity, which sizes the grid.
template <typename OffT, class Layout, bool HINT, bool LAZY, bool STATS>
__device__ __forceinline__ void sweep_graph(SweepParams p, const OffT* __restrict__ off,
                                            const int32_t* __restrict__ nbr, int64_t n,
                                            int64_t v_begin, int64_t main_waves, int64_t n_chunks,
                                            const unsigned long long* chunk_count, Layout L,
                                            unsigned long long* stats) {
  // the workgroup tier's slots (pieces.h), cleared before any wavefront of
  // the workgroup reads them
  __shared__ int32_t seen[4];
  if (p.hub_wave == 2) {
    if (threadIdx.x < 4) seen[threadIdx.x] = -1;
    __syncthreads();
  }
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int64_t vb, nv;
  if (wave < main_waves) {
    vb = v_begin + wave * p.wave_vertices;
    if (vb >= n) return;
    nv = (n - vb < p.wave_vertices) ? (n - vb) : p.wave_vertices;
    p.chunks = nullptr;
  } else {
    if (chunk_count) {
      const int64_t c = (int64_t)*chunk_count;
      n_chunks = c < n_chunks ? c : n_chunks;
    }
    const int64_t per = kPiecesPerWave;
    vb = (wave - main_waves) * per;
    if (vb >= n_chunks) return;
    nv = (n_chunks - vb < per) ? (n_chunks - vb) : per;
    p.wave_vertices = 64;
    p.disperse = 0;
    p.hub_degree = 0;
    if (p.hub_wave) {
      Counters<STATS> cnt;
      if (p.hub_wave == 2)
        sweep_pieces_wave<Layout, HINT, STATS>(p, nbr, L, vb, nv, cnt, seen, (int)(blockDim.x >> 6));
      else
        sweep_pieces_wave<Layout, HINT, STATS>(p, nbr, L, vb, nv, cnt);
      if (STATS) cnt.flush(stats);
      return;
    }
  }
  __shared__ QSlot queues[4][kQueue];  // one ring per wavefront (wg_size <= 256)
  Counters<STATS> cnt;
  sweep_block<OffT, Layout, HINT, LAZY, STATS>(p, off, nbr, L, vb, nv, queues[threadIdx.x >> 6],
                                               cnt);
  if (STATS) cnt.flush(stats);
}

template <typename OffT, class Layout, bool HINT, bool LAZY, bool STATS>
__global__ __launch_bounds__(256) void sweep_kernel(SweepParams p, const OffT* __restrict__ off,
                                                   const int32_t* __restrict__ nbr, int64_t n,
                                                   int64_t v_begin, int64_t main_waves,
                                                   int64_t n_chunks,
                                                   const unsigned long long* chunk_count, Layout L,
                                                   unsigned long long* stats) {
  sweep_graph<OffT, Layout, HINT, LAZY, STATS>(p, off, nbr, n, v_begin, main_waves, n_chunks,
                                               chunk_count, L, stats);
}

// The same sweep compiled for at least six wavefronts per SIMD (tuning
// occupancy = 6): at most 80 VGPRs, where the compiler alone takes 81 and
// gets five. The lanes' chains of dependent memory operations are the
// bound, so more wavefronts hide more of their latency; the graph's share in
// flight grows too. Instantiated only for the sweeps that fit without spills
// (not relabelled, not instrumented).
template <typename OffT, class Layout, bool HINT, bool LAZY, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void sweep_kernel_w6(
    SweepParams p, const OffT* __restrict__ off, const int32_t* __restrict__ nbr, int64_t n,
    int64_t v_begin, int64_t main_waves, int64_t n_chunks, const unsigned long long* chunk_count,
    Layout L, unsigned long long* stats) {
  sweep_graph<OffT, Layout, HINT, LAZY, STATS>(p, off, nbr, n, v_begin, main_waves, n_chunks,
                                               chunk_count, L, stats);
}

// A graph swept whole by one wavefront, its states in that wavefront's LDS
// (dynamic, whole_lds_words(n) words).
template <typename OffT, bool STATS>
__global__ __launch_bounds__(64) void whole_lds_kernel(SweepParams p, const OffT* __restrict__ off,
                                                       const int32_t* __restrict__ nbr, int64_t n,
                                                       int32_t* mate, unsigned long long* stats) {
  __shared__ QSlot q[kQueue];
  extern __shared__ uint32_t st[];
  Counters<STATS> cnt;
  sweep_whole_lds<OffT, STATS>(p, off, nbr, n, mate, st, q, cnt);
  if (STATS) cnt.flush(stats);
}

// ---------------------------------------------------------------- helpers

int grid_for(int64_t words) {
  int64_t blocks = (words / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  return (int)blocks;
}

}  // namespace

// Ring of event pairs bracketing sweep launches (MM_TIMING handles).
struct TimingRing {
  static constexpr int kCap = 512;
  hipEvent_t ev[2 * kCap] = {};
  int64_t recorded = 0;  // launches recorded since the last read
  hipError_t init() {
    for (int i = 0; i < 2 * kCap; ++i) {
      hipError_t e = hipEventCreate(&ev[i]);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  void destroy() {
    for (int i = 0; i < 2 * kCap; ++i)
      if (ev[i]) hipEventDestroy(ev[i]);
  }
  hipEvent_t before() const { return ev[2 * (recorded % kCap)]; }
  hipEvent_t after() const { return ev[2 * (recorded % kCap) + 1]; }
};

struct mm_graph {
  const void* off;
  int off64;
  const int32_t* nbr;
  int64_t n, m;
  uint8_t* ws;
  size_t ws_bytes;
  uint32_t flags;
  mm_tuning tun;
  bool lazy;  // effective lazy output
  int device;
  TimingRing* timing;
  mmk::HubChunk* chunks = nullptr;  // hub tier table (device, owned), or null
  int64_t n_chunks = 0;
  // mm_run_static: the pieces are counted on the device (n_chunks is then the
  // table's capacity), and the loop-budget flag may go to the caller's word
  const unsigned long long* chunk_count = nullptr;
  uint32_t* err_out = nullptr;
  // with a hub table: recorded on the create stream once the table is
  // filled (every run waits for it), and on the run stream after each run
  // (the destroy call orders the table's release after it)
  hipEvent_t table_ready = nullptr;
  hipEvent_t last_run = nullptr;
  bool relabel;         // sweep the graph relabelled by degree (relabel.hip)
  mmi::RelabelView rl;  // its arrays, in the workspace
  int32_t* rl_state;    // word-layout states in the new ids (relabel only)
  uint32_t* st() const { return reinterpret_cast<uint32_t*>(ws + kCtrlBytes); }
  uint32_t* hint() const {
    return tun.hint ? reinterpret_cast<uint32_t*>(ws + kCtrlBytes + mmi::state_bytes(n, tun))
                    : nullptr;
  }
};

namespace mmi {
int64_t handle_n(const mm_graph* h) { return h->n; }
int handle_off64(const mm_graph* h) { return h->off64; }
const void* handle_off(const mm_graph* h) { return h->off; }
const int32_t* handle_nbr(const mm_graph* h) { return h->nbr; }
uint8_t* handle_ws(const mm_graph* h) { return h->ws; }
uint32_t handle_flags(const mm_graph* h) { return h->flags; }
}  // namespace mmi

namespace {


// Sources the sweep visits: all vertices, or, relabelled, those with entries.
int64_t sweep_begin(const mm_graph* g) { return g->relabel ? g->rl.n_isolated : 0; }

SweepParams make_params(const mm_graph* g) {
  SweepParams p;
  p.wave_vertices = g->tun.wave_vertices;
  p.disperse = g->tun.disperse;
  p.assist_after = g->tun.assist_after;
  p.scan_width = g->tun.scan_width;
  p.stream_loads = g->tun.stream_loads;
  p.wait_release = g->tun.wait_release;
  p.upper_only = (g->tun.upper_only && (g->flags & MM_SYMMETRIC)) ? 1 : 0;
  p.hub_wave = g->tun.hub_wave;
  // the copy holds each short list's neighbours above its vertex first
  p.lower_stop = (g->tun.order_lists == 2 && p.upper_only) ? (int32_t)mmi::kOrderedMax : 0;
  p.probe_first = g->tun.probe_first;
  p.iter_cap = g->tun.iter_cap;
  p.err = g->err_out ? g->err_out : reinterpret_cast<uint32_t*>(g->ws);
  p.hub_degree = g->n_chunks > 0 ? g->tun.hub_degree : 0;
  p.hub_chunk = g->tun.hub_chunk;
  p.chunks = nullptr;
  const int64_t ns = g->n - sweep_begin(g);
  if (ns <= g->tun.whole_graph_vertices) {  // one wavefront takes the whole graph
    p.wave_vertices = std::max<int64_t>(64, (ns + 63) / 64 * 64);
    // lanes stride apart: one wavefront alone is bound by its loop trips, and
    // lanes on adjacent vertices (neighbours in a mesh) would wait on each
    // other's reservations
    p.disperse = 1;
  } else {
    // a small graph alone on the GPU: shorter blocks
    p.wave_vertices = mmi::short_blocks(ns, p.wave_vertices, g->tun.min_waves);
  }
  return p;
}

// Whether the sweep keeps the states in LDS (whole.h): a graph swept whole,
// small enough, not relabelled. The same rule as for batch members.
bool whole_in_lds(const mm_graph* g) {
  return g->tun.whole_graph_lds && !g->relabel && g->n > 0 && g->n <= g->tun.whole_graph_vertices &&
         g->n <= MM_LDS_WHOLE_MAX;
}

template <typename OffT, bool STATS>
hipError_t launch_whole_lds(const mm_graph* g, const SweepParams& p, int32_t* mate,
                            unsigned long long* stats, hipStream_t s) {
  const size_t shmem = sizeof(uint32_t) * (size_t)whole_lds_words(g->n);
  hipLaunchKernelGGL((whole_lds_kernel<OffT, STATS>), dim3(1), dim3(64), shmem, s, p,
                     static_cast<const OffT*>(g->off), g->nbr, g->n, mate, stats);
  return hipGetLastError();
}

template <typename OffT, class Layout, bool HINT, bool LAZY, bool STATS>
hipError_t launch_sweep(const mm_graph* g, const Layout& L, hipStream_t s) {
  const SweepParams p = make_params(g);
  unsigned long long* stats = reinterpret_cast<unsigned long long*>(g->ws + kStatsOffset);
  if constexpr (!Layout::kRelabelled) {
    if (whole_in_lds(g)) {
      if (g->timing) {
        hipError_t e = hipEventRecord(g->timing->before(), s);
        if (e != hipSuccess) return e;
      }
      hipError_t e = launch_whole_lds<OffT, STATS>(g, p, L.mate, stats, s);
      if (e == hipSuccess && g->timing) {
        e = hipEventRecord(g->timing->after(), s);
        ++g->timing->recorded;
      }
      return e;
    }
  }
  const int64_t v_begin = sweep_begin(g);
  const OffT* off = g->relabel ? reinterpret_cast<const OffT*>(g->rl.off)
                               : static_cast<const OffT*>(g->off);
  const int32_t* nbr = g->relabel ? g->rl.nbr : g->nbr;
  const int64_t waves = (g->n - v_begin + p.wave_vertices - 1) / p.wave_vertices;
  // the hub tier's pieces: 64 to a wavefront, after the main pass's waves
  const int64_t per = kPiecesPerWave;
  const int64_t chunk_waves = (g->n_chunks + per - 1) / per;
  SweepParams pl = p;
  pl.chunks = g->chunks;
  const int wpb = g->tun.wg_size / 64;
  const int64_t blocks = (waves + chunk_waves + wpb - 1) / wpb;
  if (blocks == 0) return hipSuccess;
  if (g->timing) {
    hipError_t e = hipEventRecord(g->timing->before(), s);
    if (e != hipSuccess) return e;
  }
  void (*kernel)(SweepParams, const OffT*, const int32_t*, int64_t, int64_t, int64_t, int64_t,
                 const unsigned long long*, Layout, unsigned long long*) =
      sweep_kernel<OffT, Layout, HINT, LAZY, STATS>;
  if constexpr (!Layout::kRelabelled && !STATS) {
    if (g->tun.occupancy == 6) kernel = sweep_kernel_w6<OffT, Layout, HINT, LAZY, STATS>;
  }
  hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(g->tun.wg_size), 0, s, pl, off, nbr, g->n,
                     v_begin, waves, g->n_chunks, g->chunk_count, L, stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g->timing) {
    e = hipEventRecord(g->timing->after(), s);
    ++g->timing->recorded;
  }
  return e;
}

template <typename OffT, class Layout, bool STATS>
hipError_t dispatch_flags(const mm_graph* g, const Layout& L, hipStream_t s) {
  const bool hint = g->tun.hint != 0;
  if constexpr (Layout::kStateIsMate && !Layout::kTwoPhase) {
    // ACC is already the output value -1: no lazy output is needed.
    return hint ? launch_sweep<OffT, Layout, true, false, STATS>(g, L, s)
                : launch_sweep<OffT, Layout, false, false, STATS>(g, L, s);
  } else {
    if (hint)
      return g->lazy ? launch_sweep<OffT, Layout, true, true, STATS>(g, L, s)
                     : launch_sweep<OffT, Layout, true, false, STATS>(g, L, s);
    return g->lazy ? launch_sweep<OffT, Layout, false, true, STATS>(g, L, s)
                   : launch_sweep<OffT, Layout, false, false, STATS>(g, L, s);
  }
}

void fill(uint32_t* p, int64_t words, uint32_t value, hipStream_t s) {
  if (words > 0)
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(words)), dim3(256), 0, s,
                       fill_region(p, words, value));
}

// Relabelled graph: states in the new ids, output written in the given ids
// (filled with -1 first). The relabelled offsets are int64.
template <bool STATS>
hipError_t run_relabelled(const mm_graph* g, int32_t* out, hipStream_t s) {
  const int64_t n = g->n;
  Hint hint{g->hint(), hint_lg(g->tun.hint)};
  if (hint.bits) fill(hint.bits, hint_words(n, g->tun.hint), 0u, s);
  if (g->tun.layout != MM_LAYOUT_U32) fill(reinterpret_cast<uint32_t*>(out), n, 0xffffffffu, s);
  const bool two = g->tun.protocol == MM_PROTOCOL_TWO_PHASE;
  const int32_t* orig = g->rl.orig;
  if (g->tun.layout == MM_LAYOUT_U32) {
    // On symmetric input an isolated vertex is nobody's neighbour, so the
    // states from the first vertex with entries (rounded down to 4) suffice.
    const int64_t s0 = (g->flags & MM_SYMMETRIC) ? (g->rl.n_isolated & ~(int64_t)3) : 0;
    uint32_t* st = reinterpret_cast<uint32_t*>(g->rl_state) + s0;
    const uint32_t acc = two ? LayoutU32<true>::kAcc : LayoutU32<false>::kAcc;
    hipLaunchKernelGGL(fill2_u32_kernel, dim3(grid_for(2 * n - s0)), dim3(256), 0, s,
                       fill_region(reinterpret_cast<uint32_t*>(out), n, 0xffffffffu),
                       fill_region(st, n - s0, acc));
    if (two) {
      using L = Relabelled<LayoutU32<true>>;
      return dispatch_flags<int64_t, L, STATS>(g, L{{g->rl_state, hint}, out, orig}, s);
    }
    using L = Relabelled<LayoutU32<false>>;
    return dispatch_flags<int64_t, L, STATS>(g, L{{g->rl_state, hint}, out, orig}, s);
  }
  // packed layouts keep their mate entries in the new ids too (in the region
  // the word layout uses for its states); the wrapper writes the output
  int32_t* mate_new = g->rl_state;
  if (g->tun.layout == MM_LAYOUT_U2) {
    fill(g->st(), (n + 15) / 16, 0u, s);
    using LT = Relabelled<LayoutPacked<2, true>>;
    using LC = Relabelled<LayoutPacked<2, false>>;
    if (two) return dispatch_flags<int64_t, LT, STATS>(g, LT{{g->st(), mate_new, hint}, out, orig}, s);
    return dispatch_flags<int64_t, LC, STATS>(g, LC{{g->st(), mate_new, hint}, out, orig}, s);
  }
  fill(g->st(), (n + 3) / 4, 0u, s);
  using LT = Relabelled<LayoutPacked<8, true>>;
  using LC = Relabelled<LayoutPacked<8, false>>;
  if (two) return dispatch_flags<int64_t, LT, STATS>(g, LT{{g->st(), mate_new, hint}, out, orig}, s);
  return dispatch_flags<int64_t, LC, STATS>(g, LC{{g->st(), mate_new, hint}, out, orig}, s);
}

template <typename OffT, bool STATS>
hipError_t run_typed(const mm_graph* g, int32_t* mate, hipStream_t s) {
  const int64_t n = g->n;
  uint32_t* mate_w = reinterpret_cast<uint32_t*>(mate);
  Hint hint{g->hint(), hint_lg(g->tun.hint)};
  if (hint.bits) fill(hint.bits, hint_words(n, g->tun.hint), 0u, s);
  const bool two = g->tun.protocol == MM_PROTOCOL_TWO_PHASE;
  hipError_t e;
  if (g->tun.layout == MM_LAYOUT_U32) {
    if (two) {
      fill(mate_w, n, LayoutU32<true>::kAcc, s);
      e = dispatch_flags<OffT, LayoutU32<true>, STATS>(g, LayoutU32<true>{mate, hint}, s);
      if (e == hipSuccess && !g->lazy) {
        hipLaunchKernelGGL(replace_u32_kernel, dim3(grid_for(n)), dim3(256), 0, s, mate_w, n,
                           LayoutU32<true>::kAcc, 0xffffffffu);
        e = hipGetLastError();
      }
      return e;
    }
    fill(mate_w, n, LayoutU32<false>::kAcc, s);
    return dispatch_flags<OffT, LayoutU32<false>, STATS>(g, LayoutU32<false>{mate, hint}, s);
  }
  if (!g->lazy) fill(mate_w, n, 0xffffffffu, s);
  if (g->tun.layout == MM_LAYOUT_U2) {
    fill(g->st(), (n + 15) / 16, 0u, s);
    using L2T = LayoutPacked<2, true>;
    using L2C = LayoutPacked<2, false>;
    if (two) return dispatch_flags<OffT, L2T, STATS>(g, L2T{g->st(), mate, hint}, s);
    return dispatch_flags<OffT, L2C, STATS>(g, L2C{g->st(), mate, hint}, s);
  }
  fill(g->st(), (n + 3) / 4, 0u, s);
  using L8T = LayoutPacked<8, true>;
  using L8C = LayoutPacked<8, false>;
  if (two) return dispatch_flags<OffT, L8T, STATS>(g, L8T{g->st(), mate, hint}, s);
  return dispatch_flags<OffT, L8C, STATS>(g, L8C{g->st(), mate, hint}, s);
}

}  // namespace

// ---------------------------------------------------------------- static scratch
// The working memory of mm_run_static: the control block (error word, hub
// piece cursor), then the packed states and the matched hint when the tuning
// has them, then the hub piece table. Each device holds its own copy from
// module load until the process ends. In host code `scratch` names a host-side
// stand-in, never the device memory: kernels get the address
// hipGetSymbolAddress returns for the current device (static_scratch below).
constexpr size_t kStaticScratchBytes = MM_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
mm_status static_scratch(uint8_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MM_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MM_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch[dev];
  return MM_OK;
}

}  // namespace

extern "C" {

const char* mm_version(void) { return "skipper-gfx950 0.3"; }

const char* mm_last_error(void) { return g_last_error.c_str(); }

void mm_default_tuning(mm_tuning* t) {
  if (!t) return;
  std::memset(t, 0, sizeof(*t));
  // Fastest measured on R-MAT scale 25 and 27 (MI355X): the word layout (the
  // state is the output, no separate fill), Algorithm 1's CAS on v, eager
  // output, wavefront assist after 64 ids.
  t->layout = MM_LAYOUT_U32;
  t->protocol = MM_PROTOCOL_CAS;
  t->hint = 0;
  t->wg_size = 256;
  t->wave_vertices = 1024;
  t->disperse = 0;
  t->assist_after = 64;
  t->lazy_init = 0;
  t->scan_width = 4;
  t->whole_graph_vertices = 16384;
  t->hub_degree = 4096;
  t->hub_chunk = 256;
  t->whole_graph_lds = 1;
  // a small graph alone keeps about 32 wavefronts in flight: fewer sources
  // racing at once, so repeated passes give matchings of nearly the same size
  t->upper_only = 0;
  // long lists' pieces swept by whole wavefronts once their source is seen
  // free: as fast as one lane a piece on R-MAT (0.3% faster in interleaved
  // runs), and twice as fast where a long list is still live
  t->hub_wave = 1;
  t->min_waves = 32;
  t->hot_degree = 2048;
  t->order_lists = 0;
  t->probe_first = 0;
  t->occupancy = 0;
  t->iter_cap = 0;
}

size_t mm_workspace_bytes_graph(int64_t n, int64_t m, const mm_tuning* tp) {
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (n < 0 || m < 0 || check_tuning(t) != MM_OK || n > mmi::max_vertices(t)) return 0;
  size_t b = kCtrlBytes + mmi::state_bytes(n, t) + mmi::hint_bytes(n, t);
  if (t.relabel) b += mmi::round_up(sizeof(int32_t) * (size_t)n, 256) + mmi::relabel_bytes(n, m);
  if (t.order_lists) b += mmi::round_up(sizeof(int32_t) * (size_t)m, 256);
  return b;
}

size_t mm_workspace_bytes(int64_t n, const mm_tuning* tp) {
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (t.relabel || t.order_lists) return 0;  // the copy depends on m
  return mm_workspace_bytes_graph(n, 0, &t);
}

size_t mm_create_device_bytes(int64_t n, int64_t m, const mm_tuning* tp) {
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (n < 0 || n > INT32_MAX || m < 0 || check_tuning(t) != MM_OK) return 0;
  size_t b = 0;
  // the hub table (kept until destroy); a graph swept whole gets none
  if (n > t.whole_graph_vertices) {
    const int64_t pieces = mmi::hub_pieces_bound(m, t.hub_degree, t.hub_chunk);
    if (pieces > 0) b += mmi::round_up(sizeof(mmk::HubChunk) * (size_t)pieces, 256);
  }
  // the relabelling's temporaries (freed before create returns)
  if (t.relabel) b += mmi::relabel_temp_bytes(n);
  // the list reordering's degree buckets (freed before create returns)
  if (t.order_lists) b += mmi::order_temp_bytes(n);
  return b;
}

mm_status mm_create(const void* offsets, mm_offset_type off_type, const int32_t* neighbors,
                    int64_t n, int64_t m, void* workspace, size_t workspace_bytes, uint32_t flags,
                    const mm_tuning* tuning, void* stream, mm_handle* out) {
  if (!out) return fail(MM_ERR_INVALID_ARG, "out handle pointer is null");
  *out = nullptr;
  if (off_type != MM_OFF_I32 && off_type != MM_OFF_I64)
    return fail(MM_ERR_INVALID_ARG, "off_type must be MM_OFF_I32 or MM_OFF_I64");
  if (n < 0 || n > INT32_MAX)
    return fail(MM_ERR_INVALID_ARG, "n = %lld out of [0, 2^31-1]", (long long)n);
  if (m < 0) return fail(MM_ERR_INVALID_ARG, "m = %lld is negative", (long long)m);
  if (off_type == MM_OFF_I32 && m > INT32_MAX)
    return fail(MM_ERR_INVALID_ARG, "m = %lld does not fit int32 offsets", (long long)m);
  if (!offsets) return fail(MM_ERR_INVALID_ARG, "offsets is null");
  if (!neighbors && m > 0) return fail(MM_ERR_INVALID_ARG, "neighbors is null");
  if (!workspace) return fail(MM_ERR_INVALID_ARG, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(MM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (flags & ~(uint32_t)(MM_VALIDATE | MM_SYMMETRIC | MM_STATS | MM_TIMING))
    return fail(MM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  mm_tuning t;
  if (tuning) t = *tuning; else mm_default_tuning(&t);
  mm_status st = check_tuning(t);
  if (st != MM_OK) return st;
  if (n > mmi::max_vertices(t))
    return fail(MM_ERR_INVALID_ARG, "n = %lld: the word layout with the two-phase protocol "
                "takes at most 2^31-2 vertices", (long long)n);
  const size_t need = mm_workspace_bytes_graph(n, m, &t);
  if (workspace_bytes < need)
    return fail(MM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, needs %zu", workspace_bytes, need);

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
  if (flags & MM_VALIDATE) {
    uint32_t* f = reinterpret_cast<uint32_t*>(ws);
    int64_t work = n > m ? n : m;
    int blocks = (int)((work + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    if (off_type == MM_OFF_I64)
      hipLaunchKernelGGL((validate_kernel<int64_t>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const int64_t*>(offsets), neighbors, n, m, f);
    else
      hipLaunchKernelGGL((validate_kernel<int32_t>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const int32_t*>(offsets), neighbors, n, m, f);
    HIP_TRY(hipGetLastError());
    uint32_t hf = 0;
    HIP_TRY(hipMemcpyAsync(&hf, f, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
    if (hf) {
      return fail(MM_ERR_INVALID_GRAPH, "invalid CSR:%s%s%s",
                  (hf & 1u) ? " offsets[0] != 0 or offsets[n] != m;" : "",
                  (hf & 2u) ? " offsets decrease;" : "",
                  (hf & 4u) ? " neighbour id out of [0, n);" : "");
    }
  }
  mmi::RelabelView rl{};
  int32_t* rl_state = nullptr;
  if (t.relabel) {
    const size_t base = kCtrlBytes + mmi::state_bytes(n, t) + mmi::hint_bytes(n, t);
    rl_state = reinterpret_cast<int32_t*>(ws + base);
    uint8_t* region = ws + base + mmi::round_up(sizeof(int32_t) * (size_t)n, 256);
    hipError_t e = mmi::build_relabel(offsets, off_type == MM_OFF_I64, neighbors, n, m, t.relabel,
                                      t.hot_degree, region, &rl, s);
    if (e != hipSuccess) return fail(MM_ERR_HIP, "relabelling failed: %s", hipGetErrorString(e));
  }
  const int32_t* sweep_nbr = neighbors;
  if (t.order_lists && m > 0) {
    int32_t* copy = reinterpret_cast<int32_t*>(ws + kCtrlBytes + mmi::state_bytes(n, t) +
                                               mmi::hint_bytes(n, t));
    hipError_t e = mmi::build_ordered_lists(offsets, off_type == MM_OFF_I64, neighbors, n,
                                            t.order_lists == 2, copy, s);
    if (e != hipSuccess) return fail(MM_ERR_HIP, "ordering the lists failed: %s", hipGetErrorString(e));
    sweep_nbr = copy;
  }
  mm_graph* g = new (std::nothrow) mm_graph();
  if (!g) return fail(MM_ERR_OUT_OF_MEMORY, "host allocation of the handle failed");
  g->relabel = t.relabel != 0;
  g->rl = rl;
  g->rl_state = rl_state;
  g->off = offsets;
  g->off64 = off_type == MM_OFF_I64;
  g->nbr = sweep_nbr;  // the reordered copy with order_lists
  g->n = n;
  g->m = m;
  g->ws = ws;
  g->ws_bytes = workspace_bytes;
  g->flags = flags;
  g->tun = t;
  // Lazy output is only sound when every edge is in both endpoints' lists
  // and both endpoints examine it, and when no hub piece can hold part of a
  // source's list (a piece cannot finalise its source). The last condition
  // is decided from the tuning and the sizes, as mm_run_static decides it
  // without counting the pieces, so that both entry points run the same
  // kernels for the same graph and tuning.
  const bool may_have_pieces = n > t.whole_graph_vertices &&
                               mmi::hub_pieces_bound(m, t.hub_degree, t.hub_chunk) > 0;
  g->lazy = t.lazy_init && (flags & MM_SYMMETRIC) && !t.relabel && !t.upper_only &&
            !may_have_pieces && !(t.layout == MM_LAYOUT_U32 && t.protocol == MM_PROTOCOL_CAS);
  // a graph swept whole by one wavefront gets no hub pieces (as in batches)
  if (t.hub_degree > 0 && m > t.hub_degree && n > t.whole_graph_vertices) {
    // the table is built on the lists the sweep reads (relabelled or given)
    hipError_t e = g->relabel
        ? mmi::build_hub_chunks(g->rl.off, 1, n, t.hub_degree, t.hub_chunk, ws, &g->chunks,
                                &g->n_chunks, s)
        : mmi::build_hub_chunks(offsets, off_type == MM_OFF_I64, n, t.hub_degree, t.hub_chunk, ws,
                                &g->chunks, &g->n_chunks, s);
    if (e != hipSuccess) {
      delete g;
      return fail(MM_ERR_HIP, "building the hub table failed: %s", hipGetErrorString(e));
    }
    if (g->n_chunks > 0) {
      g->lazy = false;  // a piece of a list cannot finalise its source
      hipError_t e1 = hipEventCreateWithFlags(&g->table_ready, hipEventDisableTiming);
      if (e1 == hipSuccess) e1 = hipEventCreateWithFlags(&g->last_run, hipEventDisableTiming);
      if (e1 == hipSuccess) e1 = hipEventRecord(g->table_ready, s);
      if (e1 != hipSuccess) {
        if (g->table_ready) hipEventDestroy(g->table_ready);
        if (g->last_run) hipEventDestroy(g->last_run);
        mmi::free_owned(g->chunks);
        delete g;
        return fail(MM_ERR_HIP, "hub table events: %s", hipGetErrorString(e1));
      }
    }
  }
  g->device = dev;
  g->timing = nullptr;
  if (flags & MM_TIMING) {
    g->timing = new (std::nothrow) TimingRing();
    if (!g->timing) {
      mm_destroy(g);
      return fail(MM_ERR_OUT_OF_MEMORY, "host allocation of the timing ring failed");
    }
    hipError_t e = g->timing->init();
    if (e != hipSuccess) {
      mm_destroy(g);
      return fail(MM_ERR_HIP, "hipEventCreate failed: %s", hipGetErrorString(e));
    }
  }
  *out = g;
  return MM_OK;
}

mm_status mm_run(mm_handle g, void* stream, int32_t* match_out) {
  if (!g) return fail(MM_ERR_INVALID_ARG, "handle is null");
  if (!match_out && g->n > 0) return fail(MM_ERR_INVALID_ARG, "match_out is null");
  if (g->n == 0) return MM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool stats = (g->flags & MM_STATS) != 0;
  hipError_t e;
  // the hub table was filled on the create call's stream
  if (g->table_ready) HIP_TRY(hipStreamWaitEvent(s, g->table_ready, 0));
  if (g->relabel)
    e = stats ? run_relabelled<true>(g, match_out, s) : run_relabelled<false>(g, match_out, s);
  else if (g->off64)
    e = stats ? run_typed<int64_t, true>(g, match_out, s) : run_typed<int64_t, false>(g, match_out, s);
  else
    e = stats ? run_typed<int32_t, true>(g, match_out, s) : run_typed<int32_t, false>(g, match_out, s);
  if (e != hipSuccess) return fail(MM_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  if (g->last_run) HIP_TRY(hipEventRecord(g->last_run, s));
  return MM_OK;
}

mm_status mm_run_static(const void* offsets, mm_offset_type off_type, const int32_t* neighbors,
                        int64_t n, int64_t m, uint32_t flags, const mm_tuning* tuning, void* stream,
                        int32_t* match_out, uint32_t* status_out) {
  if (off_type != MM_OFF_I32 && off_type != MM_OFF_I64)
    return fail(MM_ERR_INVALID_ARG, "off_type must be MM_OFF_I32 or MM_OFF_I64");
  if (n < 0 || n > INT32_MAX)
    return fail(MM_ERR_INVALID_ARG, "n = %lld out of [0, 2^31-1]", (long long)n);
  if (m < 0) return fail(MM_ERR_INVALID_ARG, "m = %lld is negative", (long long)m);
  if (off_type == MM_OFF_I32 && m > INT32_MAX)
    return fail(MM_ERR_INVALID_ARG, "m = %lld does not fit int32 offsets", (long long)m);
  if (!offsets) return fail(MM_ERR_INVALID_ARG, "offsets is null");
  if (!neighbors && m > 0) return fail(MM_ERR_INVALID_ARG, "neighbors is null");
  if (!match_out && n > 0) return fail(MM_ERR_INVALID_ARG, "match_out is null");
  if (flags & ~(uint32_t)MM_SYMMETRIC)
    return fail(MM_ERR_UNSUPPORTED, "mm_run_static takes MM_SYMMETRIC only (flags 0x%x)", flags);
  mm_tuning t;
  if (tuning) t = *tuning; else mm_default_tuning(&t);
  mm_status st = check_tuning(t);
  if (st != MM_OK) return st;
  if (n > mmi::max_vertices(t))
    return fail(MM_ERR_INVALID_ARG, "n = %lld: the word layout with the two-phase protocol "
                "takes at most 2^31-2 vertices", (long long)n);
  if (t.relabel)
    return fail(MM_ERR_UNSUPPORTED, "mm_run_static: tuning.relabel needs a workspace (mm_create)");
  if (t.order_lists)
    return fail(MM_ERR_UNSUPPORTED, "mm_run_static: tuning.order_lists needs a workspace (mm_create)");
  // what the pass needs of the scratch, as mm_create's workspace would hold it
  const size_t base = kCtrlBytes + mmi::state_bytes(n, t) + mmi::hint_bytes(n, t);
  const int64_t pieces =
      n > t.whole_graph_vertices ? mmi::hub_pieces_bound(m, t.hub_degree, t.hub_chunk) : 0;
  const size_t need = base + round_up(sizeof(mmk::HubChunk) * (size_t)pieces, 256);
  if (need > kStaticScratchBytes)
    return fail(MM_ERR_OUT_OF_MEMORY,
                "mm_run_static: this graph and tuning need %zu bytes of the static scratch, which "
                "holds %zu (states %zu, hint %zu, hub pieces up to %lld); the word layout needs no "
                "state array, hint = 0 no hint, hub_degree = 0 no piece table",
                need, kStaticScratchBytes, mmi::state_bytes(n, t), mmi::hint_bytes(n, t),
                (long long)pieces);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the caller's status word starts at 0 (a fill kernel, so that the call can
  // be captured into a graph)
  if (status_out) {
    fill(status_out, 1, 0u, s);
    HIP_TRY(hipGetLastError());
  }
  if (n == 0) return MM_OK;
  uint8_t* ws = nullptr;
  st = static_scratch(&ws);
  if (st != MM_OK) return st;
  // the control block starts at zero: error word, hub piece cursor
  fill(reinterpret_cast<uint32_t*>(ws), (int64_t)(kCtrlBytes / 4), 0u, s);
  HIP_TRY(hipGetLastError());
  mm_graph g;
  g.off = offsets;
  g.off64 = off_type == MM_OFF_I64;
  g.nbr = neighbors;
  g.n = n;
  g.m = m;
  g.ws = ws;
  g.ws_bytes = kStaticScratchBytes;
  g.flags = flags;
  g.tun = t;
  g.device = 0;
  g.timing = nullptr;
  g.relabel = false;
  g.rl = mmi::RelabelView{};
  g.rl_state = nullptr;
  g.err_out = status_out;
  // the same rule as mm_create's
  g.lazy = t.lazy_init && (flags & MM_SYMMETRIC) && pieces == 0 && !t.upper_only &&
           !(t.layout == MM_LAYOUT_U32 && t.protocol == MM_PROTOCOL_CAS);
  if (pieces > 0) {
    auto* cursor = reinterpret_cast<unsigned long long*>(ws + mmi::kHubOffset);
    g.chunks = reinterpret_cast<mmk::HubChunk*>(ws + base);
    g.n_chunks = pieces;  // capacity: the sweep reads the count from the cursor
    g.chunk_count = cursor;
    HIP_TRY(mmi::fill_hub_chunks(offsets, g.off64, n, t.hub_degree, t.hub_chunk, cursor, g.chunks, s));
  }
  hipError_t e = g.off64 ? run_typed<int64_t, false>(&g, match_out, s)
                         : run_typed<int32_t, false>(&g, match_out, s);
  if (e != hipSuccess) return fail(MM_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return MM_OK;
}

mm_status mm_sync(mm_handle g, void* stream) {
  if (!g) return fail(MM_ERR_INVALID_ARG, "handle is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, g->ws, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err) {
    HIP_TRY(hipMemsetAsync(g->ws, 0, sizeof(uint32_t), s));
    HIP_TRY(hipStreamSynchronize(s));
    return fail(MM_ERR_NO_PROGRESS, "a wavefront exceeded its loop-trip budget (%lld%s)",
                (long long)g->tun.iter_cap, g->tun.iter_cap ? "" : ": per-block default");
  }
  return MM_OK;
}

mm_status mm_get_stats(mm_handle g, void* stream, mm_stats* out) {
  if (!g || !out) return fail(MM_ERR_INVALID_ARG, "null argument");
  if (!(g->flags & MM_STATS)) return fail(MM_ERR_UNSUPPORTED, "handle was created without MM_STATS");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long c[kStatWords] = {};
  HIP_TRY(hipMemcpyAsync(c, g->ws + kStatsOffset, sizeof(c), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  mmi::stats_from_counters(c, out);
  return MM_OK;
}

mm_status mm_reset_stats(mm_handle g, void* stream) {
  if (!g) return fail(MM_ERR_INVALID_ARG, "handle is null");
  HIP_TRY(hipMemsetAsync(g->ws + kStatsOffset, 0, kStatWords * sizeof(unsigned long long),
                         static_cast<hipStream_t>(stream)));
  return MM_OK;
}

mm_status mm_get_timing(mm_handle g, int64_t* count, double* total_ms, double* min_ms,
                        double* max_ms) {
  if (!g || !count || !total_ms) return fail(MM_ERR_INVALID_ARG, "null argument");
  if (!g->timing) return fail(MM_ERR_UNSUPPORTED, "handle was created without MM_TIMING");
  TimingRing& r = *g->timing;
  const int64_t have = r.recorded < TimingRing::kCap ? r.recorded : TimingRing::kCap;
  double tot = 0.0, lo = 0.0, hi = 0.0;
  for (int64_t k = r.recorded - have; k < r.recorded; ++k) {
    const int slot = (int)(k % TimingRing::kCap);
    HIP_TRY(hipEventSynchronize(r.ev[2 * slot + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.ev[2 * slot], r.ev[2 * slot + 1]));
    tot += ms;
    if (k == r.recorded - have || ms < lo) lo = ms;
    if (k == r.recorded - have || ms > hi) hi = ms;
  }
  r.recorded = 0;
  *count = have;
  *total_ms = tot;
  if (min_ms) *min_ms = lo;
  if (max_ms) *max_ms = hi;
  return MM_OK;
}

void mm_destroy(mm_handle g) {
  if (!g) return;
  // the table is released, stream-ordered, after the last run that reads it
  if (g->last_run) hipStreamWaitEvent(nullptr, g->last_run, 0);
  mmi::free_owned(g->chunks);
  if (g->table_ready) hipEventDestroy(g->table_ready);
  if (g->last_run) hipEventDestroy(g->last_run);
  if (g->timing) {
    g->timing->destroy();
    delete g->timing;
  }
  delete g;
}

}  // extern "C"

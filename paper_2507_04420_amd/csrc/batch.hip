// Batched matching: many independent graphs in one persistent launch.
//
// Every graph is described by a GraphDesc (its offsets, neighbours, vertex
// count, and where its states, hint and mate entries live). The work is a
// table of items (graph, first source, source count), each the size of one
// wavefront block of the single-graph sweep. A persistent grid of wavefronts
// pops items from a device counter and runs the same sweep_block on each, so
// a thousand small graphs fill the GPU as well as one large graph does. Graphs
// swept whole with their states in LDS run first, in a kernel of their own
// (whole.h); mesh-like members get blocks of their own length with dispersed
// lanes. The per-pass work (state fill, queue reset, LDS kernel, persistent
// sweep, output fix-up) can be captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "internal.h"
#include "mm.h"
#include "pieces.h"
#include "sweep.h"
#include "whole.h"

using namespace mmk;
using mmi::fail;
using mmi::kCtrlBytes;
using mmi::kHubOffset;
using mmi::kQueueOffset;
using mmi::kStatsOffset;
using mmi::round_up;
#define HIP_TRY MMI_HIP_TRY

namespace mmb {

namespace {

__global__ void fill_words_kernel(uint32_t* __restrict__ p, int64_t words, uint32_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < words; j += stride)
    p[j] = value;
}

__global__ void replace_words_kernel(uint32_t* __restrict__ p, int64_t words, uint32_t from,
                                     uint32_t to) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < words; j += stride)
    if (p[j] == from) p[j] = to;
}

__global__ void reset_queue_kernel(uint32_t* queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

// Per-graph CSR check of a batch: offsets non-decreasing inside each graph,
// neighbour ids local to their graph. Thread per global vertex; the graph of a
// vertex is found by binary search over the vertex-offset table.
__global__ void validate_batch_kernel(const int64_t* __restrict__ off, const int32_t* __restrict__ nbr,
                                      const int64_t* __restrict__ vtx_off, int32_t num_graphs,
                                      int64_t N, int64_t M, uint32_t* flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t f = 0;
  if (t == 0 && (off[0] != 0 || off[N] != M)) f |= 1u;
  for (int64_t v = t; v < N; v += stride) {
    int lo = 0, hi = num_graphs;  // find g with vtx_off[g] <= v < vtx_off[g+1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (vtx_off[mid] <= v) lo = mid; else hi = mid;
    }
    const int64_t ng = vtx_off[lo + 1] - vtx_off[lo];
    const int64_t b = off[v], e = off[v + 1];
    if (e < b || b < 0 || e > M) {  // never read outside the M entries
      f |= 2u;
      continue;
    }
    for (int64_t j = b; j < e; ++j) {
      const int32_t y = nbr[j];
      if (y < 0 || (int64_t)y >= ng) f |= 4u;
    }
  }
  if (f) atomicOr(flags, f);
}

// The same check for a list batch, through the descriptors. A graph's own
// offsets must start at 0 and end at its entry count.
__global__ void validate_list_kernel(const GraphDesc* __restrict__ descs,
                                     const int64_t* __restrict__ vtx_off, int32_t num_graphs,
                                     int64_t N, uint32_t* flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t f = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
    int lo = 0, hi = num_graphs;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (vtx_off[mid] <= v) lo = mid; else hi = mid;
    }
    const GraphDesc d = descs[lo];
    const int64_t x = v - vtx_off[lo];
    const int64_t b = d.off[x], e = d.off[x + 1];
    if ((x == 0 && b != 0) || (x == d.n - 1 && e != d.m)) f |= 1u;
    if (e < b || b < 0 || e > d.m) {
      f |= 2u;
      continue;
    }
    for (int64_t j = b; j < e; ++j) {
      const int32_t y = d.nbr[j];
      if (y < 0 || (int64_t)y >= d.n) f |= 4u;
    }
  }
  if (f) atomicOr(flags, f);
}

template <class Layout>
__device__ __forceinline__ Layout layout_of(const GraphDesc& d, int32_t* mate);
template <>
__device__ __forceinline__ LayoutU32<false> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutU32<false>{mate + d.v0, Hint{d.hint, d.hint_lg}};
}
template <>
__device__ __forceinline__ LayoutU32<true> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutU32<true>{mate + d.v0, Hint{d.hint, d.hint_lg}};
}
template <>
__device__ __forceinline__ LayoutPacked<8, false> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutPacked<8, false>{d.st, mate + d.v0, Hint{d.hint, d.hint_lg}};
}
template <>
__device__ __forceinline__ LayoutPacked<8, true> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutPacked<8, true>{d.st, mate + d.v0, Hint{d.hint, d.hint_lg}};
}
template <>
__device__ __forceinline__ LayoutPacked<2, false> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutPacked<2, false>{d.st, mate + d.v0, Hint{d.hint, d.hint_lg}};
}
template <>
__device__ __forceinline__ LayoutPacked<2, true> layout_of(const GraphDesc& d, int32_t* mate) {
  return LayoutPacked<2, true>{d.st, mate + d.v0, Hint{d.hint, d.hint_lg}};
}

// Persistent sweep: every wavefront pops items until the table is exhausted;
// each item is one sweep_block of one graph. Every wavefront reaches the exit
// (the counter only grows, and each item's sweep has its own trip budget).
template <class Layout, bool HINT, bool LAZY, bool STATS>
__global__ __launch_bounds__(256) void batch_sweep_kernel(SweepParams p,
                                                         const GraphDesc* __restrict__ descs,
                                                         const WorkItem* __restrict__ items,
                                                         int64_t n_items, int32_t* mate,
                                                         uint32_t* queue,
                                                         unsigned long long* stats) {
  __shared__ QSlot queues[4][kQueue];
  Counters<STATS> cnt;
  const int lane = (int)(threadIdx.x & 63);
  while (true) {
    uint32_t it = 0;
    if (lane == 0)
      it = __hip_atomic_fetch_add(queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    it = (uint32_t)__builtin_amdgcn_readfirstlane((int)it);
    if ((int64_t)it >= n_items) break;
    const WorkItem w = items[it];
    const GraphDesc d = descs[w.desc];
    const Layout L = layout_of<Layout>(d, mate);
    SweepParams pp = p;
    int64_t nv = w.nv;
    if (nv < 0) {  // hub pieces (never with lazy output: the plan turns it off)
      nv = -nv;
      pp.wave_vertices = 64;
      pp.disperse = 0;
      pp.hub_degree = 0;
      if (pp.hub_wave) {
        sweep_pieces_wave<Layout, HINT, STATS>(pp, d.nbr, L, w.vb, nv, cnt);
        continue;
      }
    } else {
      pp.chunks = nullptr;
      if (d.flags & kWholeGraph) {  // as mm_run sweeps a graph whole
        pp.hub_degree = 0;
        pp.disperse = 1;
      } else if (d.flags & kMesh) {
        pp.disperse = 1;
      }
    }
    sweep_block<int64_t, Layout, HINT, LAZY, STATS>(pp, d.off, d.nbr, L, w.vb, nv,
                                                    queues[threadIdx.x >> 6], cnt);
  }
  if (STATS) cnt.flush(stats);
}

// Graphs flagged kWholeLds, one wavefront each, their states in LDS
// (whole.h): lds_words words of the dynamic LDS per wavefront. A kernel of its
// own, so that the persistent sweep keeps its register budget.
template <bool STATS>
__global__ __launch_bounds__(256) void batch_whole_lds_kernel(SweepParams p,
                                                             const GraphDesc* __restrict__ descs,
                                                             const WorkItem* __restrict__ items,
                                                             int64_t n_items, int32_t* mate,
                                                             unsigned long long* stats,
                                                             int32_t lds_words) {
  __shared__ QSlot queues[4][kQueue];
  extern __shared__ uint32_t whole_st[];
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (wave >= n_items) return;
  Counters<STATS> cnt;
  const GraphDesc d = descs[items[wave].desc];
  sweep_whole_lds<int64_t, STATS>(p, d.off, d.nbr, d.n, mate + d.v0,
                                  whole_st + (int64_t)(threadIdx.x >> 6) * lds_words,
                                  queues[threadIdx.x >> 6], cnt);
  if (STATS) cnt.flush(stats);
}

int grid_for(int64_t words) {
  int64_t blocks = (words + 1023) / 1024;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  return (int)blocks;
}

template <class Layout, bool HINT, bool LAZY, bool STATS>
hipError_t launch_persistent(const BatchPlan& bp, hipStream_t s) {
  auto kern = batch_sweep_kernel<Layout, HINT, LAZY, STATS>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, bp.wg_size, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const int wpb = bp.wg_size / 64;
  int64_t blocks = (int64_t)per_cu * bp.num_cus;
  const int64_t need = (bp.n_items + wpb - 1) / wpb;
  if (blocks > need) blocks = need;
  if (blocks < 1) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(bp.wg_size), 0, s, bp.params, bp.descs,
                     bp.items, bp.n_items, bp.mate, bp.queue, bp.stats);
  return hipGetLastError();
}

template <class Layout, bool STATS>
hipError_t launch_flags(const BatchPlan& bp, hipStream_t s) {
  if constexpr (Layout::kStateIsMate && !Layout::kTwoPhase) {
    return bp.hint ? launch_persistent<Layout, true, false, STATS>(bp, s)
                   : launch_persistent<Layout, false, false, STATS>(bp, s);
  } else {
    if (bp.hint)
      return bp.lazy ? launch_persistent<Layout, true, true, STATS>(bp, s)
                     : launch_persistent<Layout, true, false, STATS>(bp, s);
    return bp.lazy ? launch_persistent<Layout, false, true, STATS>(bp, s)
                   : launch_persistent<Layout, false, false, STATS>(bp, s);
  }
}

void fill(uint32_t* p, int64_t words, uint32_t v, hipStream_t s) {
  if (words > 0) hipLaunchKernelGGL(fill_words_kernel, dim3(grid_for(words)), dim3(256), 0, s, p, words, v);
}

template <bool STATS>
hipError_t launch_whole_lds(const BatchPlan& bp, hipStream_t s) {
  if (bp.n_lds == 0) return hipSuccess;
  const int wpb = bp.lds_wg / 64;
  const size_t shmem = (size_t)wpb * (size_t)bp.lds_words * 4;
  const int64_t blocks = (bp.n_lds + wpb - 1) / wpb;
  hipLaunchKernelGGL((batch_whole_lds_kernel<STATS>), dim3((unsigned)blocks), dim3(bp.lds_wg),
                     shmem, s, bp.params, bp.descs, bp.lds_items, bp.n_lds, bp.mate, bp.stats,
                     bp.lds_words);
  return hipGetLastError();
}

template <bool STATS>
hipError_t enqueue_typed(const BatchPlan& bp, hipStream_t s) {
  uint32_t* mate_w = reinterpret_cast<uint32_t*>(bp.mate);
  if (bp.hint) fill(bp.hint_base, bp.hint_words, 0u, s);
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, bp.queue);
  const bool two = bp.protocol == MM_PROTOCOL_TWO_PHASE;
  // init (the start of Algorithm 1) for every graph; the graphs kept in LDS then
  // overwrite their own mates, ahead of the persistent sweep of the rest
  if (bp.layout == MM_LAYOUT_U32) {
    fill(mate_w, bp.N, two ? LayoutU32<true>::kAcc : LayoutU32<false>::kAcc, s);
  } else {
    fill(bp.st_base, bp.st_words, 0u, s);
    if (!bp.lazy) fill(mate_w, bp.N, 0xffffffffu, s);
  }
  hipError_t e = launch_whole_lds<STATS>(bp, s);
  if (e != hipSuccess) return e;
  if (bp.layout == MM_LAYOUT_U32) {
    if (two) {
      e = launch_flags<LayoutU32<true>, STATS>(bp, s);
      if (e == hipSuccess && !bp.lazy) {
        hipLaunchKernelGGL(replace_words_kernel, dim3(grid_for(bp.N)), dim3(256), 0, s, mate_w,
                           bp.N, LayoutU32<true>::kAcc, 0xffffffffu);
        e = hipGetLastError();
      }
      return e;
    }
    return launch_flags<LayoutU32<false>, STATS>(bp, s);
  }
  if (bp.layout == MM_LAYOUT_U2)
    return two ? launch_flags<LayoutPacked<2, true>, STATS>(bp, s)
               : launch_flags<LayoutPacked<2, false>, STATS>(bp, s);
  return two ? launch_flags<LayoutPacked<8, true>, STATS>(bp, s)
             : launch_flags<LayoutPacked<8, false>, STATS>(bp, s);
}

}  // namespace

hipError_t enqueue_pass(const BatchPlan& bp, hipStream_t s) {
  return bp.stats_on ? enqueue_typed<true>(bp, s) : enqueue_typed<false>(bp, s);
}

hipError_t validate_batch(const int64_t* off, const int32_t* nbr, const int64_t* vtx_off_dev,
                          int32_t num_graphs, int64_t N, int64_t M, uint32_t* flags, hipStream_t s) {
  int64_t blocks = (N + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(validate_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, s, off, nbr,
                     vtx_off_dev, num_graphs, N, M, flags);
  return hipGetLastError();
}

hipError_t validate_list(const GraphDesc* descs, const int64_t* vtx_off_dev, int32_t num_graphs,
                         int64_t N, uint32_t* flags, hipStream_t s) {
  int64_t blocks = (N + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(validate_list_kernel, dim3((unsigned)blocks), dim3(256), 0, s, descs,
                     vtx_off_dev, num_graphs, N, flags);
  return hipGetLastError();
}

int64_t state_words_for(int64_t n, int32_t layout) {
  if (layout == MM_LAYOUT_U8) return (n + 3) / 4;
  if (layout == MM_LAYOUT_U2) return (n + 15) / 16;
  return 0;
}

}  // namespace mmb

// ---------------------------------------------------------------- C ABI

namespace {

struct BatchLayout {  // byte offsets of the workspace pieces after the control block
  size_t descs, items, vtx, st, hint, total;
  int64_t n_items, st_words, hint_words;
  int64_t wave_vertices, mesh_wave_vertices;  // block lengths (shortened for a small batch)
};

bool plan_layout(int32_t G, const int64_t* vtx_off, const mm_tuning& t, BatchLayout* out) {
  int64_t n_items = 0, st_words = 0, hint_words = 0;
  // sources swept in blocks (graphs not swept whole): too few of them for
  // min_waves wavefronts, and the blocks get shorter, as for a single graph
  int64_t blocked = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t n = vtx_off[g + 1] - vtx_off[g];
    if (n < 0 || n > mmi::max_vertices(t)) return false;
    if (n > t.whole_graph_vertices) blocked += n;
  }
  const int64_t wv_main = mmi::short_blocks(blocked, t.wave_vertices, t.min_waves);
  const int64_t wv_mesh =
      t.mesh_wave_vertices > 0 ? mmi::short_blocks(blocked, t.mesh_wave_vertices, t.min_waves) : 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t n = vtx_off[g + 1] - vtx_off[g];
    // mesh graphs may take shorter blocks: room for the shorter of the two
    const int64_t wv = wv_mesh > 0 ? std::min(wv_main, wv_mesh) : wv_main;
    n_items += n <= t.whole_graph_vertices ? (n > 0) : (n + wv - 1) / wv;
    st_words += mmb::state_words_for(n, t.layout);
    hint_words += mmk::hint_words(n, t.hint);
  }
  BatchLayout L;
  L.wave_vertices = wv_main;
  L.mesh_wave_vertices = wv_mesh;
  L.n_items = n_items;
  L.st_words = st_words;
  L.hint_words = hint_words;
  size_t off = kCtrlBytes;
  L.descs = off;
  off += round_up(sizeof(mmb::GraphDesc) * (size_t)(G > 0 ? G : 1), 256);
  L.items = off;
  off += round_up(sizeof(mmb::WorkItem) * (size_t)(n_items > 0 ? n_items : 1), 256);
  L.vtx = off;
  off += round_up(sizeof(int64_t) * (size_t)(G + 1), 256);
  L.st = off;
  off += round_up((size_t)st_words * 4, 256);
  L.hint = off;
  off += round_up((size_t)hint_words * 4, 256);
  L.total = off;
  *out = L;
  return true;
}

}  // namespace


struct mm_batch {
  int32_t G;
  int64_t N;
  uint8_t* ws;
  uint32_t flags;
  mm_tuning tun;
  BatchLayout lay;
  std::vector<int64_t> vtx_off;
  mmb::BatchPlan plan;
  int32_t* bound_mate = nullptr;  // output the captured pass writes to
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mmk::HubChunk* chunks = nullptr;  // hub piece table, inside `own`
  void* own = nullptr;  // item and piece tables when hub pieces exist (device, owned)
  hipEvent_t last_run = nullptr;  // with `own`: recorded after each run, waited for at destroy
};

namespace {

void drop_graph(mm_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Checks shared by both create forms; fills the tuning to use.
mm_status common_args(void* workspace, uint32_t flags, const mm_tuning* tuning, mm_tuning* t,
                      mm_batch_handle* out) {
  if (!out) return fail(MM_ERR_INVALID_ARG, "out handle pointer is null");
  *out = nullptr;
  if (!workspace) return fail(MM_ERR_INVALID_ARG, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(MM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (flags & ~(uint32_t)(MM_VALIDATE | MM_SYMMETRIC | MM_STATS | MM_TIMING | MM_CAPTURE))
    return fail(MM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  if (tuning) *t = *tuning; else mm_default_tuning(t);
  const mm_status st = mmi::check_tuning(*t);
  if (st != MM_OK) return st;
  if (t->relabel) return fail(MM_ERR_UNSUPPORTED, "tuning.relabel applies to single graphs only");
  if (t->order_lists)
    return fail(MM_ERR_UNSUPPORTED, "tuning.order_lists applies to single graphs only");
  return MM_OK;
}

// Completes a handle whose descriptors carry off, nbr, n, m and v0: places the
// states and hints, uploads descriptors, vertex table and work items, runs the
// optional device validation (concatenated or list form) and waits for it.
mm_status finish_create(std::vector<mmb::GraphDesc>& descs, const std::vector<int64_t>& vtx,
                        const BatchLayout& lay, const mm_tuning& t, uint8_t* ws,
                        size_t workspace_bytes, uint32_t flags, hipStream_t s,
                        const int64_t* concat_off, const int32_t* concat_nbr, int64_t M,
                        mm_batch_handle* out) {
  if (workspace_bytes < lay.total)
    return fail(MM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, needs %zu", workspace_bytes, lay.total);
  const int32_t G = (int32_t)descs.size();
  const int64_t N = vtx[G];
  uint32_t* st_base = reinterpret_cast<uint32_t*>(ws + lay.st);
  uint32_t* hint_base = reinterpret_cast<uint32_t*>(ws + lay.hint);
  int64_t st_w = 0, hint_w = 0;
  std::vector<mmb::WorkItem> items;
  items.reserve((size_t)lay.n_items);
  // graphs swept whole keep their states in LDS when they fit (whole.h); the
  // choice depends on the graph and the tuning only, never on the rest of
  // the batch
  int64_t lds_words = 0;
  std::vector<mmb::WorkItem> lds_items;  // placed after all other items
  for (int32_t g = 0; g < G; ++g) {
    mmb::GraphDesc& d = descs[g];
    d.st = t.layout == MM_LAYOUT_U32 ? nullptr : st_base + st_w;
    d.hint = t.hint ? hint_base + hint_w : nullptr;
    d.hint_lg = mmk::hint_lg(t.hint);
    d.flags = d.n <= t.whole_graph_vertices ? mmb::kWholeGraph : 0u;
    if ((d.flags & mmb::kWholeGraph) && t.whole_graph_lds && d.n > 0 && d.n <= MM_LDS_WHOLE_MAX) {
      d.flags |= mmb::kWholeLds;
      lds_words = std::max(lds_words, mmk::whole_lds_words(d.n));
    }
    st_w += mmb::state_words_for(d.n, t.layout);
    hint_w += mmk::hint_words(d.n, t.hint);
  }
  auto* descs_dev = reinterpret_cast<mmb::GraphDesc*>(ws + lay.descs);
  auto* items_dev = reinterpret_cast<mmb::WorkItem*>(ws + lay.items);
  auto* vtx_dev = reinterpret_cast<int64_t*>(ws + lay.vtx);
  uint32_t* f = reinterpret_cast<uint32_t*>(ws);
  HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
  if (G > 0)
    HIP_TRY(hipMemcpyAsync(descs_dev, descs.data(), sizeof(mmb::GraphDesc) * G,
                           hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(vtx_dev, vtx.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
  if (flags & MM_VALIDATE) {
    if (concat_off)
      HIP_TRY(mmb::validate_batch(concat_off, concat_nbr, vtx_dev, G, N, M, f, s));
    else
      HIP_TRY(mmb::validate_list(descs_dev, vtx_dev, G, N, f, s));
  }
  // hub tier, first pass: pieces per graph, counted beside the validation so
  // that a batch without long lists pays no further wait or allocation
  bool hubs_possible = false;
  if (t.hub_degree > 0)
    for (int32_t g = 0; g < G && !hubs_possible; ++g)
      hubs_possible = !(descs[g].flags & mmb::kWholeGraph) && descs[g].n > 0 &&
                      (descs[g].m < 0 || descs[g].m > t.hub_degree);
  if (hubs_possible)
    HIP_TRY(mmb::count_batch_hubs(descs_dev, vtx_dev, G, N, t.hub_degree, t.hub_chunk, ws, s));
  // meshes (no list longer than kMeshDegree) get their own block length
  const bool find_meshes = t.mesh_wave_vertices > 0;
  if (find_meshes) HIP_TRY(mmb::batch_find_meshes(descs_dev, vtx_dev, G, N, s));
  uint32_t hf = 0;
  unsigned long long n_pieces = 0;
  HIP_TRY(hipMemcpyAsync(&hf, f, sizeof(hf), hipMemcpyDeviceToHost, s));
  if (hubs_possible)
    HIP_TRY(hipMemcpyAsync(&n_pieces, ws + kHubOffset, sizeof(n_pieces), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));  // the host vectors are released after this
  if (hf) {
    HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
    HIP_TRY(hipStreamSynchronize(s));
    return fail(MM_ERR_INVALID_GRAPH, "invalid batch CSR:%s%s%s",
                (hf & 1u) ? (concat_off ? " offsets[0] != 0 or offsets[N] != M;"
                                        : " a graph's offsets do not run from 0 to m;")
                          : "",
                (hf & 2u) ? " offsets decrease;" : "",
                (hf & 4u) ? " neighbour id outside its graph;" : "");
  }
  const int64_t n_chunks = (int64_t)n_pieces;
  if (G > 0 && (n_chunks > 0 || find_meshes)) {  // per-graph results of the counting kernels
    HIP_TRY(hipMemcpyAsync(descs.data(), descs_dev, sizeof(mmb::GraphDesc) * G,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  // work items: a small graph is one item (one wavefront), a larger one an
  // item per block; a mesh's blocks are shorter, and its lanes dispersed
  bool descs_changed = false;
  for (int32_t g = 0; g < G; ++g) {
    mmb::GraphDesc& d = descs[g];
    int64_t step = lay.wave_vertices;
    if (d.flags & mmb::kWholeGraph) {
      step = d.n;
    } else if (find_meshes && !d.not_mesh) {
      d.flags |= mmb::kMesh;
      step = lay.mesh_wave_vertices;
      descs_changed = true;
    }
    for (int64_t vb = 0; vb < d.n; vb += step) {
      mmb::WorkItem w;
      w.desc = g;
      w.vb = vb;
      w.nv = (int32_t)std::min<int64_t>(step, d.n - vb);
      (d.flags & mmb::kWholeLds ? lds_items : items).push_back(w);
    }
  }
  if (descs_changed && n_chunks == 0)
    HIP_TRY(hipMemcpyAsync(descs_dev, descs.data(), sizeof(mmb::GraphDesc) * G,
                           hipMemcpyHostToDevice, s));
  // second pass, only when pieces exist: they become work items of their own
  // after the blocks, in one allocation the handle owns (item table, then
  // piece table)
  mmk::HubChunk* chunks = nullptr;
  void* own = nullptr;
  if (n_chunks > 0) {
    int64_t first = 0;
    for (int32_t g = 0; g < G; ++g) {
      const int64_t k = descs[g].pieces;
      const int64_t per = mmk::kPiecesPerWave;  // pieces per item
      for (int64_t c = 0; c < k; c += per) {
        mmb::WorkItem w;
        w.desc = g;
        w.vb = first + c;
        w.nv = -(int32_t)std::min<int64_t>(per, k - c);
        items.push_back(w);
      }
      descs[g].pieces = first;
      first += k;
    }
    const size_t items_bytes =
        round_up(sizeof(mmb::WorkItem) * (items.size() + lds_items.size()), 256);
    hipError_t e = hipMallocAsync(&own, items_bytes + sizeof(mmk::HubChunk) * (size_t)n_chunks, s);
    if (e != hipSuccess)
      return fail(MM_ERR_OUT_OF_MEMORY, "hub item and piece tables: %s", hipGetErrorString(e));
    items_dev = static_cast<mmb::WorkItem*>(own);
    chunks = reinterpret_cast<mmk::HubChunk*>(static_cast<uint8_t*>(own) + items_bytes);
    e = hipMemcpyAsync(descs_dev, descs.data(), sizeof(mmb::GraphDesc) * G, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = mmb::fill_batch_hubs(descs_dev, vtx_dev, G, N, t.hub_degree, t.hub_chunk, chunks, s);
    if (e != hipSuccess) {
      mmi::free_owned(own);
      return fail(MM_ERR_HIP, "building the hub table failed: %s", hipGetErrorString(e));
    }
  }
  const int64_t n_main = (int64_t)items.size();
  items.insert(items.end(), lds_items.begin(), lds_items.end());
  if (!items.empty()) {
    hipError_t e = hipMemcpyAsync(items_dev, items.data(), sizeof(mmb::WorkItem) * items.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host vector is released after this
    if (e != hipSuccess) {
      mmi::free_owned(own);
      return fail(MM_ERR_HIP, "uploading the work items failed: %s", hipGetErrorString(e));
    }
  }
  int cus = 0, dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  mm_batch* b = new (std::nothrow) mm_batch();
  if (!b) {
    mmi::free_owned(own);
    return fail(MM_ERR_OUT_OF_MEMORY, "host allocation of the batch handle failed");
  }
  b->chunks = chunks;
  b->own = own;
  if (own) {
    hipError_t e = hipEventCreateWithFlags(&b->last_run, hipEventDisableTiming);
    if (e != hipSuccess) {
      mm_batch_destroy(b);
      return fail(MM_ERR_HIP, "batch event: %s", hipGetErrorString(e));
    }
  }
  if (flags & MM_CAPTURE) {
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      mm_batch_destroy(b);
      return fail(MM_ERR_HIP, "capture stream: %s", hipGetErrorString(e));
    }
  }
  b->G = G;
  b->N = N;
  b->ws = ws;
  b->flags = flags;
  b->tun = t;
  b->lay = lay;
  b->vtx_off = vtx;
  mmb::BatchPlan& p = b->plan;
  p.params.wave_vertices = lay.wave_vertices;
  p.params.disperse = t.disperse;
  p.params.assist_after = t.assist_after;
  p.params.scan_width = t.scan_width;
  p.params.stream_loads = t.stream_loads;
  p.params.wait_release = t.wait_release;
  p.params.upper_only = (t.upper_only && (flags & MM_SYMMETRIC)) ? 1 : 0;
  p.params.hub_wave = t.hub_wave;
  p.params.lower_stop = 0;  // no reordered copy of a batch's lists
  p.params.probe_first = t.probe_first;
  p.params.iter_cap = t.iter_cap;
  p.params.hub_degree = n_chunks > 0 ? t.hub_degree : 0;
  p.params.hub_chunk = t.hub_chunk;
  p.params.chunks = chunks;
  p.params.err = f;
  p.descs = descs_dev;
  p.items = items_dev;
  p.n_items = n_main;
  p.lds_items = items_dev + n_main;
  p.n_lds = (int64_t)lds_items.size();
  p.queue = reinterpret_cast<uint32_t*>(ws + kQueueOffset);
  p.stats = reinterpret_cast<unsigned long long*>(ws + kStatsOffset);
  p.layout = t.layout;
  p.protocol = t.protocol;
  p.hint = t.hint != 0;
  p.lazy = t.lazy_init && (flags & MM_SYMMETRIC) && n_chunks == 0 && !t.upper_only &&
           !(t.layout == MM_LAYOUT_U32 && t.protocol == MM_PROTOCOL_CAS);
  p.stats_on = (flags & MM_STATS) != 0;
  p.wg_size = t.wg_size;
  p.num_cus = cus > 0 ? cus : 1;
  p.mate = nullptr;
  p.N = N;
  p.st_base = st_base;
  p.st_words = lay.st_words;
  p.hint_base = hint_base;
  p.lds_words = (int32_t)((lds_words + 3) / 4 * 4);  // 16-byte aligned regions
  p.lds_wg = t.wg_size;
  if (p.lds_words > 0) {
    // fewer wavefronts per workgroup if their LDS regions and the queues do
    // not fit one workgroup's LDS (results do not depend on the group size)
    int max_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t fixed = (int64_t)sizeof(mmk::QSlot) * mmk::kQueue * 4;
    p.lds_wg = t.wg_size;
    while (p.lds_wg > 64 && fixed + (int64_t)(p.lds_wg / 64) * p.lds_words * 4 > max_lds)
      p.lds_wg -= 64;
    if (fixed + (int64_t)p.lds_words * 4 > max_lds) {
      mm_batch_destroy(b);
      return fail(MM_ERR_UNSUPPORTED, "LDS per workgroup (%d bytes) too small for whole-graph "
                  "states; set tuning.whole_graph_lds = 0", max_lds);
    }
  }
  p.hint_words = lay.hint_words;
  *out = b;
  return MM_OK;
}

}  // namespace

extern "C" {

size_t mm_batch_workspace_bytes(int32_t num_graphs, const int64_t* vtx_off, const mm_tuning* tp) {
  if (num_graphs < 0 || !vtx_off) return 0;
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (mmi::check_tuning(t) != MM_OK || t.relabel || t.order_lists) return 0;
  BatchLayout L;
  if (!plan_layout(num_graphs, vtx_off, t, &L)) return 0;
  return L.total;
}

size_t mm_batch_create_device_bytes(int32_t num_graphs, const int64_t* vtx_off, int64_t M,
                                    const mm_tuning* tp) {
  if (num_graphs < 0 || !vtx_off || M < 0) return 0;
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (mmi::check_tuning(t) != MM_OK || t.relabel || t.order_lists) return 0;
  BatchLayout L;
  if (!plan_layout(num_graphs, vtx_off, t, &L)) return 0;
  bool blocked = false;  // a graph not swept whole: the only kind with pieces
  for (int32_t g = 0; g < num_graphs && !blocked; ++g)
    blocked = vtx_off[g + 1] - vtx_off[g] > t.whole_graph_vertices;
  const int64_t pieces = blocked ? mmi::hub_pieces_bound(M, t.hub_degree, t.hub_chunk) : 0;
  if (pieces == 0) return 0;
  // the item table moves to the handle's own allocation, with one item per
  // run of 64 pieces of a graph (at most pieces / 64 + num_graphs of them),
  // followed by the piece table
  const int64_t per = mmk::kPiecesPerWave;
  const int64_t items = L.n_items + pieces / per + num_graphs;
  return round_up(sizeof(mmb::WorkItem) * (size_t)items, 256) +
         round_up(sizeof(mmk::HubChunk) * (size_t)pieces, 256);
}

mm_status mm_batch_create(const int64_t* offsets_cat, const int32_t* neighbors_cat,
                          const int64_t* vtx_off, int32_t num_graphs, int64_t M, void* workspace,
                          size_t workspace_bytes, uint32_t flags, const mm_tuning* tuning,
                          void* stream, mm_batch_handle* out) {
  mm_tuning t;
  mm_status st = common_args(workspace, flags, tuning, &t, out);
  if (st != MM_OK) return st;
  if (num_graphs < 0) return fail(MM_ERR_INVALID_ARG, "num_graphs is negative");
  if (!vtx_off) return fail(MM_ERR_INVALID_ARG, "vtx_off is null");
  if (!offsets_cat) return fail(MM_ERR_INVALID_ARG, "offsets is null");
  if (!neighbors_cat && M > 0) return fail(MM_ERR_INVALID_ARG, "neighbors is null");
  if (M < 0) return fail(MM_ERR_INVALID_ARG, "M is negative");
  if (vtx_off[0] != 0) return fail(MM_ERR_INVALID_ARG, "vtx_off[0] must be 0");
  for (int32_t g = 0; g < num_graphs; ++g)
    if (vtx_off[g + 1] < vtx_off[g] || vtx_off[g + 1] - vtx_off[g] > INT32_MAX)
      return fail(MM_ERR_INVALID_ARG, "vtx_off must be non-decreasing with graphs of < 2^31 vertices");
  BatchLayout lay;
  if (!plan_layout(num_graphs, vtx_off, t, &lay))
    return fail(MM_ERR_INVALID_ARG, "a graph has more vertices than the layout allows");
  std::vector<int64_t> vtx(vtx_off, vtx_off + num_graphs + 1);
  std::vector<mmb::GraphDesc> descs((size_t)num_graphs);
  for (int32_t g = 0; g < num_graphs; ++g) {
    mmb::GraphDesc& d = descs[g];
    d.off = offsets_cat + vtx[g];
    d.nbr = neighbors_cat;
    d.n = vtx[g + 1] - vtx[g];
    d.m = -1;
    d.v0 = vtx[g];
  }
  return finish_create(descs, vtx, lay, t, static_cast<uint8_t*>(workspace), workspace_bytes,
                       flags, static_cast<hipStream_t>(stream), offsets_cat, neighbors_cat, M, out);
}

mm_status mm_batch_create_list(const int64_t* const* offsets, const int32_t* const* neighbors,
                               const int64_t* n, const int64_t* m, int32_t num_graphs,
                               void* workspace, size_t workspace_bytes, uint32_t flags,
                               const mm_tuning* tuning, void* stream, mm_batch_handle* out) {
  mm_tuning t;
  mm_status st = common_args(workspace, flags, tuning, &t, out);
  if (st != MM_OK) return st;
  if (num_graphs < 0) return fail(MM_ERR_INVALID_ARG, "num_graphs is negative");
  if (num_graphs > 0 && (!offsets || !neighbors || !n || !m))
    return fail(MM_ERR_INVALID_ARG, "a per-graph array is null");
  std::vector<int64_t> vtx((size_t)num_graphs + 1, 0);
  std::vector<mmb::GraphDesc> descs((size_t)num_graphs);
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (n[g] < 0 || n[g] > INT32_MAX) return fail(MM_ERR_INVALID_ARG, "graph %d: n out of range", g);
    if (m[g] < 0 || (n[g] == 0 && m[g] != 0))
      return fail(MM_ERR_INVALID_ARG, "graph %d: m out of range", g);
    if (n[g] > 0 && !offsets[g]) return fail(MM_ERR_INVALID_ARG, "graph %d: offsets is null", g);
    if (m[g] > 0 && !neighbors[g]) return fail(MM_ERR_INVALID_ARG, "graph %d: neighbors is null", g);
    vtx[g + 1] = vtx[g] + n[g];
    mmb::GraphDesc& d = descs[g];
    d.off = offsets[g];
    d.nbr = neighbors[g];
    d.n = n[g];
    d.m = m[g];
    d.v0 = vtx[g];
  }
  BatchLayout lay;
  if (!plan_layout(num_graphs, vtx.data(), t, &lay))
    return fail(MM_ERR_INVALID_ARG, "a graph has more vertices than the layout allows");
  return finish_create(descs, vtx, lay, t, static_cast<uint8_t*>(workspace), workspace_bytes,
                       flags, static_cast<hipStream_t>(stream), nullptr, nullptr, 0, out);
}

mm_status mm_batch_run(mm_batch_handle b, void* stream, int32_t* match_out) {
  if (!b) return fail(MM_ERR_INVALID_ARG, "batch handle is null");
  if (!match_out && b->N > 0) return fail(MM_ERR_INVALID_ARG, "match_out is null");
  if (b->plan.n_items + b->plan.n_lds == 0) return MM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (match_out != b->bound_mate) {  // a captured pass is tied to its output
    b->plan.mate = match_out;
    b->bound_mate = match_out;
    drop_graph(b);
  }
  if (b->flags & MM_CAPTURE) {
    if (!b->exec) {
      HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = mmb::enqueue_pass(b->plan, b->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return fail(MM_ERR_HIP, "capturing the batch pass failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      b->graph = g;
      HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(b->exec, s));
    if (b->last_run) HIP_TRY(hipEventRecord(b->last_run, s));
    return MM_OK;
  }
  hipError_t e = mmb::enqueue_pass(b->plan, s);
  if (e != hipSuccess) return fail(MM_ERR_HIP, "batch launch failed: %s", hipGetErrorString(e));
  if (b->last_run) HIP_TRY(hipEventRecord(b->last_run, s));
  return MM_OK;
}

mm_status mm_batch_sync(mm_batch_handle b, void* stream) {
  if (!b) return fail(MM_ERR_INVALID_ARG, "batch handle is null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, b->ws, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err) {
    HIP_TRY(hipMemsetAsync(b->ws, 0, sizeof(uint32_t), s));
    HIP_TRY(hipStreamSynchronize(s));
    return fail(MM_ERR_NO_PROGRESS, "a wavefront exceeded its loop-trip budget");
  }
  return MM_OK;
}

mm_status mm_batch_get_stats(mm_batch_handle b, void* stream, mm_stats* out) {
  if (!b || !out) return fail(MM_ERR_INVALID_ARG, "null argument");
  if (!(b->flags & MM_STATS)) return fail(MM_ERR_UNSUPPORTED, "batch was created without MM_STATS");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long c[mmi::kStatWords] = {};
  HIP_TRY(hipMemcpyAsync(c, b->ws + kStatsOffset, sizeof(c), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  mmi::stats_from_counters(c, out);
  return MM_OK;
}

int64_t mm_batch_items(mm_batch_handle b) { return b ? b->plan.n_items + b->plan.n_lds : -1; }

void mm_batch_destroy(mm_batch_handle b) {
  if (!b) return;
  drop_graph(b);
  // the tables are released, stream-ordered, after the last run that reads them
  if (b->last_run) {
    hipStreamWaitEvent(nullptr, b->last_run, 0);
    hipEventDestroy(b->last_run);
  }
  mmi::free_owned(b->own);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"

namespace mmb {
BatchInfo batch_info(const mm_batch* b) {
  BatchInfo i;
  i.descs = b->plan.descs;
  i.vtx_off = reinterpret_cast<const int64_t*>(b->ws + b->lay.vtx);
  i.G = b->G;
  i.N = b->N;
  i.ws = b->ws;
  return i;
}
}  // namespace mmb

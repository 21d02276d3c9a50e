// Batched matching: many independent graphs in one persistent launch.
//
// Every graph is described by a GraphDesc (its offsets, neighbours, vertex
// count, and where its states, hint and mate entries live). The work is a
// table of items (graph, first source, source count), each the size of one
// wavefront block of the single-graph sweep. A persistent grid of wavefronts
// pops items from a device counter and runs the same sweep_block on each, so
// a thousand small graphs fill the GPU as well as one large graph does. The
// per-pass work (state fill, queue reset, persistent sweep, output fix-up)
// can be captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "batch.h"
#include "internal.h"
#include "mm.h"
#include "sweep.h"

using namespace mmk;
using mmi::fail;
using mmi::kCtrlBytes;
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
    if (e < b) {
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

template <class Layout>
__device__ __forceinline__ Layout layout_of(const GraphDesc& d);
template <>
__device__ __forceinline__ LayoutU32<false> layout_of(const GraphDesc& d) {
  return LayoutU32<false>{d.mate, Hint{d.hint}};
}
template <>
__device__ __forceinline__ LayoutU32<true> layout_of(const GraphDesc& d) {
  return LayoutU32<true>{d.mate, Hint{d.hint}};
}
template <>
__device__ __forceinline__ LayoutPacked<8, false> layout_of(const GraphDesc& d) {
  return LayoutPacked<8, false>{d.st, d.mate, Hint{d.hint}};
}
template <>
__device__ __forceinline__ LayoutPacked<8, true> layout_of(const GraphDesc& d) {
  return LayoutPacked<8, true>{d.st, d.mate, Hint{d.hint}};
}
template <>
__device__ __forceinline__ LayoutPacked<2, false> layout_of(const GraphDesc& d) {
  return LayoutPacked<2, false>{d.st, d.mate, Hint{d.hint}};
}
template <>
__device__ __forceinline__ LayoutPacked<2, true> layout_of(const GraphDesc& d) {
  return LayoutPacked<2, true>{d.st, d.mate, Hint{d.hint}};
}

// Persistent sweep: every wavefront pops items until the table is exhausted;
// each item is one sweep_block of one graph. Every wavefront reaches the exit
// (the counter only grows, and each item's sweep has its own trip budget).
template <class Layout, bool HINT, bool LAZY, bool STATS>
__global__ __launch_bounds__(256) void batch_sweep_kernel(SweepParams p,
                                                         const GraphDesc* __restrict__ descs,
                                                         const WorkItem* __restrict__ items,
                                                         int64_t n_items, uint32_t* queue,
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
    const Layout L = layout_of<Layout>(d);
    sweep_block<int64_t, Layout, HINT, LAZY, STATS>(p, d.off, d.nbr, L, w.vb, (int64_t)w.nv,
                                                    queues[threadIdx.x >> 6], cnt);
  }
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
                     bp.items, bp.n_items, bp.queue, bp.stats);
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
hipError_t enqueue_typed(const BatchPlan& bp, hipStream_t s) {
  uint32_t* mate_w = reinterpret_cast<uint32_t*>(bp.mate);
  if (bp.hint) fill(bp.hint_base, bp.hint_words, 0u, s);
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, bp.queue);
  const bool two = bp.protocol == MM_PROTOCOL_TWO_PHASE;
  hipError_t e;
  if (bp.layout == MM_LAYOUT_U32) {
    if (two) {
      fill(mate_w, bp.N, LayoutU32<true>::kAcc, s);
      e = launch_flags<LayoutU32<true>, STATS>(bp, s);
      if (e == hipSuccess && !bp.lazy) {
        hipLaunchKernelGGL(replace_words_kernel, dim3(grid_for(bp.N)), dim3(256), 0, s, mate_w,
                           bp.N, LayoutU32<true>::kAcc, 0xffffffffu);
        e = hipGetLastError();
      }
      return e;
    }
    fill(mate_w, bp.N, LayoutU32<false>::kAcc, s);
    return launch_flags<LayoutU32<false>, STATS>(bp, s);
  }
  fill(bp.st_base, bp.st_words, 0u, s);
  if (!bp.lazy) fill(mate_w, bp.N, 0xffffffffu, s);
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
};

bool plan_layout(int32_t G, const int64_t* vtx_off, const mm_tuning& t, BatchLayout* out) {
  int64_t n_items = 0, st_words = 0, hint_words = 0;
  for (int32_t g = 0; g < G; ++g) {
    const int64_t n = vtx_off[g + 1] - vtx_off[g];
    if (n < 0 || n > INT32_MAX) return false;
    n_items += (n + t.wave_vertices - 1) / t.wave_vertices;
    st_words += mmb::state_words_for(n, t.layout);
    if (t.hint) hint_words += (n + 31) / 32;
  }
  BatchLayout L;
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
  const int64_t* off;
  const int32_t* nbr;
  int32_t G;
  int64_t N, M;
  uint8_t* ws;
  uint32_t flags;
  mm_tuning tun;
  BatchLayout lay;
  std::vector<mmb::GraphDesc> descs;  // host copy; mate pointers set per output
  std::vector<int64_t> vtx_off;
  mmb::BatchPlan plan;
  int32_t* bound_mate = nullptr;  // output the device descriptors point into
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(mm_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

size_t mm_batch_workspace_bytes(int32_t num_graphs, const int64_t* vtx_off, const mm_tuning* tp) {
  if (num_graphs < 0 || (!vtx_off && num_graphs > 0)) return 0;
  mm_tuning t;
  if (tp) t = *tp; else mm_default_tuning(&t);
  if (mmi::check_tuning(t) != MM_OK) return 0;
  BatchLayout L;
  if (!plan_layout(num_graphs, vtx_off, t, &L)) return 0;
  return L.total;
}

mm_status mm_batch_create(const int64_t* offsets_cat, const int32_t* neighbors_cat,
                          const int64_t* vtx_off, int32_t num_graphs, int64_t M, void* workspace,
                          size_t workspace_bytes, uint32_t flags, const mm_tuning* tuning,
                          void* stream, mm_batch_handle* out) {
  if (!out) return fail(MM_ERR_INVALID_ARG, "out handle pointer is null");
  *out = nullptr;
  if (num_graphs < 0) return fail(MM_ERR_INVALID_ARG, "num_graphs is negative");
  if (!vtx_off) return fail(MM_ERR_INVALID_ARG, "vtx_off is null");
  if (!offsets_cat) return fail(MM_ERR_INVALID_ARG, "offsets is null");
  if (!neighbors_cat && M > 0) return fail(MM_ERR_INVALID_ARG, "neighbors is null");
  if (M < 0) return fail(MM_ERR_INVALID_ARG, "M is negative");
  if (!workspace) return fail(MM_ERR_INVALID_ARG, "workspace is null");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(MM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (flags & ~(uint32_t)(MM_VALIDATE | MM_SYMMETRIC | MM_STATS | MM_TIMING | MM_CAPTURE))
    return fail(MM_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
  if (vtx_off[0] != 0) return fail(MM_ERR_INVALID_ARG, "vtx_off[0] must be 0");
  for (int32_t g = 0; g < num_graphs; ++g)
    if (vtx_off[g + 1] < vtx_off[g] || vtx_off[g + 1] - vtx_off[g] > INT32_MAX)
      return fail(MM_ERR_INVALID_ARG, "vtx_off must be non-decreasing with graphs of < 2^31 vertices");
  mm_tuning t;
  if (tuning) t = *tuning; else mm_default_tuning(&t);
  mm_status st = mmi::check_tuning(t);
  if (st != MM_OK) return st;
  BatchLayout lay;
  plan_layout(num_graphs, vtx_off, t, &lay);
  if (workspace_bytes < lay.total)
    return fail(MM_ERR_OUT_OF_MEMORY, "workspace has %zu bytes, needs %zu", workspace_bytes, lay.total);
  const int64_t N = vtx_off[num_graphs];
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
  if (flags & MM_VALIDATE) {
    int64_t* vdev = reinterpret_cast<int64_t*>(ws + lay.vtx);
    HIP_TRY(hipMemcpyAsync(vdev, vtx_off, sizeof(int64_t) * (num_graphs + 1), hipMemcpyHostToDevice, s));
    uint32_t* f = reinterpret_cast<uint32_t*>(ws);
    HIP_TRY(mmb::validate_batch(offsets_cat, neighbors_cat, vdev, num_graphs, N, M, f, s));
    uint32_t hf = 0;
    HIP_TRY(hipMemcpyAsync(&hf, f, sizeof(hf), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemsetAsync(ws, 0, kCtrlBytes, s));
    if (hf)
      return fail(MM_ERR_INVALID_GRAPH, "invalid batch CSR:%s%s%s",
                  (hf & 1u) ? " offsets[0] != 0 or offsets[N] != M;" : "",
                  (hf & 2u) ? " offsets decrease;" : "",
                  (hf & 4u) ? " neighbour id outside its graph;" : "");
  }
  mm_batch* b = new (std::nothrow) mm_batch();
  if (!b) return fail(MM_ERR_OUT_OF_MEMORY, "host allocation of the batch handle failed");
  b->off = offsets_cat;
  b->nbr = neighbors_cat;
  b->G = num_graphs;
  b->N = N;
  b->M = M;
  b->ws = ws;
  b->flags = flags;
  b->tun = t;
  b->lay = lay;
  b->vtx_off.assign(vtx_off, vtx_off + num_graphs + 1);
  // descriptors (mate pointers are bound at the first run) and work items
  b->descs.resize(num_graphs);
  std::vector<mmb::WorkItem> items;
  items.reserve((size_t)lay.n_items);
  uint32_t* st_base = reinterpret_cast<uint32_t*>(ws + lay.st);
  uint32_t* hint_base = reinterpret_cast<uint32_t*>(ws + lay.hint);
  int64_t st_w = 0, hint_w = 0;
  for (int32_t g = 0; g < num_graphs; ++g) {
    const int64_t n = vtx_off[g + 1] - vtx_off[g];
    mmb::GraphDesc& d = b->descs[g];
    d.off = offsets_cat + vtx_off[g];
    d.nbr = neighbors_cat;
    d.n = n;
    d.st = t.layout == MM_LAYOUT_U32 ? nullptr : st_base + st_w;
    d.hint = t.hint ? hint_base + hint_w : nullptr;
    d.mate = nullptr;
    st_w += mmb::state_words_for(n, t.layout);
    if (t.hint) hint_w += (n + 31) / 32;
    for (int64_t vb = 0; vb < n; vb += t.wave_vertices) {
      mmb::WorkItem w;
      w.desc = g;
      w.vb = vb;
      w.nv = (int32_t)std::min<int64_t>(t.wave_vertices, n - vb);
      items.push_back(w);
    }
  }
  mmb::WorkItem* items_dev = reinterpret_cast<mmb::WorkItem*>(ws + lay.items);
  hipError_t e = hipSuccess;
  if (!items.empty())
    e = hipMemcpyAsync(items_dev, items.data(), sizeof(mmb::WorkItem) * items.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  int cus = 0;
  if (e == hipSuccess) {
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  }
  if (e == hipSuccess && (flags & MM_CAPTURE)) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete b;
    return fail(MM_ERR_HIP, "batch setup failed: %s", hipGetErrorString(e));
  }
  mmb::BatchPlan& p = b->plan;
  p.params.wave_vertices = t.wave_vertices;
  p.params.disperse = t.disperse;
  p.params.assist_after = t.assist_after;
  p.params.scan_width = t.scan_width;
  p.params.stream_loads = t.stream_loads;
  p.params.iter_cap = t.iter_cap;
  p.params.err = reinterpret_cast<uint32_t*>(ws);
  p.descs = reinterpret_cast<const mmb::GraphDesc*>(ws + lay.descs);
  p.items = items_dev;
  p.n_items = lay.n_items;
  p.queue = reinterpret_cast<uint32_t*>(ws + kQueueOffset);
  p.stats = reinterpret_cast<unsigned long long*>(ws + kStatsOffset);
  p.layout = t.layout;
  p.protocol = t.protocol;
  p.hint = t.hint != 0;
  p.lazy = t.lazy_init && (flags & MM_SYMMETRIC) &&
           !(t.layout == MM_LAYOUT_U32 && t.protocol == MM_PROTOCOL_CAS);
  p.stats_on = (flags & MM_STATS) != 0;
  p.wg_size = t.wg_size;
  p.num_cus = cus > 0 ? cus : 1;
  p.mate = nullptr;
  p.N = N;
  p.st_base = st_base;
  p.st_words = lay.st_words;
  p.hint_base = hint_base;
  p.hint_words = lay.hint_words;
  *out = b;
  return MM_OK;
}

mm_status mm_batch_run(mm_batch_handle b, void* stream, int32_t* match_out) {
  if (!b) return fail(MM_ERR_INVALID_ARG, "batch handle is null");
  if (!match_out && b->N > 0) return fail(MM_ERR_INVALID_ARG, "match_out is null");
  if (b->plan.n_items == 0) return MM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (match_out != b->bound_mate) {
    // bind the descriptors to this output, then drop any graph captured for another one
    for (int32_t g = 0; g < b->G; ++g) b->descs[g].mate = match_out + b->vtx_off[g];
    HIP_TRY(hipMemcpyAsync(const_cast<mmb::GraphDesc*>(b->plan.descs), b->descs.data(),
                           sizeof(mmb::GraphDesc) * b->descs.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
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
    return MM_OK;
  }
  hipError_t e = mmb::enqueue_pass(b->plan, s);
  if (e != hipSuccess) return fail(MM_ERR_HIP, "batch launch failed: %s", hipGetErrorString(e));
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
  unsigned long long c[16] = {};
  HIP_TRY(hipMemcpyAsync(c, b->ws + kStatsOffset, sizeof(c), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  mmi::stats_from_counters(c, out);
  return MM_OK;
}

int64_t mm_batch_items(mm_batch_handle b) { return b ? b->plan.n_items : -1; }

}  // extern "C"

namespace mmb {
BatchInfo batch_info(const mm_batch* b) {
  BatchInfo i;
  i.off = b->off;
  i.nbr = b->nbr;
  i.G = b->G;
  i.N = b->N;
  i.ws = b->ws;
  i.vtx_dev = reinterpret_cast<int64_t*>(b->ws + b->lay.vtx);
  i.vtx_host = b->vtx_off.data();
  return i;
}
}  // namespace mmb

extern "C" {

void mm_batch_destroy(mm_batch_handle b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"

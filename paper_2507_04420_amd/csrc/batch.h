// Descriptor-based batched sweep shared by the batch ABI and the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sweep.h"

struct mm_batch;

namespace mmb {

// One graph of a batch. `off` is based at the graph's first vertex and indexes
// `nbr`; neighbour ids are local to the graph. Its mate entries are those at
// v0 .. v0+n-1 of the batch's output.
struct GraphDesc {
  const int64_t* off;
  const int32_t* nbr;
  int64_t n;
  int64_t m;       // entries of the graph (list batches), -1 when not known
  int64_t v0;      // first global vertex
  uint32_t* st;    // packed states, or null for the word layout
  uint32_t* hint;  // matched hint words, or null
  uint32_t hint_lg;  // log2 of vertices per hint word
  uint32_t flags;    // kWholeGraph: swept by one wavefront, no hub pieces
  int64_t pieces;    // hub table build only: piece count, then fill cursor
  int64_t not_mesh;  // create only (mesh_wave_vertices): 1 if a list exceeds kMeshDegree
};
constexpr uint32_t kWholeGraph = 1u;
constexpr uint32_t kWholeLds = 2u;  // with kWholeGraph: states in the wavefront's LDS (whole.h)
constexpr uint32_t kMesh = 4u;      // lists of at most kMeshDegree entries: dispersed lanes
constexpr int64_t kMeshDegree = 4;

// One wavefront block: sources vb .. vb+nv-1 of graph `desc`; or, with
// nv < 0, the hub pieces vb .. vb-nv-1 of the piece table (all of graph desc).
struct WorkItem {
  int32_t desc;
  int32_t nv;
  int64_t vb;
};

// Everything one pass of the batched sweep needs on the device.
struct BatchPlan {
  mmk::SweepParams params;  // hub_degree / hub_chunk / chunks: the hub tier
  const GraphDesc* descs;
  const WorkItem* items;
  int64_t n_items;
  uint32_t* queue;
  unsigned long long* stats;
  int32_t layout, protocol;
  bool hint, lazy, stats_on;
  int wg_size, num_cus;
  int32_t* mate;  // base of all mate entries (N of them)
  int64_t N;
  uint32_t* st_base;
  int64_t st_words;
  uint32_t* hint_base;
  int64_t hint_words;
  // graphs kept in LDS (kWholeLds): one item each, swept by a kernel of
  // their own before the persistent sweep
  const WorkItem* lds_items;
  int64_t n_lds;
  int32_t lds_words;  // LDS words per wavefront (0: no such graph)
  int lds_wg;         // threads per workgroup of that kernel
};

// Enqueues one pass: fills, queue reset, persistent sweep, output fix-up.
hipError_t enqueue_pass(const BatchPlan& bp, hipStream_t s);

// Device check of a concatenated CSR (bits as for the single-graph check).
hipError_t validate_batch(const int64_t* off, const int32_t* nbr, const int64_t* vtx_off_dev,
                          int32_t num_graphs, int64_t N, int64_t M, uint32_t* flags,
                          hipStream_t s);

// Device check of the graphs of a list batch, through their descriptors:
// off[0] = 0, off[n] = m, offsets non-decreasing, ids in [0, n).
hipError_t validate_list(const GraphDesc* descs, const int64_t* vtx_off_dev, int32_t num_graphs,
                         int64_t N, uint32_t* flags, hipStream_t s);

// 32-bit words of packed state for n vertices under `layout` (0 for words).
int64_t state_words_for(int64_t n, int32_t layout);

// What the device check needs from a batch handle (all device pointers).
struct BatchInfo {
  const GraphDesc* descs;
  const int64_t* vtx_off;
  int32_t G;
  int64_t N;
  uint8_t* ws;
};
BatchInfo batch_info(const mm_batch* b);

// Hub pieces of a batch (see hubs.hip): lists longer than hub_degree in
// graphs without kWholeGraph, cut into pieces of `chunk` entries. Counting
// adds each graph's pieces to descs[g].pieces (zero on entry) and all of them
// to the control block word at kHubOffset. Filling takes descs[g].pieces as
// the first table slot of graph g and writes every piece (stream-ordered).
hipError_t count_batch_hubs(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                            int64_t hub_degree, int64_t chunk, uint8_t* ctrl, hipStream_t s);
// Sets descs[g].not_mesh (zero on entry) for every graph with a list of more
// than kMeshDegree entries.
hipError_t batch_find_meshes(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                             hipStream_t s);
hipError_t fill_batch_hubs(GraphDesc* descs_dev, const int64_t* vtx_dev, int32_t G, int64_t N,
                           int64_t hub_degree, int64_t chunk, mmk::HubChunk* table, hipStream_t s);

}  // namespace mmb

// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "mm.h"

namespace mmi {

// Records a thread-local message for mm_last_error() and returns s.
mm_status fail(mm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Validates a tuning struct (wg_size, wave_vertices, layout, flags ranges).
mm_status check_tuning(const mm_tuning& t);

// Largest vertex count a graph may have under tuning t: the word layout with
// the two-phase protocol keeps ACC = INT32_MAX and RSVD = INT32_MAX - 1 in the
// same word as a mate id, so its ids must stay below INT32_MAX - 1.
inline int64_t max_vertices(const mm_tuning& t) {
  return (t.layout == MM_LAYOUT_U32 && t.protocol == MM_PROTOCOL_TWO_PHASE) ? (int64_t)INT32_MAX - 1
                                                                            : (int64_t)INT32_MAX;
}

// Workspace pieces after the control block: packed states (U8 layout only),
// then the matched hint (if enabled), each rounded to 256 bytes.
size_t state_bytes(int64_t n, const mm_tuning& t);
size_t hint_bytes(int64_t n, const mm_tuning& t);

// Accessors of a single-graph handle (defined with the handle).
int64_t handle_n(const mm_graph* h);
int handle_off64(const mm_graph* h);
const void* handle_off(const mm_graph* h);
const int32_t* handle_nbr(const mm_graph* h);
uint8_t* handle_ws(const mm_graph* h);
uint32_t handle_flags(const mm_graph* h);

// A graph relabelled by degree (see relabel.hip), in a workspace region of
// relabel_bytes(n, m) bytes: int64 offsets, new -> given id map, neighbours.
// mode 1: by log2-degree bucket; mode 2: isolated first, then the given order,
// vertices of more than hot entries last.
struct RelabelView {
  int64_t* off;
  int32_t* orig;
  int32_t* nbr;
  int64_t n_isolated;  // new ids 0 .. n_isolated-1 have no entries
};
size_t relabel_bytes(int64_t n, int64_t m);
// Upper bound of the device memory build_relabel allocates for its own
// temporaries (freed before it returns).
size_t relabel_temp_bytes(int64_t n);
// Upper bound of the hub pieces of a graph of m entries: every list longer
// than hub_degree gives ceil(d / chunk) <= d / chunk + 1 pieces, and there are
// at most m / (hub_degree + 1) such lists.
inline int64_t hub_pieces_bound(int64_t m, int64_t hub_degree, int64_t chunk) {
  if (hub_degree <= 0 || m <= hub_degree) return 0;
  return m / chunk + m / (hub_degree + 1);
}
hipError_t build_relabel(const void* off, int off64, const int32_t* nbr, int64_t n, int64_t m,
                         int mode, int64_t hot, uint8_t* region, RelabelView* view, hipStream_t s);
// The neighbour lists with each list of at most 256 entries reordered by
// ascending log2 degree of the neighbour (order.hip), with upper_first the
// neighbours above the list's vertex before those below it, written to out
// (m ids); waits for the copy before it returns. Temporary device memory: at
// most order_temp_bytes(n), freed before it returns.
constexpr int64_t kOrderedMax = 256;  // the longest list the copy reorders
hipError_t build_ordered_lists(const void* off, int off64, const int32_t* nbr, int64_t n,
                               int upper_first, int32_t* out, hipStream_t s);
size_t order_temp_bytes(int64_t n);

// The hub tier's table (see hubs.hip), allocated stream-ordered on s and
// released with free_owned by the handle's owner; *count = 0 and *table = null
// when no list is long enough. Uses two words of the control block at ctrl.
}  // namespace mmi
namespace mmk {
struct HubChunk;
}
namespace mmi {
hipError_t build_hub_chunks(const void* off, int off64, int64_t n, int64_t hub_degree,
                            int64_t chunk, uint8_t* ctrl, mmk::HubChunk** table, int64_t* count,
                            hipStream_t s);
// Fills a hub table of known capacity without counting first and without a
// wait: each long list takes its run of slots from *cursor (zero on entry),
// which ends holding the number of pieces. The caller sizes the table with
// hub_pieces_bound.
hipError_t fill_hub_chunks(const void* off, int off64, int64_t n, int64_t hub_degree, int64_t chunk,
                           unsigned long long* cursor, mmk::HubChunk* table, hipStream_t s);
// Stream-ordered release of memory a handle owns (no wait for the device).
void free_owned(void* p);

// A sweep too small to give min_waves wavefronts of wave_vertices sources gets
// shorter blocks (single graphs and batches alike), so that about min_waves
// wavefronts share it and its latency; never shorter than 64 sources.
// min_waves = 0 keeps wave_vertices whatever the size.
inline int64_t short_blocks(int64_t sources, int64_t wave_vertices, int64_t min_waves) {
  if (min_waves <= 0 || sources >= min_waves * wave_vertices) return wave_vertices;
  const int64_t w = (sources / min_waves + 63) / 64 * 64;
  return w < 64 ? 64 : w;
}

// Copies the raw device counters (sweep.h order) into the ABI struct.
void stats_from_counters(const unsigned long long* c, mm_stats* out);

// Control block at the start of every workspace: error word at 0, counters
// at kStatsOffset, the hub table build's piece count and cursor at
// kHubOffset, a work-queue counter at kQueueOffset, the six counters of the
// device check at kCheckOffset.
constexpr size_t kCtrlBytes = 4096;
constexpr size_t kStatsOffset = 256;
constexpr size_t kHubOffset = 512;
constexpr size_t kQueueOffset = 1024;
constexpr size_t kCheckOffset = 2048;
constexpr int kStatWords = 32;  // 64-bit counters at kStatsOffset

}  // namespace mmi

#define MMI_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::mmi::fail(MM_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

/*
 * mm.h: C ABI of the MI355X (gfx950) maximal-matching library.
 *
 * The library computes a maximal matching of an undirected graph with the
 * single-pass, just-in-time conflict-resolution method of Skipper
 * (Koohi Esfahani, arXiv 2507.04420, Section IV and Algorithm 1): every vertex
 * carries a state (accessible, reserved, matched); each edge (x, y), x != y,
 * is examined by the lane that owns its source, which reserves the lower-id
 * endpoint u, then tries to move the higher-id endpoint v from accessible to
 * matched, and on success marks u matched (otherwise releases u). Once a
 * source is matched the rest of its neighbour list is skipped (Section II-B,
 * CSR form of greedy matching; Fig. 6g).
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are device (HBM) addresses on the current HIP
 *    device; pointers marked "host" are host addresses.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Work
 *    is enqueued on it and the call returns without waiting.
 *  - Return codes only; nothing crosses the ABI as an exception. After a
 *    non-OK status, mm_last_error() returns a thread-local message.
 *  - The graph arrays are borrowed: the library neither copies nor frees
 *    them, and they must outlive the handle. Workspaces and outputs are
 *    caller-owned device memory. mm_run and mm_batch_run allocate nothing;
 *    the create calls may (tuning.relabel: temporary buffers;
 *    tuning.hub_degree: the hub piece table, kept until destroy), at most
 *    mm_create_device_bytes / mm_batch_create_device_bytes bytes. Those
 *    allocations are stream-ordered (hipMallocAsync on the create call's
 *    stream, hipFreeAsync at destroy), so create and destroy never wait for
 *    the whole device. A run on any stream waits for what its create call
 *    enqueued, and destroy releases the tables after the handle's last run
 *    (an event recorded on that run's stream), so a handle may be destroyed
 *    while its last run is in flight; the caller's own memory (workspace,
 *    output, CSR) must outlive every run.
 *
 * Graph format (Section II-A): CSR with `offsets` of n+1 entries (int32 or
 * int64, non-decreasing, offsets[0] = 0, offsets[n] = m) and `neighbors` of m
 * int32 ids in [0, n). Self-loops and duplicate entries are allowed and never
 * matched. A non-symmetric CSR is accepted; the result is then maximal for the
 * undirected union of its entries (Section V-C, input format).
 *
 * Output: a mate array of n int32 entries: match[v] = w if {v, w} is in the
 * matching, -1 if v is unmatched. It is symmetric, and the matching is
 * maximal. Several maximal matchings can be correct: the method is
 * non-deterministic (Section V-C).
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_graph* mm_handle;

typedef enum {
  MM_OK = 0,
  MM_ERR_INVALID_ARG = 1,    /* null pointer, bad size or bad tuning value */
  MM_ERR_INVALID_GRAPH = 2,  /* MM_VALIDATE found a malformed CSR */
  MM_ERR_OUT_OF_MEMORY = 3,  /* workspace smaller than mm_workspace_bytes() */
  MM_ERR_HIP = 4,            /* a HIP runtime call failed (message has details) */
  MM_ERR_NO_PROGRESS = 5,    /* a wavefront exceeded its loop-trip budget */
  MM_ERR_UNSUPPORTED = 6     /* option combination not supported */
} mm_status;

typedef enum { MM_OFF_I32 = 0, MM_OFF_I64 = 1 } mm_offset_type;

/* Vertex state layouts (Section IV-C keeps one byte of state per vertex). */
typedef enum {
  /* One state byte per vertex, four per 32-bit word; byte transitions use
     32-bit atomics on the containing word. The mate array is separate. */
  MM_LAYOUT_U8 = 0,
  /* One 32-bit word per vertex that is also the output: matched = the mate
     (>= 0); accessible and reserved are two reserved values (-1 and -2 with
     MM_PROTOCOL_CAS; INT32_MAX and INT32_MAX-1 with MM_PROTOCOL_TWO_PHASE, so
     that reserving is an atomic min). */
  MM_LAYOUT_U32 = 1,
  /* Two state bits per vertex, sixteen per 32-bit word, same field encoding
     and atomics as MM_LAYOUT_U8 (a denser copy of it, so that neighbour-state
     reads hit the 4 MB per-XCD L2 more often). The mate array is separate. */
  MM_LAYOUT_U2 = 2
} mm_layout;

/* Creation flags. */
enum {
  MM_VALIDATE = 1u,   /* check the CSR on the device at create (synchronous) */
  MM_SYMMETRIC = 2u,  /* caller asserts every entry (x,y) has its reverse (y,x);
                         enables lazy mate initialisation */
  MM_STATS = 4u,      /* run the instrumented kernels: counters for mm_get_stats */
  MM_TIMING = 8u,     /* record HIP events around each sweep launch (mm_get_timing) */
  MM_CAPTURE = 16u    /* batches: capture one pass into a hipGraph at the first run
                         for a given output and replay it afterwards */
};

/* How the higher endpoint v of an edge is taken (Algorithm 1's second step). */
typedef enum {
  /* As printed: one CAS moves v from accessible to matched. */
  MM_PROTOCOL_CAS = 0,
  /* v is reserved like u (fetch-or / atomic-min, no CAS), then both are marked
     matched by the holder. Same state transitions (Fig. 4), same id order. */
  MM_PROTOCOL_TWO_PHASE = 1
} mm_protocol;

/* Largest graph whose states a wavefront keeps in LDS (tuning.whole_graph_lds). */
#define MM_LDS_WHOLE_MAX 16384

/* Launch and layout parameters. None of them changes what a correct result
   is; they change only speed. Fill with mm_default_tuning() first. */
typedef struct {
  int32_t layout;        /* mm_layout */
  int32_t protocol;      /* mm_protocol */
  int32_t hint;          /* skip matched neighbours by a "matched" hint (set after
                            a vertex is matched) instead of reading its state:
                            0 none, 1 one bit per vertex (atomic or), 2 one byte
                            per vertex (plain byte store) */
  int32_t wg_size;       /* threads per workgroup: 64, 128, 192 or 256 */
  int32_t wave_vertices; /* source vertices handed to one wavefront, >= 64, multiple of 64;
                            shortened for a graph too small to give min_waves
                            wavefronts (see min_waves) */
  int32_t disperse;      /* 0: a wavefront's lanes take consecutive sources;
                            1: concurrently active lanes of a wavefront take sources
                            wave_vertices/64 apart (for high-locality graphs) */
  int32_t assist_after;  /* scan steps after which the wavefront helps a lane's
                            long scan 64 entries at a time; <= 0 disables */
  int32_t lazy_init;     /* 1: unmatched outputs written by the sweep itself instead
                            of a separate fill (needs MM_SYMMETRIC; not with
                            MM_LAYOUT_U32 + MM_PROTOCOL_CAS, where it is implicit,
                            nor with upper_only or relabel). Applies only where the
                            hub tier cannot cut a list: hub_degree = 0, m <=
                            hub_degree, or a graph swept whole by one wavefront;
                            elsewhere the output is written eagerly */
  int32_t scan_width;    /* neighbour ids a lane reads per scan step: 1..4 */
  int32_t stream_loads;  /* 1: read offsets and neighbour ids with non-temporal loads,
                            so that their lines are evicted first and the state (or
                            hint) lines stay in L2 longer */
  int32_t whole_graph_vertices; /* a graph with at most this many vertices is swept
                            by one wavefront (one work item of a batch), which makes
                            its result independent of concurrent work: the same
                            alone as inside any batch; 0 disables */
  int32_t relabel;       /* single graphs only: mm_create builds, in the
                            workspace, a copy of the graph with vertices renumbered,
                            and the sweep runs on it; output stays in the given
                            ids. 1: by ascending log2-degree bucket (isolated
                            first, given order kept inside a bucket; lists of up
                            to 64 entries sorted by new id): low-degree sources
                            first, hub states packed into few cache lines.
                            2: the given order, except that isolated vertices come
                            first and vertices of more than hot_degree entries
                            last (given order kept inside each group; lists in
                            their given order): the sweep keeps the given order
                            of sources while the states most scans read share a
                            few cache lines. 0: none. Workspace from
                            mm_workspace_bytes_graph; create allocates temporary
                            device memory for the sort */
  int32_t hub_degree;    /* lists longer than this are not swept by their block's
                            lane but cut into pieces of hub_chunk entries, each swept
                            by its own lane: by wavefronts launched after the
                            blocks' (single graphs, same launch), or as work items
                            queued after the blocks (batches; not for graphs swept
                            whole by one wavefront). 0 disables. The create call
                            counts the pieces (one kernel and one wait) and, if
                            any exist, allocates the piece table itself (device
                            memory, freed by the destroy call) */
  int32_t hub_chunk;     /* entries per piece of a long list, >= 1 */
  int32_t whole_graph_lds; /* 1: a graph swept whole by one wavefront (see
                            whole_graph_vertices) with at most MM_LDS_WHOLE_MAX
                            vertices keeps its states in that wavefront's LDS,
                            since no other wavefront reads them: 2 bits per
                            vertex, with the two-phase protocol whatever the
                            layout and protocol fields say; the mates are
                            written to the output as pairs are committed. Not
                            with relabel. 0: states in device memory, as for
                            every other graph */
  int32_t mesh_wave_vertices; /* batches: a member graph none of whose lists holds
                            more than 4 entries (a mesh) and that is not swept
                            whole is cut into blocks of this many sources (a
                            multiple of 64), its lanes taking sources
                            block/64 apart, so that lanes do not hold
                            neighbouring vertices; create measures the degrees
                            on the device. 0: such graphs are cut like the
                            others. Single graphs take their launch shape from
                            the tuning alone */
  int32_t wait_release;  /* 1: a lane that finds v reserved by another lane
                            releases u while it waits, and takes u again once
                            v is accessible (Algorithm 1 holds u meanwhile). No
                            lane then waits on a lane that is itself waiting,
                            so no chain of reservations forms, which on meshes
                            swept by many lanes at once can grow as long as a
                            column. 0: as printed */
  int32_t upper_only;    /* 1 (MM_SYMMETRIC input only; ignored otherwise): a lane
                            examines only the neighbours whose id is above its
                            source's (in the swept order: the relabelled ids
                            with relabel), without reading the states of the
                            others. Each undirected edge is then examined from
                            its lower endpoint, as Algorithm 1 iterates each
                            edge of E once; its mirror entry in the higher
                            endpoint's list is passed over. Output is eager
                            (lazy_init does not apply) */
  int32_t hub_wave;      /* 1: a wavefront takes 64 pieces of long lists
                            (hub_degree), checks their sources one per lane, and
                            sweeps each piece whose source is still free with all
                            its lanes: 64 ids per step read together, the first
                            candidate found by a ballot and reserved by one
                            lane, the source's state checked before every step;
                            2 (single graphs; batches take it as 1): the same,
                            and the wavefronts of a workgroup, which take
                            consecutive runs of pieces (mostly of the same long
                            lists), share in LDS the sources they found matched,
                            checked before every step; 0: each piece by one
                            lane, like any other source's list */
  int32_t min_waves;     /* a graph alone (mm_run) or a batch whose blocked sources
                            are too few for this many wavefronts of wave_vertices
                            sources gets shorter blocks, so that about this many
                            wavefronts share it (never shorter than 64 sources);
                            0 keeps wave_vertices whatever the size */
  int32_t hot_degree;    /* relabel = 2: vertices with more entries than this go to
                            the top of the new ids; >= 1 */
  int32_t order_lists;   /* 1 (single graphs only; not with relabel): mm_create
                            copies the neighbour ids into the workspace with every
                            list of at most 256 entries reordered by ascending
                            log2 degree of the neighbour (stable), and the sweep
                            reads the copy: low-degree neighbours, which are more
                            often still free, are examined first, so scans stop
                            sooner. Ids, offsets, states and output are the
                            given ones. Workspace from mm_workspace_bytes_graph
                            (4m bytes more); create allocates n bytes of
                            temporary device memory and waits for the copy.
                            2 (needs upper_only = 1): the same copy with each
                            such list's neighbours above its vertex first (each
                            part in that degree order), so that on symmetric
                            input a scan, which skips the neighbours below its
                            source, ends at the first of them. 0: the given
                            lists */
  int32_t probe_first;   /* 1: the first state read of each source's scan reads only
                            its first candidate (on lists in degree order that
                            one is usually free, and reading the next candidates'
                            states with it would be wasted requests); later reads
                            take the rest of a step's scan_width ids together.
                            2: every state read takes one candidate (ids are
                            still read scan_width at a time). 0: every read
                            takes a whole step's candidates */
  int32_t occupancy;     /* 6: single-graph sweeps (not relabelled, not
                            instrumented) run a build of the sweep kernel limited
                            to 80 VGPRs, so that six wavefronts share each SIMD
                            instead of five: more latency hidden, and more of the
                            graph in flight at once. 0: the compiler's register
                            budget. Batches ignore it */
  int64_t iter_cap;      /* loop-trip budget per wavefront; 0 = default of
                            65536 + 8 x (neighbour entries of its block);
                            exceeding it raises MM_ERR_NO_PROGRESS */
} mm_tuning;

/* Counters of the instrumented kernels (MM_STATS). Conflicts follow Table II
   of the paper: a failed CAS while reserving u or taking v (Algorithm 1),
   whatever state it met: a reservation by another lane (RSVD, counted
   in reserve_conflicts / match_conflicts) or a match made since the lane's
   cached read of the state (MCHD, counted in reserve_matched /
   match_matched). An edge's conflicts are those met from the moment a lane
   picks the edge (x, y) as its candidate until the edge is matched or found
   dead; conflict_hist and conflict_max count both kinds. A CAS on a packed
   word that fails only because another vertex's byte changed is not a
   conflict (word_retries). */
typedef struct {
  uint64_t sources;           /* source vertices visited */
  uint64_t sources_skipped;   /* sources already matched when visited */
  uint64_t touched;           /* neighbour ids read by scanning lanes (T_gpu) */
  uint64_t assist_reads;      /* neighbour ids read by wavefront assists */
  uint64_t reserve_attempts;  /* CAS/fetch-or on u */
  uint64_t reserve_conflicts; /* u found reserved by another lane (a conflict) */
  uint64_t reserve_matched;   /* u found matched by the atomic after a cached read
                                 saw it free (a conflict) */
  uint64_t match_attempts;    /* CAS on v */
  uint64_t match_conflicts;   /* v found reserved by another lane (a conflict) */
  uint64_t match_matched;     /* v found matched by the atomic (a conflict) */
  uint64_t word_retries;      /* U8 layout: CAS retried because another byte of
                                 the same 32-bit word changed (not a conflict) */
  uint64_t pairs;             /* matched pairs committed */
  uint64_t loop_trips;        /* sum over wavefronts of loop trips */
  uint64_t conflict_max;      /* most conflicts (either kind) met by one edge */
  uint64_t conflict_hist[10]; /* edges by conflicts met: 1, 2, 3-4, 5-8, 9-16,
                                 17-32, 33-64, 65-128, 129-256, >256 (Table II) */
  uint64_t reserved_[8];
} mm_stats;

/* Fills *t with the defaults. */
void mm_default_tuning(mm_tuning* t);

/* Bytes of device workspace a graph of n vertices and m entries needs under
   tuning t (any tuning); 0 if the arguments are invalid. */
size_t mm_workspace_bytes_graph(int64_t n, int64_t m, const mm_tuning* t);

/* Bytes of device workspace a graph of n vertices needs under tuning t
   (NULL = defaults). Returns 0 if n or t is invalid, and for a nonzero
   t.relabel, whose workspace depends on m (use mm_workspace_bytes_graph). */
size_t mm_workspace_bytes(int64_t n, const mm_tuning* t);

/* Upper bound of the device memory mm_create allocates by itself for a graph
   of n vertices and m entries under tuning t (NULL = defaults), beyond the
   caller's workspace: the hub piece table (24 bytes a piece, kept until
   mm_destroy; at most m / hub_chunk + m / (hub_degree + 1) pieces) and, with
   t.relabel, the relabelling's temporaries (freed before mm_create returns;
   their sort scratch as the device library reports it, or 16n + 64 MiB when
   no device can be asked). 0 if nothing is allocated or the arguments are
   invalid. A caller that budgets device memory adds this to the workspace
   and the output. */
size_t mm_create_device_bytes(int64_t n, int64_t m, const mm_tuning* t);

/*
 * Creates a handle for one graph.
 *  offsets    device, n+1 entries of `off_type`
 *  neighbors  device, m int32 entries
 *  n, m       vertex and entry counts; 0 <= n <= 2^31-1; m <= 2^31-1 for int32 offsets
 *  workspace  device, >= mm_workspace_bytes(n, tuning) bytes, 256-byte aligned,
 *             caller-owned, must outlive the handle; holds vertex states,
 *             counters and the error flag
 *  flags      MM_VALIDATE | MM_SYMMETRIC | MM_STATS | MM_TIMING
 *  tuning     host, NULL = defaults; copied
 * With MM_VALIDATE the call runs a device check on `stream` and waits for it;
 * a malformed CSR returns MM_ERR_INVALID_GRAPH and no handle.
 */
mm_status mm_create(const void* offsets, mm_offset_type off_type, const int32_t* neighbors,
                    int64_t n, int64_t m, void* workspace, size_t workspace_bytes,
                    uint32_t flags, const mm_tuning* tuning, void* stream, mm_handle* out);

/*
 * Enqueues one maximal-matching pass on `stream`: state initialisation, then
 * the sweep (Algorithm 1). match_out: device, n int32, caller-owned; valid
 * after the stream reaches this point. One pass at a time per handle (the
 * vertex states live in its workspace); different handles may run
 * concurrently on different streams.
 */
mm_status mm_run(mm_handle h, void* stream, int32_t* match_out);

/* Waits for `stream`, then reports a device-side failure of any earlier pass
   of this handle (MM_ERR_NO_PROGRESS) and clears it. */
mm_status mm_sync(mm_handle h, void* stream);

/* Bytes of the library's static device scratch (mm_run_static). */
#define MM_STATIC_SCRATCH_BYTES ((size_t)8 << 20)

/*
 * mm_create + mm_run in one call that allocates nothing and takes no
 * workspace, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc). The
 * pass is the same as mm_run's, with the same kernels; what a workspace would
 * hold lives in a static device array of MM_STATIC_SCRATCH_BYTES that the
 * library keeps on every device it runs on until the process ends: a 4 KiB
 * control block, then the packed states (tuning.layout U8: n bytes, U2: n/4;
 * the word layout keeps its states in match_out), the matched hint (n/8 or n
 * bytes), and the hub piece table (24 bytes per piece, sized for
 * m / hub_chunk + m / (hub_degree + 1) pieces). A graph and tuning that need
 * more return MM_ERR_OUT_OF_MEMORY before anything is enqueued (the default
 * tuning needs only the control block and the piece table: up to about 8.5e7
 * entries; hub_degree = 0 needs no piece table).
 *  offsets, off_type, neighbors, n, m   as for mm_create (borrowed, device)
 *  flags      MM_SYMMETRIC only (no device validation, counters or timing)
 *  tuning     host, NULL = defaults; tuning.relabel is not supported
 *  match_out  device, n int32, caller-owned: the mate array, as mm_run's
 *  status_out device, one uint32, caller-owned, may be NULL: set to 0 by the
 *             pass, then to 1 if a wavefront exceeded its loop-trip budget
 *             (the condition mm_sync reports as MM_ERR_NO_PROGRESS)
 * Everything is enqueued on `stream` (kernels only, no copies, memsets or
 * waits), so the call can be captured into a HIP graph. Every call on a device
 * uses that device's one scratch array and leaves its contents behind (each
 * call clears what must start at zero): calls that overlap on one device race,
 * so the caller orders them (one stream, or events).
 */
mm_status mm_run_static(const void* offsets, mm_offset_type off_type, const int32_t* neighbors,
                        int64_t n, int64_t m, uint32_t flags, const mm_tuning* tuning, void* stream,
                        int32_t* match_out, uint32_t* status_out);

/* Waits for `stream` and copies the counters accumulated since the last
   mm_reset_stats (MM_STATS handles only; others return MM_ERR_UNSUPPORTED). */
mm_status mm_get_stats(mm_handle h, void* stream, mm_stats* out);
mm_status mm_reset_stats(mm_handle h, void* stream);

/* MM_TIMING handles: waits for the events of the passes enqueued since the
   last call, and returns how many sweep launches they hold and the sum, min
   and max of their device durations in milliseconds (hipEventElapsedTime of
   events recorded on the launch stream right before and after the sweep
   kernel). Up to 512 launches are kept between calls; older ones are dropped
   (count tells how many were measured). */
mm_status mm_get_timing(mm_handle h, int64_t* count, double* total_ms, double* min_ms,
                        double* max_ms);

/* Frees the host-side handle (and its timing events). Does not touch
   caller-owned memory. */
void mm_destroy(mm_handle h);

/* ------------------------------------------------------------------ batches
 * Many independent graphs matched in one persistent launch. The graphs are
 * concatenated: offsets_cat holds N+1 int64 positions into neighbors_cat
 * (offsets_cat[0] = 0, offsets_cat[N] = M); the neighbour ids of graph g are
 * local to it (0 .. n_g-1); vtx_off (host, num_graphs+1 entries, vtx_off[0] =
 * 0) gives graph g the global vertices vtx_off[g] .. vtx_off[g+1]-1. The
 * output match_out (device, N int32) receives, for every global vertex, the
 * LOCAL id of its mate in its own graph, or -1. Each graph's result is a
 * maximal matching of that graph, computed by the same sweep as mm_run.
 */
typedef struct mm_batch* mm_batch_handle;

/* Workspace bytes for a batch (vtx_off: host). 0 if the arguments are invalid. */
size_t mm_batch_workspace_bytes(int32_t num_graphs, const int64_t* vtx_off, const mm_tuning* t);

/* Upper bound of the device memory a batch create call allocates by itself
   (vtx_off: host; M: entries of all graphs together): when hub pieces exist,
   the work-item table and the piece table, kept until mm_batch_destroy. 0 if
   nothing is allocated or the arguments are invalid. */
size_t mm_batch_create_device_bytes(int32_t num_graphs, const int64_t* vtx_off, int64_t M,
                                    const mm_tuning* t);

/* Creates a batch handle: builds the graph descriptors and the work-item
   table (one item per wavefront block of every graph) in the workspace and
   waits for the upload. Arrays are borrowed
   like those of mm_create. flags: MM_VALIDATE | MM_SYMMETRIC | MM_STATS |
   MM_CAPTURE. */
mm_status mm_batch_create(const int64_t* offsets_cat, const int32_t* neighbors_cat,
                          const int64_t* vtx_off, int32_t num_graphs, int64_t M, void* workspace,
                          size_t workspace_bytes, uint32_t flags, const mm_tuning* tuning,
                          void* stream, mm_batch_handle* out);

/* Creates a batch over graphs that live in separate allocations (a list
   batch), as a server holding many resident graphs coalesces them into one
   launch. offsets[g] and neighbors[g] (host arrays of num_graphs device
   pointers) are graph g's own CSR: n[g]+1 int64 offsets from 0 to m[g], m[g]
   int32 local ids (n, m: host arrays). The output layout is as for
   mm_batch_create with vtx_off the prefix sums of n, which is also what
   mm_batch_workspace_bytes takes. A graph with n[g] = 0 must have m[g] = 0
   and its pointers are never read. MM_VALIDATE checks every graph's CSR on
   the device. Arrays are borrowed; the host arrays may be freed on return. */
mm_status mm_batch_create_list(const int64_t* const* offsets, const int32_t* const* neighbors,
                               const int64_t* n, const int64_t* m, int32_t num_graphs,
                               void* workspace, size_t workspace_bytes, uint32_t flags,
                               const mm_tuning* tuning, void* stream, mm_batch_handle* out);

/* Enqueues one pass over every graph of the batch on `stream`; nothing is
   waited for. With MM_CAPTURE the pass is a hipGraph replay, captured at the
   first run with a given match_out (a run with another output captures
   again). */
mm_status mm_batch_run(mm_batch_handle h, void* stream, int32_t* match_out);

/* As mm_sync, for a batch. */
mm_status mm_batch_sync(mm_batch_handle h, void* stream);

/* As mm_get_stats, for a batch created with MM_STATS. */
mm_status mm_batch_get_stats(mm_batch_handle h, void* stream, mm_stats* out);

/* Number of work items of the batch (wavefront blocks, hub pieces in runs of
   64, and one per graph swept whole); -1 for a null handle. */
int64_t mm_batch_items(mm_batch_handle h);

/* Frees the host-side handle and any captured graph. */
void mm_batch_destroy(mm_batch_handle h);

/* ------------------------------------------------------------------ checks
 * Device verification of a mate array against the graph of a handle
 * (Section II-B's two conditions plus well-formedness). Waits for `stream`.
 * counts (host, 6 entries): [0] mates out of [-1, n); [1] vertices matched to
 * themselves; [2] asymmetric mates (mate[mate[x]] != x); [3] mates that are
 * not an edge in either list; [4] entries (x, y), x != y, with both ends
 * unmatched; [5] vertices whose mate is in [0, n). A maximal matching has counts[0..4] == 0.
 * For a batch, ids are local to each graph.
 */
mm_status mm_check(mm_handle h, void* stream, const int32_t* match, int64_t* counts);
mm_status mm_batch_check(mm_batch_handle h, void* stream, const int32_t* match, int64_t* counts);

/* ------------------------------------------------------------------ pair list
 * The matched pairs of a mate array as a list (the `matches` output of
 * Algorithm 1): pairs (device, 2 x cap int32) receives (u, v), u < v, for
 * every matched pair, each once, in no particular order; *count (host)
 * receives the number of pairs. Waits for `stream`. If count > cap, only cap
 * pairs are written and MM_ERR_OUT_OF_MEMORY is returned with *count set.
 * n / 2 pairs always suffice.
 */
mm_status mm_pairs(mm_handle h, void* stream, const int32_t* match, int32_t* pairs, int64_t cap,
                   int64_t* count);

/* ------------------------------------------------------------------ baseline
 * Iterated Endpoints Mutual Selection (Section II-C): the multi-pass scheme
 * the paper compares Skipper with, for measuring the work-efficiency contrast
 * (ids read, passes) on the same GPU. Each iteration, every unmatched vertex
 * selects its heaviest edge to an unmatched neighbour, and mutually selected
 * edges become matches, until no unmatched vertex has an unmatched
 * neighbour. Edge weights: w(u, v) = SplitMix64(SplitMix64(seed) ^ (min << 32
 * | max)); the result is the greedy matching in descending weight order (ties:
 * smaller key), the same on every run. Needs a handle created with
 * MM_SYMMETRIC (on a one-sided list an edge may never be selected by both
 * ends). Synchronous: waits for `stream` after every iteration. scratch:
 * device, 256-byte aligned, mm_ems_scratch_bytes(n) bytes. match_out: device,
 * n int32. stats (host, may be null): iterations run (the last one finds
 * nothing to select), ids read over all iterations, pairs.
 */
typedef struct {
  int64_t iterations;
  int64_t touched;
  int64_t pairs;
  int64_t reserved_[5];
} mm_ems_stats;
size_t mm_ems_scratch_bytes(int64_t n);
mm_status mm_ems_run(mm_handle h, void* stream, uint64_t seed, void* scratch,
                     size_t scratch_bytes, int32_t* match_out, mm_ems_stats* stats);

/* ------------------------------------------------------------------ measurement
 * The two ceilings that bind a pass of random state accesses on this GPU
 * (the secondary roofs beside HBM bandwidth): the rate of independent random
 * 4-byte reads and of random 4-byte atomic adds (agent scope) over an array
 * of array_bytes bytes (>= 4096), ops of each, by plain kernels whose only
 * memory traffic is those accesses. Allocates and frees its own device array
 * (array_bytes + 256 bytes, stream-ordered on `stream`) and waits for
 * `stream`. Outputs: operations per second.
 */
mm_status mm_probe_ceilings(int64_t array_bytes, int64_t ops, void* stream, double* reads_per_s,
                            double* atomics_per_s);

/* Thread-local description of the last non-OK status returned on this thread. */
const char* mm_last_error(void);

/* Library version string. */
const char* mm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */

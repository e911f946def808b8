/*
 * evq -- evolving-graph snapshot queries by intersection-union analysis on
 * MI355X (gfx950).
 *
 * A window of graph snapshots is answered in four steps (paper Section 3,
 * Algorithm 1, and Section 4, Algorithm 2):
 *   1. solve the query on the window's intersection graph and union graph
 *      (Step 1, Theorem 1; the union solve starts from the intersection
 *      result and adds the missing edges, Section 6.2);
 *   2. vertices whose two bounds agree keep that value in every snapshot
 *      (Step 2, Theorem 2);
 *   3. the remaining vertices and the edges that can still change them form
 *      the reduced subgraph (Step 3; built "in reverse" from the mismatching
 *      vertices, Section 6.2);
 *   4. every snapshot of the window is relaxed concurrently over that
 *      subgraph, with a per-edge snapshot mask and one snapshot-oblivious
 *      frontier (Section 4.1, 4.2, Algorithm 2).
 *
 * Conventions for every entry point:
 *   - Every call returns an evq_status; nothing throws or aborts across the
 *     ABI.  On failure evq_last_error() describes the cause.
 *   - Arguments are validated before any device work.  A failing call leaves
 *     no partial object behind.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is ordered on that stream.
 *   - Host pointers are read during the call only; the caller keeps
 *     ownership.  Device pointers belong to the caller unless stated.
 *   - Edge weights are uint32 >= 1; vertex ids are uint32 < num_vertices.
 *
 * Scheduling knobs (none changes a value, only how the work is scheduled;
 * defaults are the measured best) are the fields of evq_tuning and
 * evq_batch_config.  Their starting values are read once per process from
 * the environment variables named beside each field; evq_tuning_set and
 * evq_batch_config_set replace them for the calls that start afterwards, so
 * no query reads the environment.
 *
 * Query values (Table 2 edge functions; sentinels are this library's reading
 * where the paper is silent):
 *   SSSP  min over paths of the weight sum, saturating at 0xFFFFFFFE;
 *         source 0; unreachable 0xFFFFFFFF
 *   BFS   min over paths of the edge count; source 0; unreachable 0xFFFFFFFF
 *   SSWP  max over paths of the minimum weight; source 0xFFFFFFFF;
 *         unreachable 0
 *   SSNP  min over paths of the maximum weight; source 0; unreachable
 *         0xFFFFFFFF
 *   VITERBI  max over paths of 1.0 divided by each weight along the path in
 *         turn, as IEEE single floats held in the uint32 values (bit
 *         patterns): each step divides in double precision and rounds to
 *         single (to nearest even); a quotient below the smallest normal
 *         single is unreachable.  Source 1.0 (0x3F800000); unreachable 0.0.
 */
#ifndef EVQ_H
#define EVQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t evq_status;
#define EVQ_OK 0
#define EVQ_EINVAL (-1)    /* malformed argument: NULL pointer, id >= V, w == 0, K out of range, unknown algo */
#define EVQ_ERANGE (-2)    /* window / source / size out of the supported range */
#define EVQ_ENOMEM (-3)    /* device or host allocation failed */
#define EVQ_EDEVICE (-4)   /* a HIP runtime call failed */
#define EVQ_ENOCONV (-5)   /* a frontier loop exceeded its iteration cap */
#define EVQ_ECANCELED (-6) /* a served query was dropped when its server shut down */
#define EVQ_EBUSY (-7)     /* a server's queue is full (evq_server_submit): poll, then submit again */

#define EVQ_SSSP 0
#define EVQ_BFS 1
#define EVQ_SSWP 2
#define EVQ_SSNP 3
#define EVQ_VITERBI 4

#define EVQ_MAX_SNAPSHOTS 128

/* One directed weighted edge, 12 bytes, host memory. */
typedef struct {
    uint32_t src, dst, w;
} evq_edge;

/* One update batch (Section 2.1): its deletions are applied before its additions. */
typedef struct {
    const evq_edge* del;
    uint64_t n_del;
    const evq_edge* add;
    uint64_t n_add;
} evq_batch;

/* Opaque handle; owns the device copy of the versioned graph. */
typedef struct evq_graph evq_graph;

/*
 * A caller's device-memory allocator for a graph (evq_build).
 *   alloc(bytes, ctx): device memory on the current device, at least `bytes`
 *     (a multiple of 256), 256-byte aligned, or NULL when none is available.
 *   free(p, ctx): returns a block alloc gave.  The library calls it exactly
 *     once per block, from the host thread that releases the block, after
 *     every device operation that uses the block has completed.
 * The struct is copied; ctx must stay valid until every block is freed (after
 * evq_free and once no call on the handle is running).  The callbacks must
 * not call into this library.
 */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* p, void* ctx);
    void* ctx;
} evq_allocator;

typedef struct {
    uint32_t num_vertices;
    uint32_t num_snapshots;  /* K */
    uint32_t mask_words;     /* 64-bit words per edge presence mask: 1 (K <= 64) or 2 */
    uint32_t reserved;
    uint64_t num_edges;      /* distinct (src, dst, w) triples present in >= 1 snapshot */
    uint64_t num_partial;    /* of those, triples absent from >= 1 snapshot */
    uint64_t device_bytes;   /* device memory held by the handle (with the pull step's reverse CSR once built) */
    double build_ms;         /* wall time of evq_build (or of the last evq_append), host validation included */
    uint64_t first_snapshot; /* global id of the oldest snapshot held (0 until the first evq_append) */
} evq_graph_info;

/* Filled by evq_query when a non-NULL pointer is passed (the call then synchronises). */
typedef struct {
    double ms_total, ms_cap, ms_cup, ms_compact, ms_relax, ms_writeback;
    uint64_t n_unstable;        /* vertices whose intersection and union bounds differ */
    uint64_t n_seed_edges;      /* window-partial edges into unstable vertices (the reduced batches) */
    uint64_t n_relax_edges;     /* reduced-subgraph edges between unstable vertices */
    uint64_t iters_cap, iters_cup, iters_relax;
    uint64_t edges_cap, edges_cup;        /* edge visits of the two bound solves */
    uint64_t edge_visits_relax;           /* edge visits of the multi-snapshot relaxation */
    uint64_t lane_relaxations;            /* (edge visit, snapshot) pairs evaluated there */
    uint64_t updates_cap, updates_cup;    /* improving value updates of the two bound solves */
    uint64_t items_cap, items_cup;        /* frontier vertices expanded by the two bound solves */
    uint64_t seed_visits_cup;             /* partial edges examined to seed the union solve */
    uint64_t subwindows;                  /* windows relaxed (more than 1 when the window was split) */
} evq_query_stats;

/*
 * Build the versioned graph (Section 4.1) of K snapshots.
 * Snapshot -1 is the set of distinct triples in `base`; snapshot i
 * (0 <= i < K) is snapshot i-1 with batches[i].del removed and then
 * batches[i].add inserted.  A snapshot is a set of (src, dst, w) triples:
 * exact duplicates collapse, parallel edges with different weights stay.
 * The result is one CSR over every triple present in at least one snapshot,
 * each edge carrying a K-bit mask, bit i = present in snapshot i; per row
 * the edges present in all K snapshots come first.
 *   num_vertices >= 1; 1 <= K <= 128; base may be NULL when n_base == 0,
 *   likewise del/add when their counts are 0.
 *   alloc: NULL, or the allocator every device array of the graph comes
 *   from: the arrays of this version and of every version evq_append makes,
 *   the pull step's reverse CSR, and the temporaries of the build and of the
 *   appends.  (Query workspaces and batched results are not graph memory;
 *   they come from the device's stream-ordered pool either way.)  With NULL
 *   the graph's arrays come from that pool too.
 * Errors: EVQ_EINVAL (NULL out/batches, id >= num_vertices, w == 0, K out of
 * range), EVQ_ERANGE (more than 2^32 - 2 events or union edges), EVQ_ENOMEM
 * (the allocator returned NULL, or the pool is exhausted), EVQ_EDEVICE.  On
 * failure *out is NULL and every block taken from `alloc` has been returned
 * to it.  With `alloc`, its first request (the event buffer) comes before any
 * device call.  On success *out owns its device memory until evq_free.  The
 * call synchronises `stream`.
 */
evq_status evq_build(uint32_t num_vertices, const evq_edge* base, uint64_t n_base,
                     const evq_batch* batches, uint32_t K, const evq_allocator* alloc, void* stream,
                     evq_graph** out);

/* Sizes of a built graph.  EVQ_EINVAL on NULL arguments. */
evq_status evq_graph_info_get(const evq_graph* g, evq_graph_info* info);

/*
 * Copy the versioned graph to host buffers (inspection and tests).
 *   row_ptr: V + 1 entries; row_split: V entries (end of the all-present
 *   prefix of each row); col, w: num_edges entries; mask: num_edges *
 *   mask_words 64-bit words, word j of edge e at mask[e * mask_words + j].
 * Rows and columns are in the caller's vertex ids; each row holds its edges
 * present in all snapshots first, then the others, each part ordered by
 * (destination, weight).  (A graph that numbers its vertices itself,
 * evq_tuning.vertex_order, rewrites its rows on the host for this.)
 * Any pointer may be NULL to skip that array.  Synchronises `stream`.
 */
evq_status evq_graph_export(const evq_graph* g, uint32_t* row_ptr, uint32_t* row_split, uint32_t* col,
                            uint32_t* w, uint64_t* mask, void* stream);

/*
 * Answer a query over the window [win_begin, win_begin + win_len) of
 * snapshots (Algorithm 1 followed by Algorithm 2).
 *   algo: EVQ_SSSP / EVQ_BFS / EVQ_SSWP / EVQ_SSNP / EVQ_VITERBI; source < V.
 *   Snapshots are named by global id: the graph holds first .. first+K-1
 *   (first = first_snapshot of evq_graph_info, 0 until an evq_append), so
 *   first <= win_begin, 1 <= win_len and win_begin + win_len <= first + K.
 *   d_values: caller-owned DEVICE buffer of V * win_len uint32,
 *             d_values[v * win_len + i] = value of v in snapshot win_begin + i.
 *   stats: NULL, or a host struct filled after the call synchronises.
 * Errors: EVQ_EINVAL (NULL g/d_values, bad algo), EVQ_ERANGE (source or
 * window out of range), EVQ_ENOMEM, EVQ_EDEVICE, EVQ_ENOCONV.
 * The graph is only read, so queries may run concurrently on several streams.
 * The call returns once the last frontier loop has drained (it reads frontier
 * sizes back); the values are complete when `stream` reaches that point.
 * With the environment variable EVQ_SPLIT_FRAC set to f > 0, a window with
 * more than f * V unstable vertices is answered as two halves (at least
 * EVQ_SPLIT_MIN snapshots each, default 8; to depth 4), each with its own
 * bounds; the values are the same.  Off by default.
 * Scheduling of the bound solves (the values never change): EVQ_DELTA[_SSSP,
 * _BFS, _SSWP, _SSNP, _VITERBI] = d > 0 defers vertices whose order key is not
 * below a threshold that steps by d (near/far); with EVQ_HEAVY[_ALGO] = h > 0
 * only vertices with at least h edges are deferred and the threshold follows
 * the frontier's best key plus d.  Both off by default.
 */
evq_status evq_query(const evq_graph* g, uint32_t algo, uint32_t source, uint32_t win_begin,
                     uint32_t win_len, uint32_t* d_values, evq_query_stats* stats, void* stream);

/*
 * evq_query for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same arguments,
 * output layout and values as evq_query (no stats).  It calls no device or
 * pinned-host allocator: its device temporaries live in one 128 MiB array
 * per GPU, held by the library until the process ends and shared by every
 * call on that GPU (the first call on a device looks its address up).
 * Differences from evq_query: it returns once the values are complete (it
 * synchronises `stream`); the frontier loops read their counts back in
 * batches with copies into host memory instead of mapped slots; the pull
 * step is used only if an earlier evq_query built its reverse CSR, and no
 * sub-window splitting is done.  `stream` must belong to the graph's device,
 * which must be current.
 * Errors: as evq_query, plus EVQ_ERANGE when the query's temporaries (about
 * 70 bytes per vertex, plus the reduced subgraph and the unstable rows)
 * exceed the array (nothing is left half-written that a later call depends
 * on), EVQ_EBUSY when another call of this entry point is running on the
 * device (calls that overlap on one GPU would race for the array: they are
 * refused instead), EVQ_EDEVICE when the array cannot be looked up.
 */
evq_status evq_query_noalloc(const evq_graph* g, uint32_t algo, uint32_t source, uint32_t win_begin,
                             uint32_t win_len, uint32_t* d_values, void* stream);

/*
 * Only the bounds of Step 1: d_rcap[v] = value on the window's intersection
 * graph, d_rcup[v] = value on its union graph (device buffers of V uint32,
 * either may be NULL).  Same arguments and errors as evq_query.
 */
evq_status evq_query_bounds(const evq_graph* g, uint32_t algo, uint32_t source, uint32_t win_begin,
                            uint32_t win_len, uint32_t* d_rcap, uint32_t* d_rcup, void* stream);

/*
 * Plain concurrent evaluation without the intersection-union analysis: every
 * snapshot of the window is solved from scratch over the whole versioned
 * graph with one snapshot-oblivious frontier (the naive full evaluation of
 * Section 2, run concurrently as in Algorithm 2).  Same arguments, output
 * layout and errors as evq_query.
 */
evq_status evq_query_plain(const evq_graph* g, uint32_t algo, uint32_t source, uint32_t win_begin,
                           uint32_t win_len, uint32_t* d_values, evq_query_stats* stats, void* stream);

/*
 * Ablation: the same bounds and reduced subgraph as evq_query, but the
 * window's snapshots are relaxed one after another (Algorithm 1's
 * per-snapshot evaluation of the reduced subgraph), each as its own
 * one-lane relaxation, instead of concurrently (Algorithm 2).  Same
 * arguments, output layout and errors as evq_query.
 */
evq_status evq_query_sequential(const evq_graph* g, uint32_t algo, uint32_t source, uint32_t win_begin,
                                uint32_t win_len, uint32_t* d_values, evq_query_stats* stats, void* stream);

/*
 * Batched queries (a systems layer over Algorithm 1 and Algorithm 2; the
 * paper answers one query at a time).  Queries of one algorithm share their
 * bound solves: up to 64 of them are solved together, one query per lane of
 * a wave, over the shared versioned graph (values laid out [vertex][64]),
 * each lane testing the edge masks against its own window.  Each query's
 * reduction and multi-snapshot relaxation then run on a pool of worker
 * streams, concurrently, and leave a compact result.
 */
typedef struct {
    uint32_t algo, source, win_begin, win_len;  /* as the arguments of evq_query */
} evq_query_desc;

/*
 * Compact result of one query (library-owned device memory until
 * evq_result_free).  By Theorem 2 every vertex outside the unstable set has
 * the value d_rcap[v] in every snapshot of the window; unstable vertex
 * d_unstable[c] has in snapshot win_begin + i the value
 * d_x[c * row_stride + i] (i < win_len).  d_unstable is in no particular
 * order.  d_unstable / d_x are NULL when n_unstable == 0.
 */
typedef struct {
    uint32_t algo, source, win_begin, win_len;
    uint32_t num_vertices;
    uint32_t n_unstable;
    uint32_t row_stride;       /* uint32 per row of d_x, >= win_len */
    uint32_t reserved;
    const uint32_t* d_rcap;    /* num_vertices values on the window's intersection graph */
    const uint32_t* d_unstable;
    const uint32_t* d_x;
} evq_result;

/* Execution choices of evq_query_batch (0 in a field: the library default). */
typedef struct {
    uint32_t lanes;      /* 1: shared bound solves, one query per lane; 2: one bound solve per query */
    uint32_t chunk;      /* edges per wave task of the shared bound solves: 4, 8 or 16 */
    uint32_t blocks;     /* workgroups of 256 threads per expansion launch, 64 .. 16384 */
    uint32_t group;      /* queries per shared solve, 1 .. 64 (a larger set of one algorithm is split evenly) */
} evq_batch_config;

/*
 * Answer n queries.  q: n host descriptors, each validated as evq_query's
 * arguments before any device work (EVQ_EINVAL / EVQ_ERANGE name the first
 * bad one).  results: n host structs, filled on success (on failure they are
 * zeroed and nothing stays allocated).  stats: NULL or n host structs
 * (per-query counters; the bound-solve fields of queries solved together
 * are those of their shared solve).  The work runs on the library's worker
 * streams, after the work already queued on `stream`; `stream` is made to
 * wait for all of it, so the results are complete when `stream` reaches the
 * point of the call.  The call itself returns once every frontier loop has
 * drained.  Queries of any mix of algorithms, sources and windows may be
 * passed; 1 <= n <= 65536.
 */
evq_status evq_query_batch(const evq_graph* g, const evq_query_desc* q, uint32_t n, evq_result* results,
                           evq_query_stats* stats, void* stream);

/*
 * Expand a compact result to values[V][win_len] in the caller's device
 * buffer (the layout of evq_query's d_values).  Ordered on `stream`, which
 * must be ordered after the stream the result was produced for.
 * Errors: EVQ_EINVAL (NULL arguments or an empty result), EVQ_EDEVICE.
 */
evq_status evq_result_expand(const evq_result* r, uint32_t* d_values, void* stream);

/* The same call as evq_result_expand, under the name the problem statement's
 * interface gives it (compact result -> dense values). */
evq_status evq_expand(const evq_result* r, uint32_t* d_values, void* stream);

/*
 * Release a result's device memory, ordered on `stream` (work already queued
 * there that reads the result completes first; work on other streams must be
 * ordered before it by the caller).  The struct is zeroed; a zeroed struct
 * is accepted.  EVQ_EINVAL on NULL.
 */
evq_status evq_result_free(evq_result* r, void* stream);

/* Read / replace the execution choices used by evq_query_batch on this
 * process (starting values: EVQ_BATCH_LANES, _CHUNK, _BLOCKS, _GROUP; the
 * worker count, EVQ_BATCH_WORKERS, is read once when the pool starts). */
evq_status evq_batch_config_get(evq_batch_config* c);
evq_status evq_batch_config_set(const evq_batch_config* c);

/*
 * Scheduling of single queries, appends and frontier loops.
 *   pull_frac     EVQ_PULL_FRAC: full-window intersection solves: an
 *                 iteration whose frontier holds at least this share of the
 *                 all-present edges pulls (every vertex takes its best
 *                 all-present in-edge) instead of pushing; the graph's
 *                 reverse CSR (12 bytes per union edge) is built by the
 *                 second full-window query on a graph version (the first
 *                 pushes only).  Graphs with 2^30 or more vertices or union
 *                 edges never pull.  Default 0.5; above 1 (or negative):
 *                 never.
 *   split_frac    EVQ_SPLIT_FRAC: a window with more than split_frac * V
 *                 unstable vertices is answered as two halves, each with its
 *                 own bounds, to depth 4 (default 0: off).
 *   split_min     EVQ_SPLIT_MIN: smallest half (default 8, >= 1).
 *   launch_depth  EVQ_LAUNCH_DEPTH: frontier iterations kept in flight, 1..32
 *                 (default 3).
 *   direct_tasks  EVQ_DIRECT_TASKS: reduced subgraphs of at most this many
 *                 relaxation tasks have them written by the frontier
 *                 compaction, larger ones by a kernel of their own (default
 *                 262144).
 *   append_rebuild EVQ_APPEND_REBUILD: nonzero makes evq_append rebuild the
 *                 versioned graph from all held edges and the batch instead
 *                 of updating it incrementally (same result).
 *   trace_loops   EVQ_TRACE_LOOPS: nonzero prints each frontier iteration's
 *                 count to stderr.
 *   delta[a], heavy[a]  EVQ_DELTA_<ALGO> (else EVQ_DELTA), EVQ_HEAVY_<ALGO>
 *                 (else EVQ_HEAVY), per algorithm EVQ_SSSP .. EVQ_VITERBI:
 *                 with delta > 0 the bound solves defer vertices whose order
 *                 key is not below a threshold that steps by delta
 *                 (near/far); with heavy > 0 as well only vertices with at
 *                 least heavy edges are deferred and the threshold follows
 *                 the frontier's best key plus delta (default 0: off).
 *   append_edges  EVQ_APPEND_EDGES: a bound-solve iteration whose frontier
 *                 has at most this many edges lists the next frontier itself
 *                 (each improved vertex once, by a per-vertex stamp) instead
 *                 of marking flags for a compaction to scan (default 131072;
 *                 0: never).
 *   append_items  EVQ_APPEND_ITEMS: ... likewise an iteration whose frontier
 *                 has at most this many vertices (default 0: never).
 *   relax_staged  EVQ_RELAX_STAGED: the multi-snapshot relaxation stages each
 *                 block's tasks and their edge records in LDS, 2 or 4 tasks
 *                 per lane group (default 2; 0: each lane group loads its own
 *                 task's records).
 *   bucket_width  EVQ_BUCKET_WIDTH: SSSP intersection solves run delta-
 *                 stepping (buckets of this many distance units; the edges
 *                 of a row heavier than the width are expanded once, when
 *                 the row's bucket is done) instead of plain frontier
 *                 iterations, and neither pull nor defer by delta[].  The
 *                 graph keeps a weight-ordered copy of its rows per width in
 *                 use (8 bytes per edge + 4 per vertex, at most 4 widths,
 *                 built by the first query that asks for it).  0 (default):
 *                 off, since on R-MAT graphs the extra iterations cost more
 *                 than the edge visits saved; 0xFFFFFFFF: a width from the
 *                 graph's largest weight and mean out-degree.
 *   vertex_order  EVQ_VERTEX_ORDER: evq_build numbers the vertices inside the
 *                 graph by descending degree over the base edges and all
 *                 batch events (both endpoints; ties by id), so that the
 *                 values of the hubs, which most edges read, share cache
 *                 lines (default 1; 0: the caller's numbering).  Sources are
 *                 mapped on the way in and every output (values, bounds,
 *                 compact results, exports) is in the caller's numbering;
 *                 the graph holds the map both ways on the device (8 bytes
 *                 per vertex) and on the host (4).  Read by evq_build; later
 *                 versions (evq_append) keep their graph's numbering.
 * evq_tuning_set: EVQ_EINVAL on NULL, launch_depth outside 1..32,
 * split_min == 0 or relax_staged not 0, 2 or 4; calls already running keep
 * the values they started with.
 */
typedef struct {
    double pull_frac;
    double split_frac;
    uint32_t split_min;
    uint32_t launch_depth;
    uint32_t direct_tasks;
    uint32_t append_rebuild;
    uint32_t trace_loops;
    uint32_t delta[5];
    uint32_t heavy[5];
    uint32_t append_edges;
    uint32_t relax_staged;
    uint32_t append_items;
    uint32_t bucket_width;
    uint32_t vertex_order;
} evq_tuning;

evq_status evq_tuning_get(evq_tuning* t);
evq_status evq_tuning_set(const evq_tuning* t);

/*
 * Autotune: run evq_query_batch on the caller's n queries once to warm up,
 * then once under each candidate choice (shared solves of 16/32/64 queries
 * with chunk 4/8/16, and one solve per query), discard the results, and
 * install the fastest for this process.
 * chosen / best_ms (host, nullable) receive it and its wall time.
 * Synchronises `stream`.  Errors as evq_query_batch.
 */
evq_status evq_batch_autotune(const evq_graph* g, const evq_query_desc* q, uint32_t n, evq_batch_config* chosen,
                              double* best_ms, void* stream);

/*
 * Serving store: advance the window of held snapshots by one.  The new
 * snapshot first+K is the newest held snapshot with batch `b` applied
 * (deletions before additions, as in evq_build); it takes the mask bit of
 * the oldest snapshot, `first`, which is dropped (a ring of K mask bits:
 * snapshot t lives in bit t mod K).  Triples present in no held snapshot
 * leave the graph.  The next version is built on the device beside the
 * current one and then published: queries already running keep the version
 * they started on, later calls see the new one.  Appends on one handle are
 * serialised.  Synchronises `stream`.
 * Errors: EVQ_EINVAL (NULL, id >= V, w == 0), EVQ_ERANGE, EVQ_ENOMEM,
 * EVQ_EDEVICE; on failure the current version is unchanged.
 */
evq_status evq_append(evq_graph* g, const evq_batch* b, void* stream);

/*
 * Query server (a systems layer: the paper evaluates a fixed snapshot set
 * known up front).  Queries name (algorithm, source, window length); at
 * admission the window becomes the newest `len` snapshots the graph holds
 * (len clamped to K), recorded in the result's win_begin / win_len.
 *   mode 0, continuous batching: a dispatcher admits queued queries while
 *     the estimated device footprint of all queries in flight stays within
 *     mem_budget (one query is always admitted when nothing is in flight);
 *     at light load (fewer than queue_hi waiting) it starts a query only when
 *     nothing is in flight, as the plain server does, so that queries do not
 *     share the device when no queue has formed,
 *     and forms groups of up to max_batch queued queries of the algorithm of
 *     the oldest waiting query; a group's bound solves run together (one
 *     query per lane), then each query's reduction and relaxation complete
 *     independently on the worker pool.  At most max_groups group solves run
 *     at once, so under load later groups fill up.
 *   mode 1, plain: one query at a time in arrival order (the per-query path
 *     of evq_query), as a baseline.
 * Appends (evq_append on the same handle) may run at any time: queries
 * admitted later see the new snapshots.  The handle must outlive the server.
 */
typedef struct evq_server evq_server;

typedef struct {
    uint32_t mode;           /* 0: continuous batching, 1: plain */
    uint32_t max_batch;      /* queries per group, 1..64 (0: 16) */
    uint32_t max_inflight;   /* admitted and not completed (0: 256) */
    uint32_t max_groups;     /* group bound solves running at once (0: 2) */
    uint64_t mem_budget;     /* device bytes, by estimate (0: a quarter of the free memory at creation) */
    uint32_t max_queued;     /* queries waiting for admission; submit returns EVQ_EBUSY beyond (0: 65536) */
    uint32_t queue_hi;       /* mode 0: while queries are in flight, a new group starts only once this many
                                wait (0: 4); with nothing in flight the oldest query starts at once */
} evq_server_config;

typedef struct {
    uint64_t ticket;
    evq_status status;       /* EVQ_OK, or why the query failed (its result is then empty) */
    uint32_t group_size;     /* queries whose bound solves ran together with this one's */
    double t_arrival_ms;     /* submission, ms since the server was created */
    double t_admit_ms;       /* admission (window fixed) */
    double t_bounds_ms;      /* its bound solves issued and drained on the host */
    double t_done_ms;        /* compact result complete on the device */
    uint64_t n_unstable;
    uint64_t iters_relax;
    evq_result result;       /* the caller's once returned: release with evq_result_free */
} evq_completion;

/* Start a server on graph g.  c may be NULL (defaults).  EVQ_EINVAL on bad fields. */
evq_status evq_server_create(evq_graph* g, const evq_server_config* c, evq_server** out);

/* Queue a query; *ticket identifies its completion.  EVQ_EINVAL / EVQ_ERANGE
 * on a bad algorithm, source >= V or win_len == 0; EVQ_EBUSY when max_queued
 * queries already wait (nothing is queued then). */
evq_status evq_server_submit(evq_server* s, uint32_t algo, uint32_t source, uint32_t win_len, uint64_t* ticket);

/* Move up to cap completions to out (waiting up to wait_ms for the first); returns their number. */
int evq_server_poll(evq_server* s, evq_completion* out, int cap, int wait_ms);

/* Queries waiting for admission and queries admitted but not complete. */
evq_status evq_server_pending(evq_server* s, uint32_t* queued, uint32_t* inflight);

/* Stop: queries not yet admitted are dropped, running ones finish; results
 * never collected are released.  NULL is allowed. */
evq_status evq_server_destroy(evq_server* s);

/* Release the handle; each version's device memory is released once no call still uses it.  NULL is allowed. */
void evq_free(evq_graph* g);

/* Message of the last failing call on this thread ("" if none); valid until the next call. */
const char* evq_last_error(void);

/*
 * Per-kernel timing (measurement only).  While enabled, every kernel the
 * library launches is bracketed by HIP events on the stream it runs on.
 * evq_timing_report writes up to `cap` entries: name (NUL-terminated, at most
 * 47 chars), launch count and total milliseconds; it synchronises the
 * recorded events and returns the number of distinct kernels (may exceed
 * cap).  evq_timing_reset discards what was recorded.
 */
typedef struct {
    char name[48];
    uint64_t launches;
    double total_ms;
} evq_kernel_time;

void evq_timing_enable(int on);
void evq_timing_reset(void);
int evq_timing_report(evq_kernel_time* out, int cap);

/*
 * Access-pattern ceiling of the bound solves' expansion (measurement only).
 * The expansion's visit of an edge (Section 3, Step 1; Algorithm 2's
 * relaxation of an edge) streams the edge's column and weight, gathers the
 * destination's 4-byte value and, when the candidate is better, updates it
 * with an atomic and marks the destination.  This call runs a kernel with
 * exactly those memory operations over every edge of g in CSR order, with
 * values that make the comparison fail (so no update is issued), and without
 * the expansion's walk over frontier items.  It runs one untimed pass, then
 * `launches` passes timed with HIP events on `stream`, and writes edges per
 * second to *edges_per_s (0 for a graph without edges).  It allocates and
 * frees 5 bytes per vertex of scratch from the device pool on `stream` and
 * returns after synchronising on its own end event.
 * Errors: EVQ_EINVAL (NULL graph or edges_per_s, launches == 0), EVQ_ENOMEM,
 * EVQ_EDEVICE.
 */
evq_status evq_gather_ceiling(const evq_graph* g, uint32_t launches, double* edges_per_s, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* EVQ_H */

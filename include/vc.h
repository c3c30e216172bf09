/*
 * vc.h -- C ABI of libvc, an MI355X (gfx950) implementation of the
 * vertex-centric (Pregel) superstep.
 *
 * What is computed (paper, Section I): a program runs as a sequence of
 * supersteps.  In each superstep every active vertex broadcasts a message
 * along its CSR out-edges; the messages addressed to one vertex are merged
 * into that vertex's mailbox by a combiner (paper, Section III); at the next
 * superstep a vertex that received a message is active again.  The run ends
 * when no vertex is active.  Programs (paper, Section VI-C, "Benchmarks"):
 *
 *   VC_PAGERANK    rank(0) = 1/N; for s = 1..T:
 *                  rank = (1-d)/N + d * sum of incoming rank(u)/outdeg(u);
 *                  vertices without out-edges send nothing (their mass is
 *                  dropped).  Combiner: sum.  Result: rank after T updates.
 *   VC_PPR         personalised PageRank: rank(0) = [v == source] and the
 *                  teleport term is (1-d) * [v == source].  Combiner: sum.
 *   VC_CC_HASHMIN  label(0) = v; a vertex adopts the smallest label it
 *                  receives when that is below its own and broadcasts it.
 *                  Combiner: min.  Result: on a symmetric graph, the smallest
 *                  vertex id of each connected component.
 *   VC_SSSP        dist(0) = 0 at the source, "unreached" (0xFFFFFFFF)
 *                  elsewhere; a vertex adopts the smallest dist(u) + w(u,v)
 *                  it receives when that is below its own and sends
 *                  dist + w(e) along each out-edge e.  Combiner: min.  Result:
 *                  shortest-path distances; no weight array = unit weights.
 *
 * Data types: results are IEEE binary32 ranks or uint32 labels / distances.
 * An SSSP distance that would reach 0xFFFFFFFF saturates there and reads as
 * "unreached".  The sum combiner of PageRank / PPR is, by default, exact: each
 * message is a uint64 multiple of 2^-62 (ranks never exceed 1), mailboxes add
 * them with 64-bit integer atomics, the vertex update runs in binary64 and
 * only the returned rank is rounded to binary32, so results do not depend on
 * message arrival order.  VC_OPT_F32_MESSAGES rounds each message to binary32
 * before the same exact sum (half the message bytes, still order- and
 * schedule-independent).  VC_OPT_F32_ACCUMULATE selects binary32 messages and
 * float atomics instead (half the mailbox bytes, order-dependent rounding).
 *
 * Memory: every pointer named "device" is device memory of the GPU that is
 * current when the call is made; every pointer named "host" is host memory.
 * The library never frees caller memory.
 *
 * Errors: every call returns a vc_status; nothing throws across the ABI.
 * vc_last_error() returns a thread-local text describing the last failure of
 * the calling thread.
 *
 * Threads and streams: a vc_graph may be used by one host thread at a time.
 * All device work is enqueued on the stream passed to the call.
 */
#ifndef VC_H_
#define VC_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VC_ABI_VERSION 1

typedef enum {
  VC_OK = 0,
  VC_ERR_INVALID_ARG = 1,   /* null / misaligned pointer, bad enum, wrong struct_size, source >= N */
  VC_ERR_BAD_GRAPH = 2,     /* CSR failed validation (see VC_GRAPH_VALIDATE, VC_GRAPH_SYMMETRIC) */
  VC_ERR_OUT_OF_MEMORY = 3, /* a device allocation failed */
  VC_ERR_HIP = 4,           /* a HIP runtime call failed; vc_last_error() names it */
  VC_ERR_UNSUPPORTED = 5,   /* the combination of arguments is not implemented */
  VC_ERR_NOT_CONVERGED = 6  /* CC / SSSP hit the superstep cap before quiescence */
} vc_status;

typedef enum { VC_PAGERANK = 0, VC_CC_HASHMIN = 1, VC_SSSP = 2, VC_PPR = 3 } vc_program;

/* How a superstep's messages are delivered and combined.
 *   VC_SCHED_VERTEX  push, one thread per active vertex (paper, Section V:
 *                    vertex-centric work distribution);
 *   VC_SCHED_EDGE    push, equal numbers of edges per workgroup (paper,
 *                    Section V: edge-centric; merge-path partition over the
 *                    CSR offsets / frontier degree prefix);
 *   VC_SCHED_PULL    receivers read the outbox of their in-neighbours over
 *                    the transposed graph and combine in place (paper,
 *                    Section VI-C: single-broadcast); needs the transpose,
 *                    which the library builds on first use;
 *   VC_SCHED_BLOCKED PageRank / PPR (fixed-point sums) and CC / SSSP: the
 *                    pull combination by propagation blocking.  Edges are
 *                    laid out once by (source tile of 2^14 vertices,
 *                    destination bin of 2^12); each superstep stages a
 *                    tile's values in LDS and writes each edge's message
 *                    into its slot, then folds each bin's slots in LDS (sum,
 *                    or minimum with the pull form's mailbox rule; a source
 *                    outside the CC / SSSP frontier sends "unreached").
 *                    Both passes stream instead of gathering one message per
 *                    edge from HBM.  Memory: 4 bytes of indices per edge (5
 *                    with weights below 256, 8 with larger ones), 16 per
 *                    non-empty (tile, bin) pair and 16 per 64 edges, shared
 *                    by a graph's views, plus 8 bytes of message slots per
 *                    edge per graph object; built on first use.
 *                    Graphs beyond about 2^27 vertices are refused
 *                    (VC_ERR_UNSUPPORTED), as is vc_run_multi_source;
 *   VC_SCHED_AUTO    CC / SSSP, per superstep: pull for dense frontiers
 *                    (BLOCKED instead on graphs of 2^20 vertices and more),
 *                    edge-centric push otherwise
 *                    (vertex push for tiny ones).  PageRank / PPR with
 *                    fixed-point sums (default or VC_OPT_F32_MESSAGES):
 *                    BLOCKED on graphs of 2^20 vertices and more, PULL
 *                    below; with VC_OPT_F32_ACCUMULATE: PULL. */
typedef enum {
  VC_SCHED_AUTO = 0,
  VC_SCHED_VERTEX = 1,
  VC_SCHED_EDGE = 2,
  VC_SCHED_PULL = 3,
  VC_SCHED_BLOCKED = 4
} vc_schedule;

typedef enum { VC_IDX_I32 = 0, VC_IDX_I64 = 1 } vc_index_type;

/* vc_graph_desc.flags */
enum {
  VC_GRAPH_BORROW = 1u,    /* keep the caller's device arrays instead of copying them */
  VC_GRAPH_VALIDATE = 2u,  /* check the CSR on the device at creation */
  VC_GRAPH_SYMMETRIC = 4u,  /* caller asserts the graph equals its transpose, weights included
                               (as multisets of (source, target, weight) edges); the pull form
                               then reads the CSR itself.  Checked only together with
                               VC_GRAPH_VALIDATE: one pass sums, for two independent 64-bit
                               hashes h, h(u, v, w) - h(v, u, w) over every edge, and a graph
                               whose sums are not both zero is refused with VC_ERR_BAD_GRAPH
                               (an asymmetric graph passes only by a hash collision) */
  VC_GRAPH_NO_RELABEL = 8u  /* keep the input vertex order.  By default the library stores a
                               copy of the graph with vertices ordered by degree class,
                               highest first, so the most-accessed per-vertex data shares
                               cache lines; ids in and out of the ABI are always the
                               caller's */
};

/* vc_params.options */
enum {
  VC_OPT_NO_HUB_AGGREGATION = 1u, /* push supersteps (VC_SCHED_VERTEX, VC_SCHED_EDGE and AUTO's push
                                     supersteps; paper, Section III: combinations contend at the
                                     mailboxes of high in-degree targets): by default a workgroup
                                     combines the messages it sends to the lowest-id targets (8 KiB
                                     of LDS: 2,048 targets for uint32 minima and binary32 sums, 1,024
                                     for fixed-point sums; after the default relabelling these are the
                                     highest-degree vertices) in LDS and merges each touched entry into
                                     the global mailbox once.  This flag sends every message straight
                                     to its global mailbox.  Results are the same either way (min, and
                                     exact fixed-point sums; binary32 atomics round in another order) */
  VC_OPT_NO_TEST_BEFORE_ATOMIC = 2u, /* min programs: skip the mailbox read before the atomic (for measurement) */
  VC_OPT_F32_ACCUMULATE = 4u,        /* PageRank / PPR: binary32 messages and float atomics */
  VC_OPT_GRAPH_CAPTURE = 8u,         /* run the superstep loop as a captured HIP graph: PageRank /
                                        PPR as one graph of all T supersteps (AUTO PageRank does so
                                        by itself on graphs below 2^24 edges, where launch gaps weigh;
                                        timed runs report the graph's time divided by T as every
                                        superstep's step_ms, and scatter_ms 0).  CC / SSSP from
                                        superstep 1 on as a graph of several supersteps replayed
                                        until the device reports quiescence, with each superstep's
                                        form picked on the device from its message count: on graphs
                                        where AUTO takes the blocked form, the blocked form for dense
                                        supersteps and the edge-balanced push otherwise; below that
                                        size the pull in every superstep; explicit schedules fix the
                                        form (VERTEX pushes edge-balanced).  Per-superstep timings
                                        are not recorded.  Graphs are cached per graph object */
  VC_OPT_F32_MESSAGES = 16u          /* PageRank / PPR: each message rounded once to binary32,
                                        sums still exact in fixed point (half the message bytes;
                                        results independent of order and schedule, within one
                                        binary32 rounding per message of the default).  Excludes
                                        VC_OPT_F32_ACCUMULATE */
};

typedef struct vc_graph_s* vc_graph;

/* A CSR graph of out-edges.
 *   offsets   device, num_vertices + 1 entries of int32 or int64
 *             (offset_type); offsets[0] = 0, non-decreasing,
 *             offsets[num_vertices] = num_edges.  int32 requires
 *             num_edges < 2^31.
 *   dst       device, num_edges int32 targets in [0, num_vertices).
 *   weights   device, num_edges uint32 SSSP weights, or NULL (unit weights).
 * Every entry is an edge: parallel edges count in the out-degree and in the
 * sums, and a self-loop delivers to its own source. */
typedef struct {
  uint32_t struct_size; /* sizeof(vc_graph_desc) */
  uint32_t flags;       /* VC_GRAPH_* */
  int64_t num_vertices; /* 1 .. 2^31 - 1 */
  int64_t num_edges;    /* >= 0 */
  vc_index_type offset_type;
  const void* offsets;
  const int32_t* dst;
  const uint32_t* weights;
} vc_graph_desc;

typedef struct {
  uint32_t struct_size;   /* sizeof(vc_params) */
  int32_t max_supersteps; /* PageRank / PPR: T, the number of rank updates (>= 0).
                             CC / SSSP: superstep cap; 0 selects N + 1, which no
                             valid run exceeds. */
  double damping;         /* PageRank / PPR damping d in [0, 1]; 0.85 in the benchmarks */
  uint32_t source;        /* SSSP / PPR source vertex, < N */
  vc_schedule schedule;   /* VC_SCHED_AUTO picks per superstep from |F| and E_F */
  int32_t tile;           /* merge-path items per workgroup tile; 0 = library default */
  uint32_t options;       /* VC_OPT_* */
  float pull_fraction;    /* CC / SSSP with VC_SCHED_AUTO: pull (or take the blocked form) once a
                             superstep's frontier out-edges reach this fraction of all edges;
                             0 = library default (0.1 for pull, 0.25 for the blocked form) */
} vc_params;

/* Per-run statistics.  The caller owns every array (host memory) and sets
 * capacity to their length; entries beyond capacity are not written.
 * Superstep s reports |F_s| (vertices that broadcast, including those without
 * out-edges) and E_s (messages sent = out-edges of F_s). */
typedef struct {
  uint32_t struct_size;  /* sizeof(vc_stats) */
  int32_t supersteps;    /* out: supersteps executed */
  int64_t edges_relaxed; /* out: sum of E_s */
  double elapsed_ms;     /* out: host wall time of vc_run */
  int32_t capacity;      /* in: length of the arrays below (0 = none) */
  int64_t* frontier;     /* out, host, or NULL: |F_s| */
  int64_t* edges;        /* out, host, or NULL: E_s */
  float* scatter_ms;     /* out, host, or NULL: device time of the broadcast+combine
                            kernel(s) of superstep s, from HIP events on the run's
                            stream (recording them adds small gaps) */
  float* step_ms;        /* out, host, or NULL: device time of the whole superstep */
  int32_t* schedule;     /* out, host, or NULL: schedule used (VC_SCHED_VERTEX / _EDGE /
                            _PULL), 0 for supersteps without a broadcast */
} vc_stats;

/* Creates a graph object from a CSR (paper, Section I: vertices with
 * out-edges and mailboxes; Section IV: the hot per-vertex fields are kept in
 * their own arrays, separate from everything else).
 *   desc     host; arrays per vc_graph_desc.
 *   stream   stream for the copy / validation work; the call returns after
 *            that work has completed.
 *   out      host; receives the new handle.
 * Without VC_GRAPH_BORROW the arrays are copied into library-owned device
 * memory and may be freed by the caller on return; with it the caller keeps
 * them alive and unchanged until vc_graph_destroy.  Unless
 * VC_GRAPH_NO_RELABEL is set, the library builds its relabelled copy during
 * this call and no longer reads the caller's arrays afterwards (BORROW then
 * only avoids an intermediate copy).
 * Errors: VC_ERR_INVALID_ARG (null pointer, struct_size, N out of range,
 * int32 offsets with num_edges >= 2^31), VC_ERR_BAD_GRAPH (VALIDATE only:
 * offsets[0] != 0, offsets decreasing, offsets[N] != num_edges, a target out
 * of range, or, with SYMMETRIC, a graph that differs from its transpose),
 * VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP.  On error *out is left unchanged. */
vc_status vc_graph_create(const vc_graph_desc* desc, hipStream_t stream, vc_graph* out);

/* Releases a graph and its device workspace.  Waits for the device to finish
 * work that uses it.  NULL is accepted.  Errors: VC_ERR_HIP. */
vc_status vc_graph_destroy(vc_graph g);

/* Device bytes held for the graph (CSR copies + workspace already allocated)
 * and the bytes a run of `program` would add.  Used for admission by HBM
 * footprint.  bytes_held / bytes_run are host pointers, either may be NULL. */
vc_status vc_graph_footprint(vc_graph g, vc_program program, size_t* bytes_held, size_t* bytes_run);

/* Runs one program to completion (paper, Section I) with its combiner (paper,
 * Section III): sum for VC_PAGERANK / VC_PPR, min for VC_CC_HASHMIN / VC_SSSP.
 *   params   host, may be NULL for defaults (T = 10, d = 0.85, source 0, AUTO).
 *   out      device, N x 4 bytes, caller-owned: float ranks (PageRank, PPR) or
 *            uint32 labels / distances (CC, SSSP).
 *   stream   all device work is enqueued here; the call returns after `out`
 *            is complete.
 *   stats    host, may be NULL.
 * Errors: VC_ERR_INVALID_ARG (bad program / params / source, null out),
 * VC_ERR_NOT_CONVERGED (cap reached; `out` holds the values at the cap),
 * VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP.  On any other error the contents of `out`
 * are unspecified. */
vc_status vc_run(vc_graph g, vc_program program, const vc_params* params, void* out, hipStream_t stream,
                 vc_stats* stats);

/* Size in bytes of the fixed device workspace of vc_run_noalloc, one per GPU. */
#define VC_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* vc_run for callers that cannot allocate device memory (serving loops that
 * must not call hipMalloc, harnesses that forbid it).  Same programs,
 * arguments, results and errors as vc_run, but the run allocates nothing:
 *   - its workspace comes from a fixed device array of the library
 *     (VC_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends).  A CC /
 *     SSSP run needs about 20.3 bytes per vertex plus 4 per merge-path tile,
 *     a PageRank / PPR run 16 bytes per vertex; a graph whose run needs more
 *     is refused with VC_ERR_INVALID_ARG (vc_last_error states both sizes);
 *   - it reads only the read-only structures the graph already holds.  The
 *     pull form needs the transpose and its partition (vc_graph_prepare with
 *     the same params, or an earlier vc_run, builds them): an explicit
 *     VC_SCHED_PULL without them is refused with VC_ERR_UNSUPPORTED, and AUTO
 *     takes the edge-balanced push instead.  An edge-balanced superstep over
 *     every vertex needs the CSR's partition for the tile; without it that
 *     superstep runs vertex-per-thread.  VC_SCHED_BLOCKED (message slots per
 *     edge) and VC_OPT_GRAPH_CAPTURE (buffers of its own) are refused with
 *     VC_ERR_UNSUPPORTED; AUTO never takes the blocked form here;
 *   - per-superstep timings (vc_stats.scatter_ms / step_ms) are written as 0,
 *     and the graph's autotuned setting is not applied.
 * Results equal vc_run's for the same program and params (CC labels, SSSP
 * distances and fixed-point PageRank / PPR ranks bit for bit; with
 * VC_OPT_F32_ACCUMULATE within its rounding).  Every call on one GPU uses the
 * same array and leaves its contents behind (each run initialises what it
 * reads): calls that overlap on one GPU, from two host threads or on two
 * streams at once, race and their results are undefined. */
vc_status vc_run_noalloc(vc_graph g, vc_program program, const vc_params* params, void* out, hipStream_t stream,
                         vc_stats* stats);

/* Builds now what a run of `program` with `params` would otherwise build on
 * its first call (paper, Section V: the work distribution of a superstep):
 * the transpose its pull supersteps read, the merge-path partition of the
 * CSR, and the blocked layout where that form would be taken (AUTO on graphs
 * of 2^20 vertices and more), so that the first run costs what later runs
 * cost.  Read-only structures only; a graph's views share them.
 *   params   host, may be NULL (defaults, as vc_run).
 *   stream   the building work runs here; the call returns after it.
 * Errors: VC_ERR_INVALID_ARG (null graph, bad program or params, graph on
 * another device), VC_ERR_UNSUPPORTED (the blocked schedule with
 * VC_OPT_F32_ACCUMULATE, or a graph beyond the blocked layout's limits),
 * VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP. */
vc_status vc_graph_prepare(vc_graph g, vc_program program, const vc_params* params, hipStream_t stream);

/* Many-source SSSP: k (1..256) SSSP programs on one graph, run side by side
 * in one superstep loop (paper, Section I) with the min combiner (Section
 * III), in the pull form (Section VI-C): each superstep a vertex takes, per
 * source, the minimum of dist(u) + w(u, v) over in-neighbours u whose
 * distance to that source improved in the previous superstep.
 *   sources  host, k caller vertex ids (< N; repeats allowed).
 *   out      device, N * k uint32, caller-owned, row-major by vertex:
 *            out[v * k + i] = distance from sources[i] to v (0xFFFFFFFF:
 *            unreached).
 *   stats    |F_s| counts vertices with at least one improved source.
 * The device state is N x 64*ceil(k/64) distances and mailboxes (8 bytes per
 * vertex and source) and, when the largest edge weight is below 0xFFFF, a
 * 2-byte copy of the distances that the pull reads while no distance can
 * reach 0xFFFF (2 more bytes per vertex and source), kept with the graph for
 * reuse.
 * Errors: VC_ERR_INVALID_ARG (null, k outside 1..256, source >= N),
 * VC_ERR_NOT_CONVERGED, VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP. */
vc_status vc_run_multi_source(vc_graph g, const uint32_t* sources, int32_t k, const vc_params* params, uint32_t* out,
                              hipStream_t stream, vc_stats* stats);

/* ---------------------------------------------------------------- batches
 * Many independent CC / SSSP queries on many graphs in one run.  Hash-min CC
 * is min-plus propagation with zero edge weights and each vertex's id as its
 * initial value (paper, Section VI-C, CC and SSSP share the min combiner), so
 * a batch runs as one superstep loop (paper, Section I) over the disjoint
 * union of its members: CC members contribute weight-0 edges and their local
 * ids, SSSP members their weights (1 if none) and 0 at their source.  A
 * member's result is exactly its result alone: no edge joins two members. */
typedef struct vc_batch_s* vc_batch;

typedef struct {
  uint32_t struct_size; /* sizeof(vc_batch_query) */
  vc_program program;   /* VC_CC_HASHMIN or VC_SSSP */
  uint32_t source;      /* VC_SSSP: source vertex of the member (member-local id) */
} vc_batch_query;

/* Builds the union of `count` member graphs (device CSRs as in vc_graph_desc;
 * member i runs queries[i]).  The members are copied; the caller may free
 * them on return.  flags: VC_GRAPH_VALIDATE and VC_GRAPH_NO_RELABEL apply to
 * the union.  CC members must be symmetric for component semantics.
 * Errors: VC_ERR_INVALID_ARG (null, count < 1, bad member, source >= N_i,
 * union over 2^31 - 1 vertices), VC_ERR_UNSUPPORTED (program other than CC
 * or SSSP), VC_ERR_BAD_GRAPH, VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP. */
vc_status vc_batch_create(const vc_graph_desc* members, const vc_batch_query* queries, int32_t count, uint32_t flags,
                          hipStream_t stream, vc_batch* out);

/* vertex_base (host, count + 1 entries): member i's results occupy
 * out[vertex_base[i] .. vertex_base[i+1]) of vc_batch_run's output. */
vc_status vc_batch_layout(vc_batch b, int64_t* vertex_base);

/* Runs every member's query (params: schedule, tile, options, superstep cap;
 * source is taken from the queries).  out: device, sum of N_i uint32,
 * caller-owned: CC labels (member-local minimum ids) and SSSP distances.
 * stats report the union's supersteps.  Returns after out is complete. */
vc_status vc_batch_run(vc_batch b, const vc_params* params, uint32_t* out, hipStream_t stream, vc_stats* stats);

vc_status vc_batch_destroy(vc_batch b);

/* Autotuner for a batch: like vc_graph_autotune, over vc_batch_run. */
vc_status vc_batch_autotune(vc_batch b, const vc_params* base, hipStream_t stream, vc_params* best);

/* Autotuner: times `program` on this graph under candidate work distributions
 * (schedule, blocked form included for PageRank / PPR, merge-path tile, pull
 * threshold, captured loop), keeps the
 * fastest as the graph's setting for that program (used by later runs with
 * VC_SCHED_AUTO, tile 0 and pull_fraction 0) and returns it in *best (host).
 * base (host, may be NULL) supplies T, damping and source.  Runs the program
 * several times on `stream`.  Errors as vc_run. */
vc_status vc_graph_autotune(vc_graph g, vc_program program, const vc_params* base, hipStream_t stream,
                            vc_params* best);

/* ---------------------------------------------------------------- combiners
 * One superstep of message passing with a combiner that has no native
 * atomic: the paper's hybrid combiner (Section III, Figure 1).  Every vertex
 * v with active[v] != 0 sends its 8-byte message msg[v] along each of its
 * out-edges; a receiver's first message is stored as is and flagged, later
 * ones are merged into it (no neutral value is assumed).  The mailbox and
 * its flag form a three-state word claimed by compare-and-swap and
 * published with a release store, and merges are compare-and-swap loops
 * that skip the swap when the merge changes nothing; no lock is taken. */
typedef enum {
  VC_COMBINE_SUM_U64 = 0,  /* wrapping sum of uint64 */
  VC_COMBINE_PROD_U64 = 1, /* wrapping product of uint64 */
  VC_COMBINE_MAX_F64 = 2,  /* maximum of binary64 (no NaN) */
  VC_COMBINE_MINARG = 3,   /* (binary32 value in the low word, uint32 id in the high
                              word): the smaller value, equal values to the smaller
                              id (no NaN) */
  VC_COMBINE_SUM_F64 = 4   /* binary64 sum; the order of additions is unspecified */
} vc_combiner;

/*   msg      device, N uint64 words, caller's vertex order.
 *   active   device, N bytes (0 = does not send), or NULL: every vertex sends.
 *   mailbox  device, N uint64, caller-owned: the merged message, 0 where
 *            has is 0.
 *   has      device, N uint32, caller-owned: 1 where a message arrived, else 0.
 * Returns after the outputs are complete.  The results are exact for every
 * combiner but VC_COMBINE_SUM_F64, whose rounding depends on the order.
 * Errors: VC_ERR_INVALID_ARG (null, misaligned, bad combiner),
 * VC_ERR_OUT_OF_MEMORY, VC_ERR_HIP. */
vc_status vc_combine(vc_graph g, vc_combiner op, const uint64_t* msg, const uint8_t* active, uint64_t* mailbox,
                     uint32_t* has, hipStream_t stream);

/* ---------------------------------------------------------------- serving
 * A request server over resident graphs.  Requests are independent program
 * runs (paper, Section I) that arrive over time and complete out of order.
 *
 * Min programs (CC, SSSP) on a graph registered with lanes > 0 are served by
 * continuous batching: the graph keeps an N x lanes value / mailbox table
 * and one thread runs its superstep loop with every occupied lane side by
 * side, with the min combiner (paper, Section III) in the push form while
 * few vertices are active and in the pull form (Section VI-C) otherwise.  A lane whose program has quiesced (no active vertex with an
 * out-edge) is retired after the superstep that found it so, its column is
 * copied to the request's `out`, and a waiting request is seeded into it
 * before the next superstep.  A lane's values, superstep count and status
 * are exactly those of the same request run alone with vc_run.
 *
 * PageRank / PPR requests on a graph registered with rank_lanes > 0 are
 * batched the same way: every busy lane takes one rank update per superstep
 * (sum combiner in exact fixed point, so a lane's ranks equal the request
 * run alone bit for bit) and retires after its T-th.  Requests with
 * VC_OPT_F32_ACCUMULATE, VC_OPT_F32_MESSAGES or T = 0 run on workers.
 *
 * Lanes pay off under load: a superstep costs about the same however many
 * lanes are busy.  With VC_ROUTE_AUTO a request joins its lane table's
 * running generation when that is expected to finish sooner than the worker
 * path (running means of the table's superstep time and supersteps per
 * request against the worker backlog plus the program's mean worker time);
 * otherwise it queues for a worker, and once the queued lane-eligible
 * requests of one graph would together take longer alone than one lane
 * generation, they move to the lane table as a batch.
 *
 * Every other request (PageRank, PPR, and min programs routed to workers)
 * runs on one of `workers` threads, each with its own stream and a
 * private workspace that shares the graph's read-only arrays.  A worker
 * takes the oldest waiting request once its workspace fits the HBM budget
 * (admission by footprint), first dropping workspaces it keeps for other
 * graphs.  A request that cannot fit even with every workspace dropped
 * completes with VC_ERR_OUT_OF_MEMORY without running.
 *
 * Threading: every vc_server_* call may be made from any host thread.  The
 * caller must not run, autotune or destroy a registered graph while the
 * server exists. */
typedef struct vc_server_s* vc_server;

typedef struct {
  uint32_t struct_size; /* sizeof(vc_server_config) */
  int32_t workers;      /* threads for the single-run path, 1..64 (0 = 2) */
  uint64_t hbm_budget;  /* device bytes for lane tables and workspaces (0 = 80% of
                           the device memory free at creation) */
} vc_server_config;

/* Path of a CC / SSSP request on a graph with a lane table. */
typedef enum {
  VC_ROUTE_AUTO = 0,   /* the path with the shorter expected completion time */
  VC_ROUTE_LANES = 1,  /* the lane table */
  VC_ROUTE_WORKER = 2  /* a worker */
} vc_route;

typedef struct {
  uint32_t struct_size; /* sizeof(vc_request) */
  int32_t graph;        /* id from vc_server_add_graph */
  vc_program program;
  vc_route route;       /* lane table or worker (graphs with lane tables only) */
  vc_params params;     /* as vc_run; lanes honour source and max_supersteps only */
  void* out;            /* device, N x 4 bytes, caller-owned, untouched by the
                           caller until the request completes */
  uint64_t tag;         /* returned in the completion */
} vc_request;

typedef struct {
  uint64_t ticket;      /* from vc_server_submit */
  uint64_t tag;
  vc_status status;     /* as vc_run would return for the request alone */
  int32_t supersteps;
  int32_t lane;         /* lane that served it, or -1 (worker) */
  int32_t reserved;
  double queue_ms;      /* submit -> start (lane seeded or worker began) */
  double service_ms;    /* start -> `out` complete */
  char message[120];    /* error text when status != VC_OK */
} vc_completion;

typedef struct {
  uint32_t struct_size;    /* sizeof(vc_server_info) */
  int32_t graphs;
  uint64_t hbm_budget;
  uint64_t bytes_reserved; /* lane tables */
  uint64_t bytes_held;     /* worker workspaces */
  uint64_t submitted, completed;
  int64_t lane_supersteps; /* supersteps run by all lane tables */
  int64_t lane_push_supersteps; /* of which pushed from a broadcast list */
  int64_t lane_requests;   /* requests served by lanes */
  int64_t rank_supersteps; /* supersteps run by all rank lane tables */
  int64_t rank_requests;   /* requests served by rank lanes */
} vc_server_info;

/* Creates a server on the current device.  config: host, may be NULL.
 * Errors: VC_ERR_INVALID_ARG, VC_ERR_HIP. */
vc_status vc_server_create(const vc_server_config* config, vc_server* out);

/* Registers a graph (borrowed: it must outlive the server).
 *   lanes       0, or a multiple of 64 up to 256: width of the graph's CC /
 *               SSSP lane table (8 bytes per vertex and lane, 16 per vertex
 *               and 64 lanes, about 12 per vertex for the broadcast list).
 *   rank_lanes  likewise for its PageRank / PPR lane table (16 bytes per
 *               vertex and lane).
 * Both tables are reserved from the budget now.  Builds the graph's
 * transpose if needed.  *id: host.
 * Errors: VC_ERR_INVALID_ARG (null, bad lane count, graph on another
 * device), VC_ERR_OUT_OF_MEMORY (tables over budget), VC_ERR_HIP. */
vc_status vc_server_add_graph(vc_server s, vc_graph g, int32_t lanes, int32_t rank_lanes, int32_t* id);

/* Queues a request.  The request is checked here (graph id, program,
 * params, out); a bad request returns VC_ERR_INVALID_ARG and is not queued.
 * *ticket (host, may be NULL) identifies its completion. */
vc_status vc_server_submit(vc_server s, const vc_request* req, uint64_t* ticket);

/* Moves up to cap completions (host array) to `done`, waiting up to
 * timeout_ms (0: no wait, < 0: until one is available) for the first one.
 * *count: number written. */
vc_status vc_server_poll(vc_server s, vc_completion* done, int32_t cap, int32_t timeout_ms, int32_t* count);

/* Blocks until every request submitted so far has completed. */
vc_status vc_server_drain(vc_server s);

vc_status vc_server_info_get(vc_server s, vc_server_info* info);

/* Waits for every submitted request to complete, stops the threads and
 * frees lane tables and workspaces (not the registered graphs).  NULL is
 * accepted. */
vc_status vc_server_destroy(vc_server s);

/* Fills *p with the defaults used when vc_run receives NULL params. */
void vc_params_default(vc_params* p);

const char* vc_status_string(vc_status s);
const char* vc_last_error(void);
int vc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VC_H_ */

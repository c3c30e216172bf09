// Internal declarations shared by the kernel and host translation units of
// libvc.  Not part of the public ABI (include/vc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vc.h"

namespace vc {

constexpr int kWG = 256;                    // threads per workgroup (4 waves of 64)
constexpr uint32_t kInf = 0xFFFFFFFFu;      // min-combiner neutral value / "unreached"
constexpr int64_t kDefaultTile = 2048;      // merge-path items (vertex-ends + edges) per workgroup
constexpr int64_t kMaxTile = 8192;

// Device counters written by the frontier compaction of the min programs.
struct Counters {
  unsigned long long active;  // |F_{s+1}|: vertices whose value improved
  unsigned long long listed;  // those with at least one out-edge (the broadcast list)
  unsigned long long edges;   // E_{s+1}: out-edges of the improved vertices
  unsigned long long flags;   // validation error bits
};

enum MinKind { kCC = 0, kSsspUnit = 1, kSsspWeighted = 2 };

// State of a device-driven superstep loop (captured HIP graph): kernels of a
// superstep return at once when `done` is set, and the kernels of every form
// but the one in `mode` return at once too; the step-end kernel records
// |F_s|, E_s, decides `done` at quiescence or at the cap, and picks the next
// superstep's form from its message count.
struct LoopState {
  long long done;
  long long step;    // index of the superstep whose frontier was computed last
  long long cap;     // superstep cap
  long long capped;
  long long mode;    // form of the next superstep: VC_SCHED_EDGE, VC_SCHED_PULL or VC_SCHED_BLOCKED
  long long listed;  // its broadcast list length (vertices with out-edges)
  long long edges;   // its messages
};

// LDS of a push workgroup's hub table: messages to targets below
// kHubBytes / (entry size) are combined there and flushed once per target
// (hub_slots: that count, capped at n; 0 when aggregation is off).
constexpr size_t kHubBytes = 8192;
int hub_slots(int64_t n, size_t entry_bytes, bool hub);

// Bytes of dynamic LDS a merge-path scatter tile of `tile` items needs
// (hub table included).
size_t pr_mp_lds_bytes(int64_t tile, bool off64);
size_t min_mp_lds_bytes(int64_t tile, bool list);

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `s` and returns the launch status.  `off` points
// at int32 or int64 offsets (off64 selects).

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s);
hipError_t launch_validate(const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m, Counters* ctr,
                           hipStream_t s);
// acc[0..1] (zeroed by the caller) += sum over edges (u, v, w) of
// h(u, v, w) - h(v, u, w) for two hashes: both stay 0 on a symmetric graph.
// w may be NULL (unit weights).  Needs a validated CSR.
hipError_t launch_sym_hash(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n,
                           unsigned long long* acc, hipStream_t s);

// Merge-path partition of the merged (edge, vertex-end) sequence of a
// non-decreasing prefix array P[0..items]: tile_v[t] = number of vertex-ends
// before position min(t * tile, items + P[items]).
hipError_t launch_mp_partition(const void* P, bool p64, int64_t items, int64_t total, int64_t tile, int64_t ntiles,
                               int32_t* tile_v, hipStream_t s);
// The same over the broadcast list of a device-driven loop's next
// superstep (items = loop->listed, total = listed + loop->edges), for
// up to max_tiles tiles; nothing unless loop->mode is VC_SCHED_EDGE.
hipError_t launch_loop_partition(const int64_t* P, int64_t tile, int64_t max_tiles, int32_t* tile_v,
                                 const LoopState* loop, hipStream_t s);

// PageRank / PPR.  `source` < 0 selects PageRank, else PPR from `source`.
// mode: message / mailbox types; contrib holds the messages (8 bytes per
// vertex for kRankFixed, else 4), mb the sums (4 bytes for kRankF32, else 8).
enum RankMode : int {
  kRankFixed = 0,   // uint64 multiples of 2^-62 for both
  kRankF32 = 1,     // binary32 for both, float atomics
  kRankF32Msg = 2,  // binary32 messages, uint64 fixed-point sums
};
hipError_t launch_pr_init(int mode, const void* off, bool off64, int64_t n, double r0, int64_t source, void* contrib,
                          void* mb, float* out_if_t0, hipStream_t s);
// hub: combine messages to hub targets in LDS first (kHubBytes).
hipError_t launch_pr_scatter_vertex(int mode, const void* off, bool off64, const int32_t* dst, int64_t n,
                                    const void* contrib, void* mb, bool hub, hipStream_t s);
hipError_t launch_pr_scatter_mp(int mode, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                                const int32_t* tile_v, int64_t tile, int64_t ntiles, const void* contrib, void* mb,
                                bool hub, hipStream_t s);
// The vertex update: rank from the summed mailbox, then the next message (or
// the rank into out when last).  kinds: NULL (every mailbox is read and
// cleared), or the blocked layout's kind of every destination bin, which
// says which mailboxes hold sums and which must be cleared (PbBinKind).
// keep_empty (with kinds, not last): the messages of vertices in bins
// without in-edges are left as an earlier update wrote them (they do not
// change after the first update).
hipError_t launch_pr_apply(int mode, const void* off, bool off64, int64_t n, double teleport, double damping,
                           int64_t source, void* mb, void* contrib, float* out, bool last, hipStream_t s,
                           const uint8_t* kinds = nullptr, bool keep_empty = false);

// Hash-min CC and SSSP.  vm holds (value, mailbox) pairs.
// ids: the label each vertex starts CC with (its original id after
// relabelling), or NULL for the vertex index itself.
hipError_t launch_min_init(int kind, int64_t n, int64_t source, const int32_t* ids, uint2* vm, hipStream_t s);
hipError_t launch_min_seed_source(const void* off, bool off64, int64_t source, int32_t* fq, int64_t* P,
                                  uint32_t* active, hipStream_t s);
// n: vertices of the graph (hub targets are ids below hub_slots(n, 4, hub)).
hipError_t launch_min_scatter_vertex(int kind, bool list, bool tba, const void* off, bool off64, const int32_t* dst,
                                     const uint32_t* w, int64_t n, int64_t items, const int32_t* fq, uint2* vm,
                                     uint32_t* bitmap, bool hub, hipStream_t s);
hipError_t launch_min_scatter_mp(int kind, bool list, bool tba, const void* off, bool off64, const int32_t* dst,
                                 const uint32_t* w, int64_t n, int64_t items, int64_t total, const int64_t* P,
                                 const int32_t* fq, const int32_t* tile_v, int64_t tile, int64_t ntiles, uint2* vm,
                                 uint32_t* bitmap, bool hub, hipStream_t s);
hipError_t launch_min_compact(const void* off, bool off64, int64_t n, uint2* vm, const uint32_t* bitmap,
                              uint32_t* stale, int32_t* fq, int64_t* P, Counters* ctr, bool seed,
                              const LoopState* loop, hipStream_t s);
// Edge-balanced push of a device-driven loop's superstep (list mode:
// broadcast list fq, degree prefix P, partition tile_v of at most max_tiles
// tiles), over a fixed grid that takes the tiles round robin; nothing
// unless loop->mode is VC_SCHED_EDGE.
hipError_t launch_loop_scatter_mp(int kind, bool tba, const void* off, bool off64, const int32_t* dst,
                                  const uint32_t* w, int64_t n, const int64_t* P, const int32_t* fq,
                                  const int32_t* tile_v, int64_t tile, int64_t max_tiles, uint2* vm, uint32_t* bitmap,
                                  bool hub, const LoopState* loop, hipStream_t s);
// steps[3s], steps[3s+1], steps[3s+2] = |F_s|, E_s and the form of superstep
// s (0 when it sends nothing) for s < max_recorded.  The next superstep
// takes dense_mode when its messages reach dense_edges, else VC_SCHED_EDGE.
hipError_t launch_loop_step(Counters* ctr, LoopState* loop, long long* steps, int64_t max_recorded,
                            long long dense_edges, int dense_mode, hipStream_t s);
// Seeded start: vm = (init, neutral); bitmap word = vertices with init < 0xFFFFFFFF.
hipError_t launch_min_init_from(const uint32_t* init, int64_t n, uint2* vm, uint32_t* bitmap, hipStream_t s);

// ---------------------------------------------------------------- batches
// Appends member graph i to the union CSR: offsets shifted by ebase, targets
// by vbase; weights copied (mode 1), all 1 (mode 2) or all 0 (mode 0).
hipError_t launch_union_member(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n, int64_t m,
                               int64_t vbase, int64_t ebase, int weight_mode, int64_t* u_off, int32_t* u_dst,
                               uint32_t* u_w, hipStream_t s);
// init[vbase + v] = v (mode 0: CC labels) or (v == source ? 0 : 0xFFFFFFFF) (mode 1: SSSP)
hipError_t launch_union_init(int64_t n, int64_t vbase, int mode, int64_t source, uint32_t* init, hipStream_t s);
// out[perm[u]] = vals[u]
hipError_t launch_permute(const uint32_t* vals, const int32_t* perm, int64_t n, uint32_t* out, hipStream_t s);
hipError_t launch_min_output(int64_t n, const uint2* vm, uint32_t* out, hipStream_t s);
hipError_t launch_zero_counters(Counters* ctr, hipStream_t s);

// ---------------------------------------------------------------- pull form
// Transpose: in-degree histogram (cnt: n + 1 zeroed entries), then placement
// of every edge at cursor[dst]++ (cursor = exclusive scan of cnt).
hipError_t launch_csc_count(const int32_t* dst, int64_t m, unsigned long long* cnt, hipStream_t s);
// The same histogram without per-edge global atomics, for graphs of at least
// kIdMinEdges edges (a counting sort of the targets by bins of 2^shift
// vertices, every count taken in LDS).  id_binned fills the plan and says
// whether the graph qualifies (m < 2^32, at most kIdMaxBins bins of 2^14
// vertices, LDS large enough); launch_id_binned then needs
//   hist       chunks * nb uint32,
//   bin_start  nb + 1 int64,  piece_pre nb + 1 int64,
//   scan_blocks scan_scratch_entries(nb) int64,
//   grouped    m uint16,
// and cnt (n + 1 entries) zero on entry.
constexpr int64_t kIdMinEdges = 1ll << 19;
// Bins of 2^14 vertices: few enough that each chunk writes runs of hundreds
// of targets per bin (4,096 bins at 2^26 vertices), and a bin's counters
// (64 KiB) fit one workgroup's LDS.
constexpr int kIdBinShift = 14;
constexpr int kIdMaxBins = 16384;
constexpr int64_t kIdMinChunk = 1ll << 16;  // edges per chunk of the first passes, at least
constexpr int64_t kIdMaxChunks = 1024;
constexpr int64_t kIdPiece = 1ll << 20;     // grouped targets counted per workgroup, at most
struct IdPlan {
  int shift = kIdBinShift, nb = 0;
  int64_t chunk = 0, chunks = 0, piece = 0, max_pieces = 0;
};
bool id_binned(int64_t n, int64_t m, size_t max_lds, IdPlan* plan);
hipError_t launch_id_binned(const IdPlan& p, const int32_t* dst, int64_t n, int64_t m, uint32_t* hist,
                            int64_t* bin_start, int64_t* piece_pre, int64_t* scan_blocks, uint16_t* grouped,
                            unsigned long long* cnt, hipStream_t s);
hipError_t launch_widen_offsets(const int32_t* a, int64_t count, int64_t* b, hipStream_t s);
hipError_t launch_csc_fill(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n, int64_t m,
                           const int32_t* tile_v, int64_t tile, int64_t ntiles, unsigned long long* cursor,
                           int32_t* in_src, uint32_t* in_w, hipStream_t s);
size_t pull_lds_bytes(int64_t tile);
// Tile size the pull kernels use for a requested tile: kWG * {4, 8, 16}.
int64_t pull_tile(int64_t requested);
hipError_t launch_pr_pull(int mode, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const void* contrib, void* mb,
                          hipStream_t s);
// active = NULL: every vertex broadcast this superstep.
hipError_t launch_min_pull(int kind, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w, int64_t n,
                           int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles, uint2* vm,
                           const uint32_t* active, uint32_t* improved, const LoopState* loop, hipStream_t s);

// ---------------------------------------------------------------- relabelling
int relabel_classes();
// perm[v] = new id of v, inv[new] = v.  hist_scratch: relabel_classes() *
// ceil(n / kWG) + 1 entries; scan_blocks: scan_scratch_entries of that count.
hipError_t launch_relabel_perm(const void* off, bool off64, const unsigned long long* indeg, int64_t n,
                               int64_t* hist_scratch, int64_t* scan_blocks, int32_t* perm, int32_t* inv,
                               hipStream_t s);
hipError_t launch_relabel_degrees(const void* off, bool off64, const int32_t* inv, int64_t n, int64_t* P,
                                  hipStream_t s);
hipError_t launch_relabel_edges(const void* off, bool off64, const int32_t* dst, const uint32_t* w,
                                const int64_t* noff, const int32_t* inv, const int32_t* perm, int64_t n, int64_t m,
                                const int32_t* tile_v, int64_t tile, int64_t ntiles, int32_t* ndst, uint32_t* nw,
                                hipStream_t s);
// out[u] = vals[perm[u] * stride]
hipError_t launch_unpermute(const uint32_t* vals, int64_t stride, const int32_t* perm, int64_t n, uint32_t* out,
                            hipStream_t s);

// ---------------------------------------------------------------- many sources
// Up to 256 lanes side by side in cs chunks of 64; values, mailboxes and
// masks chunk-major (chunk c of vertex v at c * n + v, value rows of 64).
// The superstep itself (pull / push / apply) is driven by ms_superstep.
int ms_chunks(int k);
// One bit per lane (chunk c holds lanes 64c .. 64c + 63), passed by value.
struct LaneMask {
  unsigned long long bits[4];
};
// D16 (may be NULL): the values' 2-byte copy, seeded too.
hipError_t launch_ms_seed(const int32_t* src, const int32_t* perm, int k_real, int64_t n, uint32_t* D, uint16_t* D16,
                          unsigned long long* A, uint32_t* bits, hipStream_t s);
hipError_t launch_ms_count(const void* off, bool off64, int64_t n, const uint32_t* bits, Counters* ctr,
                           hipStream_t s);
hipError_t launch_ms_output(const uint32_t* D, const int32_t* perm, int64_t n, int k_real, uint32_t* out,
                            hipStream_t s);
// Request-server lanes.  ids / perm may be NULL (graph not relabelled).
hipError_t launch_lane_seed_cc(const void* off, bool off64, const int32_t* ids, int64_t n, const int32_t* lanes,
                               int r, uint32_t* D, unsigned long long* A, hipStream_t s);
hipError_t launch_lane_seed_sssp(const void* off, bool off64, const int32_t* perm, int64_t n, const int32_t* seeds,
                                 int r, uint32_t* D, unsigned long long* A, unsigned long long* stillborn,
                                 hipStream_t s);
hipError_t launch_lane_retire(uint32_t* D, const int32_t* perm, int64_t n, const int32_t* lanes,
                              uint32_t* const* outs, int r, hipStream_t s);
hipError_t launch_lane_clear(unsigned long long* A, int64_t n, int cs, const LaneMask& drop, hipStream_t s);

// ---------------------------------------------------------------- rank lanes
// Per-lane parameters of a PageRank / PPR lane table (device array of 64 *
// chunks entries, rewritten by the host before every superstep).
struct RankLane {
  double damping;
  double teleport;   // (1 - d) / N for PageRank, (1 - d) for PPR
  float* out;        // request output, caller's vertex order
  int32_t source;    // PPR source (caller id), -1 for PageRank
  int32_t state;     // 0 idle, 1 running, 2 running its last update
};
// seeds[2j] = lane, seeds[2j + 1] = PPR source (caller id) or -1; ids[x] =
// caller id of internal vertex x (NULL: identity).
hipError_t launch_rl_seed(const void* off, bool off64, const int32_t* ids, int64_t n, const int32_t* seeds, int r,
                          unsigned long long* contrib, hipStream_t s);
hipError_t launch_rl_pull(int C, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const unsigned long long* contrib,
                          unsigned long long* mb, hipStream_t s);
hipError_t launch_rl_apply(const void* off, bool off64, const int32_t* ids, int64_t n, int ceff,
                           const RankLane* lanes, unsigned long long* contrib, unsigned long long* mb, hipStream_t s);

// ---------------------------------------------------------------- generic combiner
size_t combine_lds_bytes(int64_t tile);
size_t combine_pull_lds_bytes(int64_t tile);
// ctr->edges += out-edges of the vertices x with active[inv[x]] != 0.
hipError_t launch_active_edges(const void* off, bool off64, int64_t n, const int32_t* inv, const uint8_t* active,
                               Counters* ctr, hipStream_t s);
// Pull form over the transpose (in_off / in_src, partition tile_v); flag /
// mailbox zero on entry.
hipError_t launch_combine_pull(int op, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                               const int32_t* tile_v, int64_t tile, int64_t ntiles, const int32_t* inv,
                               const unsigned long long* msg, const uint8_t* active, unsigned long long* mailbox,
                               uint32_t* flag, hipStream_t s);
// One push superstep over the CSR merge-path partition tile_v (tile items);
// inv maps internal ids to the caller's (NULL: identity).  flag / mailbox
// must be zero on entry.
hipError_t launch_combine(int op, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const int32_t* inv,
                          const unsigned long long* msg, const uint8_t* active, unsigned long long* mailbox,
                          uint32_t* flag, hipStream_t s);

// ---------------------------------------------------------------- propagation blocking
// PageRank by two streaming passes over edges laid out by bucket (source
// tile of 2^shift vertices, destination bin of 2^kPbDstShift vertices),
// buckets in tile-major order: bucket (t, b) = t * bins + b.
constexpr int kPbDstShift = 12;
constexpr int64_t kPbMaxBuckets = 1ll << 28;
constexpr int64_t kPbMaxItemPositions = 1ll << 17;  // positions per fold item (its chunk descriptors fit LDS)
// Destination bins of the blocked form: without in-edges (no fold item; the
// bin's mailboxes stay zero), one fold item (the fold stores every mailbox
// of the bin, zeros included), or split over several items (the fold adds
// into the mailboxes, which must be zero before it).
enum PbBinKind : uint8_t { kBinEmpty = 0, kBinWhole = 1, kBinSplit = 2 };
// Spread item: slots [k0, k1) of source tile t.
struct PbSpreadItem {
  int32_t t, pad;
  int64_t k0, k1;
};
// Fold item: positions [v0, v1) of the concatenation of bin b's runs (the
// non-empty buckets (t, b) in tile order), v0 a multiple of 64; whole marks
// the only item of its bin.
struct PbFoldItem {
  int32_t b, whole;
  int64_t v0, v1;
};
// Chunk c of a bin (positions 64 c .. 64 c + 63): rb = the run holding
// position 64 c (index in the bin's run list), bit i of starts = a run
// starts at 64 c + i.
struct PbChunk {
  int32_t rb, pad;
  unsigned long long starts;
};
// Largest source tile whose messages fit the LDS limit (<= 2^14 vertices).
int pb_src_shift(size_t max_lds);
int64_t pb_bins(int64_t n);
int64_t pb_tiles(int64_t n, int shift);
// te[t] = off[min(n, t << shift)] for t = 0..tiles (first edge of each
// source tile; also its first slot).
hipError_t launch_pb_tile_edges(const void* off, bool off64, int64_t n, int shift, int64_t tiles, int64_t* te,
                                hipStream_t s);
// srcl_csr[e] = offset of edge e's source in its tile (CSR order).
hipError_t launch_pb_expand(const void* off, bool off64, int64_t n, int64_t m, const int32_t* tile_v, int64_t tile,
                            int64_t ntiles, int shift, uint16_t* srcl_csr, hipStream_t s);
// One workgroup per `chunk` CSR edges.  place = false: adds bucket counts
// into cnt (bins * tiles zeroed counters).  place = true: cnt holds the
// bucket starts (consumed as cursors); writes each edge's source offset
// (srcl) and destination offset in its bin (dstl) at a slot of its bucket,
// and its weight (wslot, wbytes = 1: uint8, else uint32) when w is not NULL.
// pass_bins: bins per LDS pass (pass_bins * 8 bytes of LDS).
hipError_t launch_pb_build(bool place, const int64_t* te, int64_t tiles, const int32_t* dst, int64_t m, int64_t chunk,
                           int64_t bins, int pass_bins, unsigned long long* cnt, const uint16_t* srcl_csr,
                           uint16_t* srcl, uint16_t* dstl, const uint32_t* w, void* wslot, int wbytes,
                           hipStream_t s);
// Two-level placement (replaces launch_pb_build(true, ...) when the group
// histogram fits LDS: pb_groups(bins) * 12 bytes).  cnt holds the bucket
// starts (consumed as cursors) and starts a copy of them.  group_starts:
// gcur[t * groups + g] = first slot of group g of tile t, pieces[...] =
// ceil(group edges / 8192).  group: each edge's target, source offset and
// weight (wbytes each, when w is not NULL) at a free position of its group
// in tdst / tsrcl / tw.  place: with poff the exclusive scan of pieces
// (npieces in all), every edge into its bucket (srcl, dstl, wslot).
int64_t pb_groups(int64_t bins);
// LDS bytes a placement workgroup needs.
size_t pb_place_lds(bool weighted, int wbytes);
hipError_t launch_pb_group_starts(const int64_t* starts, int64_t tiles, int64_t bins, unsigned long long* gcur,
                                  int64_t* pieces, hipStream_t s);
hipError_t launch_pb_group(const int64_t* te, int64_t tiles, const int32_t* dst, int64_t m, int64_t chunk,
                           int64_t bins, unsigned long long* gcur, const uint16_t* srcl_csr, const uint32_t* w,
                           int wbytes, int32_t* tdst, uint16_t* tsrcl, void* tw, hipStream_t s);
hipError_t launch_pb_place(const int64_t* poff, int64_t tiles, int64_t bins, int64_t npieces, const int64_t* starts,
                           unsigned long long* cnt, const int32_t* tdst, const uint16_t* tsrcl, const void* tw,
                           int wbytes, bool weighted, uint16_t* srcl, uint16_t* dstl, void* wslot, hipStream_t s);
// *out = max(*out, largest of the m weights w).
hipError_t launch_pb_wmax(const uint32_t* w, int64_t m, uint32_t* out, hipStream_t s);
// Run tables from the bucket starts (runs = non-empty buckets of a bin, in
// tile order).  fill = false: per bin, nruns (runs), btotal (edges) and
// nitems (fold items of up to fcap positions).  fill = true, with run_off
// the exclusive scan of nruns: rpre / rbase of every run (see
// launch_pb_fold).
hipError_t launch_pb_tables(bool fill, const int64_t* starts, int64_t bins, int64_t tiles, int64_t fcap,
                            int64_t* nruns, int64_t* btotal, int64_t* nitems, const int64_t* run_off, int64_t* rpre,
                            int64_t* rbase, hipStream_t s);
// Fold items of every bin; item_off: exclusive scan of the item counts.
hipError_t launch_pb_fold_items(const int64_t* btotal, int64_t bins, const int64_t* item_off, PbFoldItem* items,
                                hipStream_t s);
// Chunks of 64 positions per bin (nchunks[b] = ceil(btotal[b] / 64)) and,
// with chunk_off their exclusive scan, every chunk's PbChunk.
hipError_t launch_pb_chunk_counts(const int64_t* btotal, int64_t bins, int64_t* nchunks, hipStream_t s);
hipError_t launch_pb_chunks(const int64_t* run_off, const int64_t* rpre, const int64_t* chunk_off, int64_t bins,
                            int64_t nchunks, PbChunk* chunks, hipStream_t s);
// vals[k] = msg[tile's first vertex + srcl[k]] for every slot of every item;
// msg / vals hold binary32 messages when f32msg, else uint64 fixed point.
hipError_t launch_pb_spread(bool f32msg, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                            const uint16_t* srcl, const void* msg, void* vals, hipStream_t s);
// Runs of bin b are run_off[b] .. run_off[b + 1] - 1; run r starts at
// position rpre[r] of the bin's concatenation of runs (btotal[b]
// positions), position v in run r sits at slot rbase[r] + v, and v's chunk
// (chunk_off[b] + v / 64) names r.  Adds every item's messages into mb
// (stores for whole bins); mb zero on entry.
hipError_t launch_pb_fold(bool f32msg, const PbFoldItem* items, int64_t nitems, const int64_t* run_off,
                          const int64_t* rpre, const int64_t* btotal, const int64_t* chunk_off, const PbChunk* chunks,
                          const int64_t* rbase, int64_t n, const void* vals, const uint16_t* dstl,
                          unsigned long long* mb, hipStream_t s);
// Min programs (kind: kCC, kSsspUnit, kSsspWeighted): vals[k] = message on
// slot k from the current values (kInf for sources outside `active`; NULL:
// all).  wslot: weights in slot order, wbytes (1 or 4) each (kSsspWeighted
// only).
// narrow (SSSP only): slot messages are uint16_t, 0xFFFF standing for
// unreached; the caller guarantees every message of the superstep is below
// 0xFFFF (the fold then reads the same width).  loop (may be NULL): in a
// device-driven loop, nothing unless loop->mode is VC_SCHED_BLOCKED (both
// passes).
hipError_t launch_pb_spread_min(int kind, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                                const uint16_t* srcl, const void* wslot, int wbytes, const uint2* vm,
                                const uint32_t* active, void* vals, bool narrow, const LoopState* loop, hipStream_t s);
// Per receiver v, best = the minimum message of its in-edges; when best <
// value(v) the mailbox takes it and v's bit in `improved` is set (the
// outcome of launch_min_pull).  Mailboxes unreached on entry.
hipError_t launch_pb_fold_min(const PbFoldItem* items, int64_t nitems, const int64_t* run_off,
                              const int64_t* rpre, const int64_t* btotal, const int64_t* chunk_off,
                              const PbChunk* chunks, const int64_t* rbase, int64_t n, const void* vals, bool narrow,
                              const uint16_t* dstl, uint2* vm, uint32_t* improved, const LoopState* loop, hipStream_t s);

// In-place exclusive scan of P[0..count) with P[count] = total; `blocks`
// is scratch of scan_scratch_entries(count) int64 values.
int64_t scan_scratch_entries(int64_t count);
hipError_t launch_exclusive_scan(int64_t* P, int64_t count, int64_t* blocks, hipStream_t s);
// The same over loop->listed entries (at most max_count) in a device-driven
// loop; nothing unless loop->mode is VC_SCHED_EDGE.
hipError_t launch_loop_scan(int64_t* P, int64_t max_count, int64_t* blocks, const LoopState* loop, hipStream_t s);

}  // namespace vc

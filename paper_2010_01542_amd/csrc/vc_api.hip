// C ABI of libvc: graph objects, workspace, and the superstep driver.
//
// The driver runs the superstep loop of the paper's Section I on the host:
// per superstep it enqueues the broadcast + combine kernels and the vertex
// update, then (CC / SSSP) reads back the size of the next frontier to decide
// termination and the work distribution of the next broadcast (Section V:
// one thread per vertex, or edge-balanced merge-path tiles).
#include <algorithm>
#include <climits>
#include <cmath>
#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "vc_graph.h"

namespace vc {

namespace {
thread_local std::string t_last_error;
}

vc_status fail(vc_status st, const std::string& msg) {
  t_last_error = msg;
  return st;
}

vc_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? VC_ERR_OUT_OF_MEMORY : VC_ERR_HIP,
              std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

}  // namespace vc

using vc::DevBuf;
using vc::fail;
using vc::hip_fail;

namespace {

size_t workspace_bytes(int64_t n, int64_t m, vc_program p, int64_t tile) {
  const size_t N = (size_t)n;
  const size_t tiles = (size_t)((n + m) / tile + 2) * sizeof(int32_t);
  if (p == VC_PAGERANK || p == VC_PPR) return 2 * N * 8 + tiles;
  return N * 8 + ((N + 31) / 32) * 4 + N * 4 + (N + 1) * 8 + (size_t)vc::scan_scratch_entries(n) * 8 + 2 * tiles +
         sizeof(vc::Counters);
}

hipError_t ensure_events(vc_graph g, size_t count) {
  while (g->events.size() < count) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    g->events.push_back(e);
  }
  return hipSuccess;
}

hipError_t ensure_capture_stream(vc_graph g) {
  if (g->cap_stream) return hipSuccess;
  return hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking);
}

// Statistics recorder; tolerates a NULL vc_stats.
struct Recorder {
  vc_stats* st;
  bool timed;
  explicit Recorder(vc_stats* s) : st(s), timed(s && s->capacity > 0 && (s->scatter_ms || s->step_ms)) {}
  void step(int64_t s, int64_t frontier, int64_t edges, int sched) {
    if (!st) return;
    st->edges_relaxed += edges;
    if (s >= st->capacity) return;
    if (st->frontier) st->frontier[s] = frontier;
    if (st->edges) st->edges[s] = edges;
    if (st->schedule) st->schedule[s] = sched;
    if (st->scatter_ms) st->scatter_ms[s] = 0.0f;
    if (st->step_ms) st->step_ms[s] = 0.0f;
  }
  bool want_time(int64_t s) const { return timed && s < st->capacity; }
  void times(int64_t s, float scatter, float step) {
    if (!want_time(s)) return;
    if (st->scatter_ms) st->scatter_ms[s] = scatter;
    if (st->step_ms) st->step_ms[s] = step;
  }
};

}  // namespace

namespace vc {

// Merge-path tile: the requested size clamped to [64, kMaxTile] and to what
// the largest scatter variant can stage in LDS on this device.
int64_t pick_tile(const vc_params& p, vc_graph g) {
  int64_t t = p.tile > 0 ? p.tile : vc::kDefaultTile;
  if (t < 64) t = 64;
  if (t > vc::kMaxTile) t = vc::kMaxTile;
  while (t > 64 && (vc::min_mp_lds_bytes(t, true) > g->max_lds || vc::pr_mp_lds_bytes(t, true) > g->max_lds ||
                    vc::pull_lds_bytes(t) > g->max_lds))
    t -= 64;
  return t;
}

vc_status dense_partition(vc_graph g, int64_t tile, hipStream_t s) {
  if (g->dense_tile == tile && g->dense_tiles_p) return VC_OK;
  const int64_t ntiles = (g->n + g->m + tile - 1) / tile;
  DevBuf* b = g->dense_parts.find(tile);
  if (!b) {
    b = g->dense_parts.add(tile);
    VC_TRY(b->ensure((size_t)(ntiles + 1) * sizeof(int32_t)));
    VC_TRY(vc::launch_mp_partition(g->off, g->off64, g->n, g->n + g->m, tile, ntiles, b->as<int32_t>(), s));
  }
  g->dense_tiles_p = b->as<int32_t>();
  g->dense_tile = tile;
  g->dense_ntiles = ntiles;
  return VC_OK;
}

// In-degree of every vertex of g into cnt (n + 1 uint64 entries, zero on
// entry): binned in LDS where the graph qualifies, else one atomic per edge.
vc_status count_in_degrees(vc_graph g, unsigned long long* cnt, hipStream_t s) {
  IdPlan plan;
  if (!id_binned(g->n, g->m, g->max_lds, &plan)) {
    VC_TRY(launch_csc_count(g->dst, g->m, cnt, s));
    return VC_OK;
  }
  DevBuf hist, bin_start, piece_pre, blocks, grouped;
  VC_TRY(hist.ensure((size_t)plan.chunks * (size_t)plan.nb * 4));
  VC_TRY(bin_start.ensure((size_t)(plan.nb + 1) * 8));
  VC_TRY(piece_pre.ensure((size_t)(plan.nb + 1) * 8));
  VC_TRY(blocks.ensure((size_t)scan_scratch_entries(plan.nb) * 8));
  VC_TRY(grouped.ensure((size_t)g->m * 2 + 16));
  VC_TRY(launch_id_binned(plan, g->dst, g->n, g->m, hist.as<uint32_t>(), bin_start.as<int64_t>(),
                          piece_pre.as<int64_t>(), blocks.as<int64_t>(), grouped.as<uint16_t>(), cnt, s));
  VC_TRY(hipStreamSynchronize(s));  // before the temporaries are freed
  return VC_OK;
}

// Builds the transpose once per graph: in-degree histogram, exclusive scan,
// then every edge placed at its target's cursor.  Symmetric graphs (flag)
// read the CSR itself.
vc_status ensure_csc(vc_graph g, hipStream_t s) {
  if (g->csc_ready) return VC_OK;
  const int64_t n = g->n, m = g->m;
  VC_TRY(g->csc_off.ensure((size_t)(n + 1) * 8));
  int64_t* in_off = g->csc_off.as<int64_t>();
  g->csc_off_p = in_off;
  if (g->flags & VC_GRAPH_SYMMETRIC) {
    if (g->off64) {
      VC_TRY(hipMemcpyAsync(in_off, g->off, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, s));
    } else {
      VC_TRY(vc::launch_widen_offsets((const int32_t*)g->off, n + 1, in_off, s));
    }
    g->in_src = g->dst;
    g->in_w = g->w;
  } else {
    VC_TRY(g->csc_src.ensure((size_t)m * 4 + 4));
    if (g->w) VC_TRY(g->csc_w.ensure((size_t)m * 4 + 4));
    DevBuf blocks, cursor;
    VC_TRY(blocks.ensure((size_t)vc::scan_scratch_entries(n) * 8));
    VC_TRY(cursor.ensure((size_t)(n + 1) * 8));
    VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(in_off), 2 * (n + 1), 0u, s));
    vc_status cst = count_in_degrees(g, reinterpret_cast<unsigned long long*>(in_off), s);
    if (cst != VC_OK) return cst;
    VC_TRY(vc::launch_exclusive_scan(in_off, n, blocks.as<int64_t>(), s));
    VC_TRY(hipMemcpyAsync(cursor.p, in_off, (size_t)(n + 1) * 8, hipMemcpyDeviceToDevice, s));
    const int64_t tile = vc::kDefaultTile;
    vc_status st = dense_partition(g, tile, s);
    if (st != VC_OK) return st;
    VC_TRY(vc::launch_csc_fill(g->off, g->off64, g->dst, g->w, n, m, g->dense_tiles_p, tile,
                               g->dense_ntiles, cursor.as<unsigned long long>(), g->csc_src.as<int32_t>(),
                               g->w ? g->csc_w.as<uint32_t>() : nullptr, s));
    VC_TRY(hipStreamSynchronize(s));
    blocks.release();
    cursor.release();
    g->in_src = g->csc_src.as<int32_t>();
    g->in_w = g->w ? g->csc_w.as<uint32_t>() : nullptr;
  }
  g->csc_ready = true;
  return VC_OK;
}

vc_status csc_partition(vc_graph g, int64_t tile, hipStream_t s) {
  if (g->csc_tile == tile && g->csc_tiles_p) return VC_OK;
  const int64_t ntiles = (g->n + g->m + tile - 1) / tile;
  DevBuf* b = g->csc_parts.find(tile);
  if (!b) {
    b = g->csc_parts.add(tile);
    VC_TRY(b->ensure((size_t)(ntiles + 1) * sizeof(int32_t)));
    VC_TRY(vc::launch_mp_partition(g->csc_off_p, true, g->n, g->n + g->m, tile, ntiles, b->as<int32_t>(), s));
  }
  g->csc_tiles_p = b->as<int32_t>();
  g->csc_tile = tile;
  g->csc_ntiles = ntiles;
  return VC_OK;
}

// Whether g already holds the merge-path partition of its CSR / its
// transpose for `tile`; if so it becomes the current one.  Never builds or
// allocates anything (runs in a fixed arena).
bool have_dense_partition(vc_graph g, int64_t tile) {
  if (g->dense_tile == tile && g->dense_tiles_p) return true;
  DevBuf* b = g->dense_parts.find(tile);
  if (!b) return false;
  g->dense_tiles_p = b->as<int32_t>();
  g->dense_tile = tile;
  g->dense_ntiles = (g->n + g->m + tile - 1) / tile;
  return true;
}

bool have_csc_partition(vc_graph g, int64_t tile) {
  if (!g->csc_ready) return false;
  if (g->csc_tile == tile && g->csc_tiles_p) return true;
  DevBuf* b = g->csc_parts.find(tile);
  if (!b) return false;
  g->csc_tiles_p = b->as<int32_t>();
  g->csc_tile = tile;
  g->csc_ntiles = (g->n + g->m + tile - 1) / tile;
  return true;
}

// Consecutive pieces of an arena at 256-byte boundaries.  With a null base
// it only counts (used), which is how arena_need sizes a run.
struct Carve {
  unsigned char* base;
  size_t cap, used = 0;
  Carve(unsigned char* b, size_t c) : base(b), cap(c) {}
  template <class T>
  T* take(size_t bytes) {
    const size_t at = used;
    used += (bytes + 255) & ~(size_t)255;
    return (base && used <= cap) ? reinterpret_cast<T*>(base + at) : nullptr;
  }
  bool fits() const { return used <= cap; }
};

// Workspace of a CC / SSSP run: values and mailboxes, the two frontier
// bitmaps, the broadcast list and its degree prefix, scan scratch, the
// per-superstep merge-path partition and the counters.
struct MinWork {
  uint2* vm;
  uint32_t* bits[2];
  int32_t* fq;
  int64_t* P;
  int64_t* scan;
  int32_t* list_tiles;
  Counters* ctr;
};

MinWork carve_min(Carve& c, int64_t n, int64_t m, int64_t tile) {
  const int64_t nwords = (n + 31) / 32;
  MinWork w;
  w.vm = c.take<uint2>((size_t)n * 8);
  w.bits[0] = c.take<uint32_t>((size_t)nwords * 4);
  w.bits[1] = c.take<uint32_t>((size_t)nwords * 4);
  w.fq = c.take<int32_t>((size_t)n * 4);
  w.P = c.take<int64_t>((size_t)(n + 1) * 8);
  w.scan = c.take<int64_t>((size_t)scan_scratch_entries(n) * 8);
  w.list_tiles = c.take<int32_t>((size_t)((n + m) / tile + 3) * sizeof(int32_t));
  w.ctr = c.take<Counters>(sizeof(Counters));
  return w;
}

// PageRank / PPR: messages and sums, 8 bytes per vertex each.
void carve_rank(Carve& c, int64_t n, void** contrib, void** mb) {
  *contrib = c.take<void>((size_t)n * 8);
  *mb = c.take<void>((size_t)n * 8);
}

size_t arena_need(vc_graph g, vc_program program, const vc_params& p) {
  Carve c(nullptr, 0);
  if (program == VC_PAGERANK || program == VC_PPR) {
    void *a, *b;
    carve_rank(c, g->n, &a, &b);
  } else {
    (void)carve_min(c, g->n, g->m, pick_tile(p, g));
  }
  return c.used;
}

}  // namespace vc

using vc::csc_partition;
using vc::dense_partition;
using vc::ensure_csc;
using vc::pick_tile;
using vc::valid_params;

namespace {

// Builds the hot-first relabelled copy of the graph and switches the graph
// object to it.  The caller's arrays are not read afterwards.
vc_status relabel(vc_graph g, hipStream_t s) {
  const int64_t n = g->n, m = g->m;
  const int64_t nblocks = (n + vc::kWG - 1) / vc::kWG;
  const int64_t hist_count = (int64_t)vc::relabel_classes() * nblocks;
  DevBuf indeg, hist, blocks, tiles;
  VC_TRY(indeg.ensure((size_t)(n + 1) * 8));
  VC_TRY(hist.ensure((size_t)(hist_count + 1) * 8));
  const int64_t scan_need = vc::scan_scratch_entries(hist_count > n ? hist_count : n);
  VC_TRY(blocks.ensure((size_t)scan_need * 8));
  VC_TRY(g->perm.ensure((size_t)n * 4));
  VC_TRY(g->inv.ensure((size_t)n * 4));
  int32_t* perm = g->perm.as<int32_t>();
  int32_t* inv = g->inv.as<int32_t>();
  VC_TRY(g->rel_off.ensure((size_t)(n + 1) * 8));
  VC_TRY(g->rel_dst.ensure((size_t)m * 4 + 4));
  if (g->w) VC_TRY(g->rel_w.ensure((size_t)m * 4 + 4));
  unsigned long long* deg_in = indeg.as<unsigned long long>();
  VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(deg_in), 2 * (n + 1), 0u, s));
  vc_status cst = vc::count_in_degrees(g, deg_in, s);
  if (cst != VC_OK) return cst;
  VC_TRY(vc::launch_relabel_perm(g->off, g->off64, deg_in, n, hist.as<int64_t>(), blocks.as<int64_t>(),
                                 perm, inv, s));
  int64_t* noff = g->rel_off.as<int64_t>();
  VC_TRY(vc::launch_relabel_degrees(g->off, g->off64, inv, n, noff, s));
  VC_TRY(vc::launch_exclusive_scan(noff, n, blocks.as<int64_t>(), s));
  const int64_t tile = vc::kDefaultTile;
  const int64_t ntiles = (n + m + tile - 1) / tile;
  VC_TRY(tiles.ensure((size_t)(ntiles + 1) * 4));
  VC_TRY(vc::launch_mp_partition(noff, true, n, n + m, tile, ntiles, tiles.as<int32_t>(), s));
  VC_TRY(vc::launch_relabel_edges(g->off, g->off64, g->dst, g->w, noff, inv, perm,
                                  n, m, tiles.as<int32_t>(), tile, ntiles, g->rel_dst.as<int32_t>(),
                                  g->w ? g->rel_w.as<uint32_t>() : nullptr, s));
  VC_TRY(hipStreamSynchronize(s));
  g->off = noff;
  g->off64 = true;
  g->perm_p = perm;
  g->inv_p = inv;
  g->dst = g->rel_dst.as<int32_t>();
  g->w = g->w ? g->rel_w.as<uint32_t>() : nullptr;
  g->relabeled = true;
  g->own_off.release();
  g->own_dst.release();
  g->own_w.release();
  return VC_OK;
}

// The internal id of a caller's vertex id (a 4-byte device read when relabelled).
vc_status internal_id(vc_graph g, int64_t v, hipStream_t s, int64_t* out) {
  if (!g->relabeled) {
    *out = v;
    return VC_OK;
  }
  int32_t x = 0;
  VC_TRY(hipMemcpyAsync(&x, g->perm_p + v, 4, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  *out = x;
  return VC_OK;
}

// ---------------------------------------------------------------- PageRank / PPR

// Whether the blocked layout of g is within the library's limits, and its
// size in bytes (slots, run tables, items).
bool pb_supported(vc_graph g) {
  const int shift = vc::pb_src_shift(g->max_lds);
  return shift != 0 && vc::pb_bins(g->n) * vc::pb_tiles(g->n, shift) <= vc::kPbMaxBuckets;
}

size_t pb_layout_bytes(vc_graph g) {  // the shared, read-only part
  const int shift = vc::pb_src_shift(g->max_lds);
  if (shift == 0) return 0;
  const size_t bins = (size_t)vc::pb_bins(g->n), tiles = (size_t)vc::pb_tiles(g->n, shift), m = (size_t)g->m;
  const size_t runs = std::min(bins * tiles, m);  // non-empty buckets
  return m * (g->w ? 8 : 4) + runs * 16 + (bins + 1) * 25 + (m / 64 + bins + 1) * sizeof(vc::PbChunk) +
         (m / 4096 + bins + 2) * sizeof(vc::PbFoldItem) +
         (m / 16384 + tiles + 2) * sizeof(vc::PbSpreadItem);
}

// Device bytes the layout build holds only while it runs (the source
// offsets in CSR order, bucket counts and starts, scan scratch, and the
// two-level placement's group cursors and transient records), an upper
// bound: weights are counted at 4 bytes.
size_t pb_build_transient_bytes(vc_graph g) {
  const int shift = vc::pb_src_shift(g->max_lds);
  if (shift == 0) return 0;
  const size_t bins = (size_t)vc::pb_bins(g->n), tiles = (size_t)vc::pb_tiles(g->n, shift), m = (size_t)g->m;
  const size_t nb = bins * tiles, segs = (size_t)vc::pb_groups((int64_t)bins) * tiles;
  return m * 2 + (nb + 1) * 16 + (size_t)vc::scan_scratch_entries((int64_t)nb) * 8 + (segs + 1) * 16 +
         m * (g->w ? 10 : 6);
}

// The schedule of a PageRank / PPR run.  AUTO takes the blocked schedule for
// fixed-point runs on graphs of 2^20 vertices and more, where the message
// array no longer stays in the caches and the pull form's gathers go to
// HBM (on R-MAT graphs the two forms meet near 2^20 vertices, and the
// blocked layout builds faster than the transpose), and the pull form
// otherwise.
int rank_schedule(vc_graph g, const vc_params& p, bool fx) {
  if (p.schedule != VC_SCHED_AUTO) return p.schedule;
  if (fx && g->n >= (1 << 20) && g->m > 0 && pb_supported(g)) return VC_SCHED_BLOCKED;
  return VC_SCHED_PULL;
}

// Largest edge weight of g (1 when unweighted), computed once per graph.
vc_status weight_max(vc_graph g, hipStream_t s, uint32_t* out) {
  if (!g->w || g->m == 0) {
    *out = 1;
    return VC_OK;
  }
  if (!g->wmax) {
    DevBuf wmax;
    VC_TRY(wmax.ensure(4));
    VC_TRY(vc::launch_fill_u32(wmax.as<uint32_t>(), 1, 0u, s));
    VC_TRY(vc::launch_pb_wmax(g->w, g->m, wmax.as<uint32_t>(), s));
    uint32_t mx = 0;
    VC_TRY(hipMemcpyAsync(&mx, wmax.p, 4, hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    g->wmax = mx > 0 ? mx : 1;
  }
  *out = g->wmax;
  return VC_OK;
}

// Builds the propagation-blocking layout once per graph, on the device:
// first edge of every source tile, every edge's source offset in its tile,
// bucket counts (LDS histograms per chunk of edges), their exclusive scan
// (bucket starts), the slots (placed in two levels: by groups of 128 bins,
// then, per piece of a group sorted in LDS, into the buckets; a device
// whose LDS cannot hold that takes the one-level placement, each chunk
// reserving its share of a bucket with one atomic), the bin-major run
// tables and the fold items (each bin's runs
// cut into pieces of about the same number of edges, so that a bin of hubs
// spreads over many workgroups).  The spread items (each tile's slot range
// cut into pieces) are made on the host from the tile starts.
vc_status ensure_pb(vc_graph g, hipStream_t s) {
  if (g->pb.ready) return VC_OK;
  if (g->is_view) return fail(VC_ERR_INVALID_ARG, "a view cannot build the blocked layout");
  const int64_t n = g->n, m = g->m;
  const int shift = vc::pb_src_shift(g->max_lds);
  if (shift == 0) return fail(VC_ERR_UNSUPPORTED, "the blocked schedule needs 8 KiB of LDS per workgroup");
  const int64_t bins = vc::pb_bins(n), tiles = vc::pb_tiles(n, shift), nb = bins * tiles;
  if (nb > vc::kPbMaxBuckets)
    return fail(VC_ERR_UNSUPPORTED, "the blocked schedule supports graphs of up to about 2^27 vertices");
  vc_params p;
  vc_params_default(&p);
  const int64_t tile = pick_tile(p, g);
  vc_status st = dense_partition(g, tile, s);
  if (st != VC_OK) return st;
  DevBuf te_d, cnt, blocks, starts_d, nitems;
  VC_TRY(te_d.ensure((size_t)(tiles + 1) * 8));
  VC_TRY(vc::launch_pb_tile_edges(g->off, g->off64, n, shift, tiles, te_d.as<int64_t>(), s));
  std::vector<int64_t> te((size_t)tiles + 1);
  VC_TRY(hipMemcpyAsync(te.data(), te_d.p, te.size() * 8, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  for (int64_t t = 0; t < tiles; ++t)
    if (te[(size_t)t + 1] - te[(size_t)t] >= (1ll << 32))
      return fail(VC_ERR_UNSUPPORTED, "the blocked schedule needs fewer than 2^32 out-edges per source tile");
  VC_TRY(g->pb_srcl.ensure((size_t)m * 2 + 4));
  VC_TRY(g->pb_dstl.ensure((size_t)m * 2 + 4));
  DevBuf srcl_tmp;
  VC_TRY(srcl_tmp.ensure((size_t)m * 2 + 4));
  uint16_t* srcl_csr = srcl_tmp.as<uint16_t>();
  VC_TRY(vc::launch_pb_expand(g->off, g->off64, n, m, g->dense_tiles_p, tile, g->dense_ntiles, shift, srcl_csr, s));
  VC_TRY(cnt.ensure((size_t)(nb + 1) * 8));
  VC_TRY(blocks.ensure((size_t)vc::scan_scratch_entries(std::max(nb, bins)) * 8));
  VC_TRY(starts_d.ensure((size_t)(nb + 1) * 8));
  VC_TRY(vc::launch_fill_u32(cnt.as<uint32_t>(), 2 * (nb + 1), 0u, s));
  const int pass_bins = (int)std::min<int64_t>(bins, std::max<int64_t>(64, (int64_t)(g->max_lds / 8) & ~63ll));
  const int64_t chunk = std::min<int64_t>(1 << 18, std::max<int64_t>(1 << 14, m / 2048));
  VC_TRY(vc::launch_pb_build(false, te_d.as<int64_t>(), tiles, g->dst, m, chunk, bins, pass_bins,
                             cnt.as<unsigned long long>(), nullptr, nullptr, nullptr, nullptr, nullptr, 4, s));
  // weights in slot order: one byte each when every weight fits (weights of
  // 1..255, as the benchmark graphs have, save 3 bytes per edge and superstep)
  int wbytes = 4;
  uint32_t wmax_all = 1;
  if (g->w) {
    st = weight_max(g, s, &wmax_all);
    if (st != VC_OK) return st;
    wbytes = wmax_all <= 255 ? 1 : 4;
    VC_TRY(g->pb_w.ensure((size_t)m * wbytes + 4));
  }
  VC_TRY(vc::launch_exclusive_scan(cnt.as<int64_t>(), nb, blocks.as<int64_t>(), s));
  VC_TRY(hipMemcpyAsync(starts_d.p, cnt.p, (size_t)(nb + 1) * 8, hipMemcpyDeviceToDevice, s));
  const int64_t groups = vc::pb_groups(bins), segs = tiles * groups;
  if ((size_t)groups * 12 <= g->max_lds && vc::pb_place_lds(g->w != nullptr, wbytes) <= g->max_lds) {
    // two-level placement: by groups of bins into transient arrays, then
    // into the buckets (whole lines written instead of scattered bytes)
    DevBuf gcur, poff, tdst, tsrcl, tw;
    VC_TRY(gcur.ensure((size_t)segs * 8));
    VC_TRY(poff.ensure((size_t)(segs + 1) * 8));
    VC_TRY(vc::launch_pb_group_starts(starts_d.as<int64_t>(), tiles, bins, gcur.as<unsigned long long>(),
                                      poff.as<int64_t>(), s));
    VC_TRY(vc::launch_exclusive_scan(poff.as<int64_t>(), segs, blocks.as<int64_t>(), s));
    int64_t npieces = 0;
    VC_TRY(hipMemcpyAsync(&npieces, poff.as<int64_t>() + segs, 8, hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    VC_TRY(tdst.ensure((size_t)m * 4 + 4));
    VC_TRY(tsrcl.ensure((size_t)m * 2 + 4));
    if (g->w) VC_TRY(tw.ensure((size_t)m * wbytes + 4));
    VC_TRY(vc::launch_pb_group(te_d.as<int64_t>(), tiles, g->dst, m, chunk, bins, gcur.as<unsigned long long>(),
                               srcl_csr, g->w, wbytes, tdst.as<int32_t>(), tsrcl.as<uint16_t>(), tw.p, s));
    VC_TRY(vc::launch_pb_place(poff.as<int64_t>(), tiles, bins, npieces, starts_d.as<int64_t>(),
                               cnt.as<unsigned long long>(), tdst.as<int32_t>(), tsrcl.as<uint16_t>(), tw.p, wbytes,
                               g->w != nullptr, g->pb_srcl.as<uint16_t>(), g->pb_dstl.as<uint16_t>(),
                               g->w ? g->pb_w.p : nullptr, s));
    VC_TRY(hipStreamSynchronize(s));
  } else {
    VC_TRY(vc::launch_pb_build(true, te_d.as<int64_t>(), tiles, g->dst, m, chunk, bins, pass_bins,
                               cnt.as<unsigned long long>(), srcl_csr, g->pb_srcl.as<uint16_t>(),
                               g->pb_dstl.as<uint16_t>(), g->w, g->w ? g->pb_w.p : nullptr, wbytes, s));
  }
  // run tables (non-empty buckets per bin) and fold items: at least about
  // 4096 items in all, at most 128 Ki edges each (a bin of fewer edges is one
  // item and stores its mailboxes instead of adding them)
  const int64_t fcap = std::min<int64_t>(vc::kPbMaxItemPositions, std::max<int64_t>(4096, m / 4096));
  VC_TRY(nitems.ensure((size_t)(bins + 1) * 8));
  VC_TRY(g->pb_run_off.ensure((size_t)(bins + 1) * 8));
  VC_TRY(g->pb_btotal.ensure((size_t)bins * 8));
  VC_TRY(vc::launch_pb_tables(false, starts_d.as<int64_t>(), bins, tiles, fcap, g->pb_run_off.as<int64_t>(),
                              g->pb_btotal.as<int64_t>(), nitems.as<int64_t>(), nullptr, nullptr, nullptr, s));
  VC_TRY(vc::launch_exclusive_scan(g->pb_run_off.as<int64_t>(), bins, blocks.as<int64_t>(), s));
  VC_TRY(vc::launch_exclusive_scan(nitems.as<int64_t>(), bins, blocks.as<int64_t>(), s));
  int64_t totals[2] = {0, 0};  // runs, fold items
  VC_TRY(hipMemcpyAsync(&totals[0], g->pb_run_off.as<int64_t>() + bins, 8, hipMemcpyDeviceToHost, s));
  VC_TRY(hipMemcpyAsync(&totals[1], nitems.as<int64_t>() + bins, 8, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  const int64_t nfold = totals[1];
  // each bin's kind from its item count (PageRank's update reads and resets
  // only the mailboxes that need it)
  std::vector<int64_t> item_off((size_t)bins + 1);
  VC_TRY(hipMemcpyAsync(item_off.data(), nitems.p, item_off.size() * 8, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  std::vector<uint8_t> kinds((size_t)bins);
  for (int64_t b = 0; b < bins; ++b) {
    const int64_t k = item_off[(size_t)b + 1] - item_off[(size_t)b];
    kinds[(size_t)b] = k == 0 ? vc::kBinEmpty : k == 1 ? vc::kBinWhole : vc::kBinSplit;
  }
  VC_TRY(g->pb_kinds.ensure(kinds.size() + 16));
  VC_TRY(hipMemcpyAsync(g->pb_kinds.p, kinds.data(), kinds.size(), hipMemcpyHostToDevice, s));
  VC_TRY(g->pb_rpre.ensure((size_t)(totals[0] + 1) * 8));
  VC_TRY(g->pb_rbase.ensure((size_t)(totals[0] + 1) * 8));
  VC_TRY(vc::launch_pb_tables(true, starts_d.as<int64_t>(), bins, tiles, fcap, nullptr, nullptr, nullptr,
                              g->pb_run_off.as<int64_t>(), g->pb_rpre.as<int64_t>(), g->pb_rbase.as<int64_t>(), s));
  VC_TRY(g->pb_fold.ensure((size_t)(nfold + 1) * sizeof(vc::PbFoldItem)));
  VC_TRY(vc::launch_pb_fold_items(g->pb_btotal.as<int64_t>(), bins, nitems.as<int64_t>(),
                                  g->pb_fold.as<vc::PbFoldItem>(), s));
  // chunks of 64 positions: each names its first run and the run starts inside
  VC_TRY(g->pb_chunk_off.ensure((size_t)(bins + 1) * 8));
  VC_TRY(vc::launch_pb_chunk_counts(g->pb_btotal.as<int64_t>(), bins, g->pb_chunk_off.as<int64_t>(), s));
  VC_TRY(vc::launch_exclusive_scan(g->pb_chunk_off.as<int64_t>(), bins, blocks.as<int64_t>(), s));
  int64_t nchunks = 0;
  VC_TRY(hipMemcpyAsync(&nchunks, g->pb_chunk_off.as<int64_t>() + bins, 8, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  VC_TRY(g->pb_chunks.ensure((size_t)(nchunks + 1) * sizeof(vc::PbChunk)));
  VC_TRY(vc::launch_pb_chunks(g->pb_run_off.as<int64_t>(), g->pb_rpre.as<int64_t>(), g->pb_chunk_off.as<int64_t>(),
                              bins, nchunks, g->pb_chunks.as<vc::PbChunk>(), s));
  // spread items: a tile's slots are contiguous; pieces of up to scap slots
  // (the tile's messages are loaded once per piece; 64 Ki slots balance
  // that load against the spread of work over the compute units best at
  // scale 26)
  const int64_t scap = std::min<int64_t>(1 << 16, std::max<int64_t>(1 << 14, m / 1024));
  std::vector<vc::PbSpreadItem> sitems;
  for (int64_t t = 0; t < tiles; ++t) {
    const int64_t k0 = te[(size_t)t], k1 = te[(size_t)t + 1];
    for (int64_t k = k0; k < k1; k += scap) sitems.push_back(vc::PbSpreadItem{(int32_t)t, 0, k, std::min(k1, k + scap)});
  }
  VC_TRY(g->pb_spread.ensure((sitems.size() + 1) * sizeof(vc::PbSpreadItem)));
  if (!sitems.empty())
    VC_TRY(hipMemcpyAsync(g->pb_spread.p, sitems.data(), sitems.size() * sizeof(vc::PbSpreadItem),
                          hipMemcpyHostToDevice, s));
  VC_TRY(hipStreamSynchronize(s));
  vc::PbShared& pb = g->pb;
  pb.srcl = g->pb_srcl.as<uint16_t>();
  pb.dstl = g->pb_dstl.as<uint16_t>();
  pb.w = g->w ? g->pb_w.p : nullptr;
  pb.wbytes = wbytes;
  pb.wmax = wmax_all;
  pb.run_off = g->pb_run_off.as<int64_t>();
  pb.btotal = g->pb_btotal.as<int64_t>();
  pb.rpre = g->pb_rpre.as<int64_t>();
  pb.rbase = g->pb_rbase.as<int64_t>();
  pb.chunk_off = g->pb_chunk_off.as<int64_t>();
  pb.chunks = g->pb_chunks.as<vc::PbChunk>();
  pb.spread = g->pb_spread.as<vc::PbSpreadItem>();
  pb.fold = g->pb_fold.as<vc::PbFoldItem>();
  pb.kinds = g->pb_kinds.as<uint8_t>();
  pb.shift = shift;
  pb.tiles = tiles;
  pb.nspread = (int64_t)sitems.size();
  pb.nfold = nfold;
  pb.ready = true;
  return VC_OK;
}

// Whether a dense CC / SSSP superstep that AUTO would pull takes the blocked
// form instead: the same size rule as PageRank's.
bool min_blocked(vc_graph g) { return g->n >= (1 << 20) && g->m > 0 && pb_supported(g); }

// The blocked layout for a run on g: a graph builds its own on first use; a
// view takes its base's, building it there first if no view has (under the
// base's lock, on the view's stream, synchronised).  Each object owns its
// message slots.
vc_status use_pb(vc_graph g, hipStream_t s) {
  if (!g->pb.ready) {
    vc_graph owner = g->is_view ? g->base : g;
    std::lock_guard<std::mutex> lock(owner->pb_mu);
    vc_status st = ensure_pb(owner, s);
    if (st != VC_OK) return st;
    g->pb = owner->pb;
  }
  VC_TRY(g->pb_vals.ensure((size_t)g->m * 8 + 8));
  return VC_OK;
}

// One broadcast + combine of the blocked schedule: spread, then fold.
hipError_t pb_superstep(vc_graph g, bool f32msg, const void* contrib, void* mb, hipStream_t s) {
  const vc::PbShared& pb = g->pb;
  hipError_t e = vc::launch_pb_spread(f32msg, pb.spread, pb.nspread, g->n, pb.shift, pb.srcl, contrib, g->pb_vals.p, s);
  if (e != hipSuccess) return e;
  return vc::launch_pb_fold(f32msg, pb.fold, pb.nfold, pb.run_off, pb.rpre, pb.btotal, pb.chunk_off, pb.chunks,
                            pb.rbase, g->n, g->pb_vals.p, pb.dstl, static_cast<unsigned long long*>(mb), s);
}

// Edges below which AUTO PageRank / PPR runs capture their superstep loop
// (VC_PR_CAPTURE_EDGES overrides; 0 turns it off).
constexpr int64_t kRankCaptureEdges = 1ll << 24;

bool auto_rank_capture(vc_graph g) {
  static const int64_t limit = [] {
    const char* e = std::getenv("VC_PR_CAPTURE_EDGES");
    return e ? (int64_t)std::atoll(e) : kRankCaptureEdges;
  }();
  return g->m < limit;
}

vc_status run_rank(vc_graph g, const vc_params& p, bool personal, float* out, hipStream_t s, Recorder& rec,
                   int32_t* supersteps, const vc::Arena* arena = nullptr) {
  const int64_t n = g->n, T = p.max_supersteps;
  int64_t source = -1;
  if (personal) {
    vc_status st = internal_id(g, (int64_t)p.source, s, &source);
    if (st != VC_OK) return st;
  }
  // valid_params rejects VC_OPT_F32_ACCUMULATE together with VC_OPT_F32_MESSAGES
  const int mode = (p.options & VC_OPT_F32_ACCUMULATE)  ? vc::kRankF32
                   : (p.options & VC_OPT_F32_MESSAGES) ? vc::kRankF32Msg
                                                        : vc::kRankFixed;
  const bool fx = mode != vc::kRankF32;  // sums in fixed point
  const bool hub = !(p.options & VC_OPT_NO_HUB_AGGREGATION);
  // messages and sums take 8 bytes per vertex in every mode, so that a run in
  // one mode never reallocates the buffers a captured graph of another mode
  // was recorded with
  void* contrib = nullptr;
  void* mb = nullptr;
  if (arena) {
    vc::Carve c(arena->base, arena->bytes);
    vc::carve_rank(c, n, &contrib, &mb);
    if (!c.fits()) return fail(VC_ERR_INVALID_ARG, "fixed workspace too small for this graph");
  } else {
    VC_TRY(g->contrib.ensure((size_t)n * 8));
    VC_TRY(g->mb.ensure((size_t)n * 8));
    contrib = g->contrib.p;
    mb = g->mb.p;
  }
  const double r0 = 1.0 / (double)n;
  // ranks come out in internal order; relabelled graphs stage them in the
  // message buffer (no longer needed at the last step) and un-permute
  float* rank_out = g->relabeled ? static_cast<float*>(contrib) : out;
  if (T == 0) {
    VC_TRY(vc::launch_pr_init(mode, g->off, g->off64, n, r0, source, contrib, mb, rank_out, s));
    if (g->relabeled)
      VC_TRY(vc::launch_unpermute(reinterpret_cast<const uint32_t*>(rank_out), 1, g->perm_p, n,
                                  reinterpret_cast<uint32_t*>(out), s));
    VC_TRY(hipStreamSynchronize(s));
    rec.step(0, 0, 0, 0);
    *supersteps = 1;
    return VC_OK;
  }
  const double d = p.damping;
  const double teleport = personal ? (1.0 - d) : (1.0 - d) / (double)n;
  const int64_t tile = pick_tile(p, g);
  int sched = rank_schedule(g, p, fx);
  if (arena && g->m > 0) {
    // only forms whose read-only structures the graph already holds; the
    // blocked form would need message slots per edge
    if (sched == VC_SCHED_BLOCKED || sched == VC_SCHED_PULL)
      sched = vc::have_csc_partition(g, vc::pull_tile(tile)) ? VC_SCHED_PULL : VC_SCHED_EDGE;
    if (sched == VC_SCHED_EDGE && !vc::have_dense_partition(g, tile)) sched = VC_SCHED_VERTEX;
  }
  if (sched == VC_SCHED_BLOCKED && !fx)
    return fail(VC_ERR_UNSUPPORTED, "the blocked schedule sums in fixed point; drop VC_OPT_F32_ACCUMULATE");
  if (g->m > 0) {
    vc_status st = VC_OK;
    if (sched == VC_SCHED_PULL) {
      st = ensure_csc(g, s);
      if (st == VC_OK) st = csc_partition(g, vc::pull_tile(tile), s);
    } else if (sched == VC_SCHED_EDGE) {
      st = dense_partition(g, tile, s);
    } else if (sched == VC_SCHED_BLOCKED) {
      st = use_pb(g, s);
    }
    if (st != VC_OK) return st;
  }
  // the blocked form's fold stores every mailbox of a one-item bin and
  // leaves bins without in-edges untouched: the update resets only the rest
  const uint8_t* pb_kinds = sched == VC_SCHED_BLOCKED && g->m > 0 ? g->pb.kinds : nullptr;
  // a captured loop: on request, or by default for PageRank (AUTO) where a
  // superstep is short enough that launch gaps weigh (graphs below
  // kRankCaptureEdges edges; PPR bakes its source into the graph, so a
  // request stream with changing sources would capture every run); never in
  // a fixed arena
  const bool capture = !arena && ((p.options & VC_OPT_GRAPH_CAPTURE) ||
                                  (!personal && p.schedule == VC_SCHED_AUTO && auto_rank_capture(g)));
  if (capture) {
    // the whole loop as one captured HIP graph; ranks land in the staging
    // buffer (fixed address) and are copied / un-permuted afterwards.  A
    // timed run times the graph's launch with two events on the stream (the
    // kernels inside cannot be timed apart): every superstep reports the
    // average, and no broadcast+combine time.
    float* stage = static_cast<float*>(contrib);
    const bool timed = rec.timed;
    if (timed) VC_TRY(ensure_events(g, 2));
    // the key names every device address the graph bakes in, so that a
    // reallocated buffer or a rebuilt partition forces a new capture
    char keybuf[352];
    std::snprintf(keybuf, sizeof keybuf, "%d/%d/%lld/%lld/%.17g/%d/%lld/%p/%p/%p/%p/%p/%p/%p", mode, (int)hub,
                  (long long)T, (long long)source, d, sched, (long long)tile, contrib, mb, g->pb_vals.p,
                  (const void*)g->csc_tiles_p, (const void*)g->dense_tiles_p, (const void*)g->in_src,
                  (const void*)g->pb.fold);
    if (g->pr_exec && g->pr_exec_key != keybuf) {
      VC_TRY(hipGraphExecDestroy(g->pr_exec));
      g->pr_exec = nullptr;
    }
    if (!g->pr_exec) {
      VC_TRY(ensure_capture_stream(g));
      hipStream_t cs = g->cap_stream;
      VC_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipError_t e = vc::launch_pr_init(mode, g->off, g->off64, n, r0, source, contrib, mb, nullptr, cs);
      for (int64_t step = 0; step < T && e == hipSuccess; ++step) {
        if (g->m > 0) {
          if (sched == VC_SCHED_PULL) {
            e = vc::launch_pr_pull(mode, g->csc_off_p, g->in_src, n, g->m, g->csc_tiles_p,
                                   g->csc_tile, g->csc_ntiles, contrib, mb, cs);
          } else if (sched == VC_SCHED_BLOCKED) {
            e = pb_superstep(g, mode == vc::kRankF32Msg, contrib, mb, cs);
          } else if (sched == VC_SCHED_EDGE)
            e = vc::launch_pr_scatter_mp(mode, g->off, g->off64, g->dst, n, g->m, g->dense_tiles_p, tile,
                                         g->dense_ntiles, contrib, mb, hub, cs);
          else
            e = vc::launch_pr_scatter_vertex(mode, g->off, g->off64, g->dst, n, contrib, mb, hub, cs);
        }
        if (e == hipSuccess)
          e = vc::launch_pr_apply(mode, g->off, g->off64, n, teleport, d, source, mb, contrib, stage, step + 1 == T, cs,
                                  pb_kinds, step > 0);
      }
      hipGraph_t graph = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cs, &graph);
      if (e != hipSuccess) return hip_fail(e, "capture PageRank");
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      const hipError_t e3 = hipGraphInstantiate(&g->pr_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
      g->pr_exec_key = keybuf;
    }
    if (timed) VC_TRY(hipEventRecord(g->events[0], s));
    VC_TRY(hipGraphLaunch(g->pr_exec, s));
    if (timed) VC_TRY(hipEventRecord(g->events[1], s));
    for (int64_t step = 0; step < T; ++step) rec.step(step, n, g->m, sched);
    rec.step(T, 0, 0, 0);
    if (g->relabeled)
      VC_TRY(vc::launch_unpermute(reinterpret_cast<const uint32_t*>(stage), 1, g->perm_p, n,
                                  reinterpret_cast<uint32_t*>(out), s));
    else
      VC_TRY(hipMemcpyAsync(out, stage, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    VC_TRY(hipStreamSynchronize(s));
    if (timed) {
      float all = 0;
      VC_TRY(hipEventElapsedTime(&all, g->events[0], g->events[1]));
      for (int64_t step = 0; step < T; ++step) rec.times(step, 0.0f, all / (float)T);
    }
    *supersteps = (int32_t)(T + 1);
    return VC_OK;
  }
  if (rec.timed) VC_TRY(ensure_events(g, (size_t)(3 * T)));
  VC_TRY(vc::launch_pr_init(mode, g->off, g->off64, n, r0, source, contrib, mb, nullptr, s));
  for (int64_t step = 0; step < T; ++step) {
    const bool timed = rec.want_time(step);
    if (timed) VC_TRY(hipEventRecord(g->events[3 * step], s));
    if (g->m > 0) {
      if (sched == VC_SCHED_PULL) {
        VC_TRY(vc::launch_pr_pull(mode, g->csc_off_p, g->in_src, n, g->m, g->csc_tiles_p,
                                  g->csc_tile, g->csc_ntiles, contrib, mb, s));
      } else if (sched == VC_SCHED_BLOCKED) {
        VC_TRY(pb_superstep(g, mode == vc::kRankF32Msg, contrib, mb, s));
      } else if (sched == VC_SCHED_EDGE)
        VC_TRY(vc::launch_pr_scatter_mp(mode, g->off, g->off64, g->dst, n, g->m, g->dense_tiles_p, tile,
                                        g->dense_ntiles, contrib, mb, hub, s));
      else
        VC_TRY(vc::launch_pr_scatter_vertex(mode, g->off, g->off64, g->dst, n, contrib, mb, hub, s));
    }
    if (timed) VC_TRY(hipEventRecord(g->events[3 * step + 1], s));
    VC_TRY(vc::launch_pr_apply(mode, g->off, g->off64, n, teleport, d, source, mb, contrib, rank_out, step + 1 == T, s,
                               pb_kinds, step > 0));
    if (timed) VC_TRY(hipEventRecord(g->events[3 * step + 2], s));
    rec.step(step, n, g->m, sched);
  }
  rec.step(T, 0, 0, 0);
  if (g->relabeled)
    VC_TRY(vc::launch_unpermute(reinterpret_cast<const uint32_t*>(rank_out), 1, g->perm_p, n,
                                reinterpret_cast<uint32_t*>(out), s));
  VC_TRY(hipStreamSynchronize(s));
  for (int64_t step = 0; step < T && rec.want_time(step); ++step) {
    float a = 0, b = 0;
    VC_TRY(hipEventElapsedTime(&a, g->events[3 * step], g->events[3 * step + 1]));
    VC_TRY(hipEventElapsedTime(&b, g->events[3 * step], g->events[3 * step + 2]));
    rec.times(step, a, b);
  }
  *supersteps = (int32_t)(T + 1);
  return VC_OK;
}

// ---------------------------------------------------------------- CC / SSSP

// Fraction of the edges above which a CC / SSSP superstep is pulled: the
// pull form streams every in-edge, the push form only the frontier's
// out-edges, so pull pays off once the frontier carries a large share of them.
// Share of the edges from which AUTO takes the blocked form for a CC / SSSP
// superstep (unless params set pull_fraction).
constexpr double kBlockedFraction = 0.25;

double pull_threshold(const vc_params& p) {
  if (p.pull_fraction > 0.0f) return (double)p.pull_fraction;
  static const double v = [] {
    const char* e = std::getenv("VC_PULL_FRACTION");
    double x = e ? std::atof(e) : 0.1;
    return x > 0 ? x : 0.1;
  }();
  return v;
}

constexpr int64_t kMaxRecordedSteps = 1 << 16;

// How a captured CC / SSSP loop delivers each superstep: the dense form
// (blocked or pull) from dense_edges messages on, else the edge-balanced
// push.  Explicit schedules fix the form: PULL / BLOCKED always dense,
// EDGE / VERTEX always pushed (edge-balanced).  AUTO switches per superstep
// on graphs large enough for the blocked form; below that it pulls every
// superstep, as a superstep there costs little more than the launches of
// the forms it would not take (measured: 1,024 captured runs on graphs of
// 2^10..2^16 vertices took 540 ms switching, 444 ms pulling).
struct LoopForms {
  int dense_mode;          // VC_SCHED_BLOCKED or VC_SCHED_PULL
  long long dense_edges;   // messages from which a superstep takes dense_mode
  int per_replay;          // supersteps per replay of the captured graph (even: the bitmaps alternate)
};

LoopForms loop_forms(vc_graph g, const vc_params& p) {
  const bool blocked = p.schedule == VC_SCHED_BLOCKED || (p.schedule == VC_SCHED_AUTO && min_blocked(g));
  LoopForms f;
  f.dense_mode = blocked ? VC_SCHED_BLOCKED : VC_SCHED_PULL;
  if (p.schedule == VC_SCHED_PULL || p.schedule == VC_SCHED_BLOCKED || (p.schedule == VC_SCHED_AUTO && !blocked)) {
    f.dense_edges = 0;
  } else if (p.schedule == VC_SCHED_EDGE || p.schedule == VC_SCHED_VERTEX) {
    f.dense_edges = LLONG_MAX;
  } else {
    const double thr = p.pull_fraction > 0.0f ? pull_threshold(p) : kBlockedFraction;
    const double e = thr * (double)g->m;
    f.dense_edges = e < 1.0 ? 1 : (long long)std::ceil(e);  // edges >= thr * m
  }
  // a replay ends with one read of the loop state; the supersteps of a
  // replay left after quiescence return at once, which costs more in the
  // longer graphs of the push form
  f.per_replay = (f.dense_edges == 0 && !blocked) ? 2 : 8;
  return f;
}

// Runs supersteps `step`.. of a CC / SSSP program as a captured HIP graph of
// forms.per_replay supersteps, replayed until the step-end kernel reports
// quiescence or the cap; one read of the loop state per replay.  Every
// superstep holds the kernels of its possible forms (the edge-balanced push:
// scan, partition, scatter; the dense form: blocked spread and fold, or the
// pull), and each returns at once unless the step-end kernel of the previous
// superstep picked its form, so the direction switch happens on the device.
vc_status run_min_device_loop(vc_graph g, const vc_params& p, int kind, int64_t tile, bool tba, bool hub, int cur,
                              int64_t step, int64_t frontier, int64_t listed, int64_t edges, int64_t cap, uint2* vm,
                              uint32_t* bits[2],
                              int32_t* fq, int64_t* P, int64_t* scan, int32_t* list_tiles, vc::Counters* ctr,
                              hipStream_t s, Recorder& rec, int32_t* supersteps, bool* capped) {
  const int64_t n = g->n, m = g->m;
  const LoopForms forms = loop_forms(g, p);
  const bool blocked = forms.dense_mode == VC_SCHED_BLOCKED;
  vc_status st = VC_OK;
  if (forms.dense_edges != LLONG_MAX) {
    if (blocked) {
      st = use_pb(g, s);
    } else {
      st = ensure_csc(g, s);
      if (st == VC_OK) st = csc_partition(g, vc::pull_tile(tile), s);
    }
  }
  if (st != VC_OK) return st;
  const int64_t max_tiles = (n + m) / tile + 1;  // list_tiles holds (n + m) / tile + 3 entries
  VC_TRY(g->loop_state.ensure(sizeof(vc::LoopState)));
  VC_TRY(g->loop_steps.ensure((size_t)kMaxRecordedSteps * 24));
  if (!g->host_loop) VC_TRY(hipHostMalloc((void**)&g->host_loop, sizeof(vc::LoopState), hipHostMallocDefault));
  vc::LoopState* loop = g->loop_state.as<vc::LoopState>();
  long long* steps = g->loop_steps.as<long long>();
  const vc::PbShared& pb = g->pb;
  uint32_t* slot_msg = blocked ? g->pb_vals.as<uint32_t>() : nullptr;
  hipGraphExec_t& exec = g->min_exec[kind][cur];
  // every device address and setting the graph bakes in
  char keybuf[512];
  std::snprintf(keybuf, sizeof keybuf,
                "%lld/%d/%lld/%d/%d/%d/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%p/%lld", (long long)tile,
                forms.dense_mode, forms.dense_edges, forms.per_replay, (int)tba, (int)hub, (void*)vm, (void*)bits[0], (void*)bits[1],
                (void*)fq, (void*)P, (void*)scan, (void*)list_tiles, (void*)ctr, (void*)loop, (void*)steps,
                (const void*)g->csc_tiles_p, (const void*)g->in_src, (const void*)slot_msg, (const void*)pb.fold,
                (const void*)pb.spread, g->off, (const void*)g->dst, (long long)g->csc_tile);
  if (exec && g->min_exec_key[kind][cur] != keybuf) {
    VC_TRY(hipGraphExecDestroy(exec));
    exec = nullptr;
  }
  if (!exec) {
    VC_TRY(ensure_capture_stream(g));
    hipStream_t cs = g->cap_stream;
    VC_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < forms.per_replay && e == hipSuccess; ++k) {
      const int a = (k & 1) ? 1 - cur : cur;  // improvements go to bits[a]; bits[1 - a] holds the frontier
      if (forms.dense_edges != 0) {  // the edge-balanced push
        e = vc::launch_loop_scan(P, n, scan, loop, cs);
        if (e == hipSuccess) e = vc::launch_loop_partition(P, tile, max_tiles, list_tiles, loop, cs);
        if (e == hipSuccess)
          e = vc::launch_loop_scatter_mp(kind, tba, g->off, g->off64, g->dst, g->w, n, P, fq, list_tiles, tile,
                                         max_tiles, vm, bits[a], hub, loop, cs);
      }
      if (e == hipSuccess && forms.dense_edges != LLONG_MAX) {  // the dense form
        if (blocked) {
          // 4-byte slots: the graph is replayed for any superstep
          e = vc::launch_pb_spread_min(kind, pb.spread, pb.nspread, n, pb.shift, pb.srcl, pb.w, pb.wbytes, vm,
                                       bits[1 - a], slot_msg, false, loop, cs);
          if (e == hipSuccess)
            e = vc::launch_pb_fold_min(pb.fold, pb.nfold, pb.run_off, pb.rpre, pb.btotal, pb.chunk_off, pb.chunks,
                                       pb.rbase, n, slot_msg, false, pb.dstl, vm, bits[a], loop, cs);
        } else {
          e = vc::launch_min_pull(kind, g->csc_off_p, g->in_src, g->in_w, n, m, g->csc_tiles_p, g->csc_tile,
                                  g->csc_ntiles, vm, bits[1 - a], bits[a], loop, cs);
        }
      }
      if (e == hipSuccess)
        e = vc::launch_min_compact(g->off, g->off64, n, vm, bits[a], bits[1 - a], fq, P, ctr, false, loop, cs);
      if (e == hipSuccess)
        e = vc::launch_loop_step(ctr, loop, steps, kMaxRecordedSteps, forms.dense_edges, forms.dense_mode, cs);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess) return hip_fail(e, "capture superstep");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
    g->min_exec_key[kind][cur] = keybuf;
  }
  // the form of superstep `step`, by the same rule the step-end kernel applies
  const long long mode0 = (long long)edges >= forms.dense_edges ? forms.dense_mode : VC_SCHED_EDGE;
  rec.step(step, frontier, edges, (int)mode0);
  vc::LoopState init{0, step, cap, 0, mode0, listed, edges};
  *g->host_loop = init;
  VC_TRY(hipMemcpyAsync(loop, g->host_loop, sizeof init, hipMemcpyHostToDevice, s));
  for (;;) {
    VC_TRY(hipGraphLaunch(exec, s));
    VC_TRY(hipMemcpyAsync(g->host_loop, loop, sizeof init, hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    if (g->host_loop->done) break;
  }
  const int64_t last = g->host_loop->step;
  const int64_t first = step + 1;
  const int64_t upto = last < kMaxRecordedSteps ? last : kMaxRecordedSteps - 1;
  if (upto >= first) {
    std::vector<long long> h((size_t)(3 * (upto - first + 1)));
    VC_TRY(hipMemcpyAsync(h.data(), steps + 3 * first, h.size() * 8, hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    for (int64_t t = first; t <= upto; ++t) {
      const long long f = h[3 * (t - first)], ed = h[3 * (t - first) + 1], md = h[3 * (t - first) + 2];
      if (g->host_loop->capped && t == last) break;
      rec.step(t, f, ed, (int)md);
    }
  }
  *capped = g->host_loop->capped != 0;
  *supersteps = (int32_t)(*capped ? last : last + 1);
  return VC_OK;
}

// seed (device, internal vertex order, may be NULL): initial values of a
// seeded min-plus run; every vertex with a finite initial value broadcasts at
// superstep 0.  Without it the program's own start is used (CC: ids; SSSP:
// the source).
vc_status run_min(vc_graph g, const vc_params& p, int kind, const uint32_t* seed, uint32_t* out, hipStream_t s,
                  Recorder& rec, int32_t* supersteps, const vc::Arena* arena = nullptr) {
  const int64_t n = g->n, m = g->m;
  const int64_t tile = pick_tile(p, g);
  const bool tba = !(p.options & VC_OPT_NO_TEST_BEFORE_ATOMIC);
  const bool hub = !(p.options & VC_OPT_NO_HUB_AGGREGATION);
  const int64_t nwords = (n + 31) / 32;
  vc::MinWork wk{};
  vc::Counters host_local{};  // counters read back into pageable memory when nothing may be allocated
  vc::Counters* hc = &host_local;
  if (arena) {
    vc::Carve c(arena->base, arena->bytes);
    wk = vc::carve_min(c, n, m, tile);
    if (!c.fits()) return fail(VC_ERR_INVALID_ARG, "fixed workspace too small for this graph");
  } else {
    VC_TRY(g->vm.ensure((size_t)n * 8));
    VC_TRY(g->bitmap.ensure((size_t)nwords * 4));
    VC_TRY(g->bitmap2.ensure((size_t)nwords * 4));
    VC_TRY(g->fq.ensure((size_t)n * 4));
    VC_TRY(g->prefix.ensure((size_t)(n + 1) * 8));
    VC_TRY(g->scan_blocks.ensure((size_t)vc::scan_scratch_entries(n) * 8));
    VC_TRY(g->list_tiles.ensure((size_t)((n + m) / tile + 3) * sizeof(int32_t)));
    VC_TRY(g->counters.ensure(sizeof(vc::Counters)));
    if (!g->host_ctr) VC_TRY(hipHostMalloc((void**)&g->host_ctr, sizeof(vc::Counters), hipHostMallocDefault));
    hc = g->host_ctr;
    wk.vm = g->vm.as<uint2>();
    wk.bits[0] = g->bitmap.as<uint32_t>();
    wk.bits[1] = g->bitmap2.as<uint32_t>();
    wk.fq = g->fq.as<int32_t>();
    wk.P = g->prefix.as<int64_t>();
    wk.scan = g->scan_blocks.as<int64_t>();
    wk.list_tiles = g->list_tiles.as<int32_t>();
    wk.ctr = g->counters.as<vc::Counters>();
  }
  uint2* vm = wk.vm;
  uint32_t* bits[2] = {wk.bits[0], wk.bits[1]};
  int32_t* fq = wk.fq;
  int64_t* P = wk.P;
  int32_t* list_tiles = wk.list_tiles;
  vc::Counters* ctr = wk.ctr;

  int64_t source = -1;
  if (kind != vc::kCC && !seed) {
    vc_status st = internal_id(g, (int64_t)p.source, s, &source);
    if (st != VC_OK) return st;
  }
  VC_TRY(vc::launch_fill_u32(bits[0], nwords, 0u, s));
  VC_TRY(vc::launch_fill_u32(bits[1], nwords, 0u, s));
  VC_TRY(vc::launch_zero_counters(ctr, s));
  if (rec.timed) VC_TRY(ensure_events(g, 4));

  // improvements of superstep s go to bits[cur]; bits[1 - cur] holds F_s
  int cur = 0;
  bool dense = kind == vc::kCC && !seed;  // superstep 0: every vertex (CC), the source (SSSP), or the seeded ones
  bool prefix_ready = false;
  int64_t frontier = 0, listed = 0, edges = 0;
  if (seed) {
    // the seeded senders become F_0: bitmap, broadcast list and counters as
    // if they had just improved
    VC_TRY(vc::launch_min_init_from(seed, n, vm, bits[1], s));
    VC_TRY(vc::launch_min_compact(g->off, g->off64, n, vm, bits[1], bits[0], fq, P, ctr, true, nullptr, s));
    VC_TRY(hipMemcpyAsync(hc, ctr, sizeof(vc::Counters), hipMemcpyDeviceToHost, s));
    VC_TRY(vc::launch_zero_counters(ctr, s));
    VC_TRY(hipStreamSynchronize(s));
    frontier = (int64_t)hc->active;
    listed = (int64_t)hc->listed;
    edges = (int64_t)hc->edges;
  } else if (dense) {
    VC_TRY(vc::launch_min_init(kind, n, source, g->relabeled ? g->inv_p : nullptr, vm, s));
    frontier = n;
    listed = n;
    edges = m;
  } else {
    VC_TRY(vc::launch_min_init(kind, n, source, g->relabeled ? g->inv_p : nullptr, vm, s));
    int64_t o[2] = {0, 0};
    if (g->off64) {
      VC_TRY(hipMemcpyAsync(o, (const int64_t*)g->off + source, 16, hipMemcpyDeviceToHost, s));
      VC_TRY(hipStreamSynchronize(s));
    } else {
      int32_t o32[2] = {0, 0};
      VC_TRY(hipMemcpyAsync(o32, (const int32_t*)g->off + source, 8, hipMemcpyDeviceToHost, s));
      VC_TRY(hipStreamSynchronize(s));
      o[0] = o32[0];
      o[1] = o32[1];
    }
    frontier = 1;
    edges = o[1] - o[0];
    listed = edges > 0 ? 1 : 0;
    VC_TRY(vc::launch_min_seed_source(g->off, g->off64, source, fq, P, bits[1], s));
    prefix_ready = true;
  }
  const int64_t cap = p.max_supersteps > 0 ? (int64_t)p.max_supersteps : n + 1;
  vc_status status = VC_OK;
  int64_t step = 0;
  const bool capture = (p.options & VC_OPT_GRAPH_CAPTURE) != 0;
  for (;;) {
    if (frontier == 0 || edges == 0) {
      rec.step(step, frontier, edges, 0);
      *supersteps = (int32_t)(step + 1);
      break;
    }
    if (capture && step >= 1) {
      // the rest runs on the device: form switch and termination decided there
      bool capped = false;
      vc_status st = run_min_device_loop(g, p, kind, tile, tba, hub, cur, step, frontier, listed, edges, cap, vm, bits,
                                         fq, P, wk.scan, list_tiles, ctr, s, rec, supersteps, &capped);
      if (st != VC_OK) return st;
      if (capped) status = fail(VC_ERR_NOT_CONVERGED, "superstep cap reached before quiescence");
      break;
    }
    int sched = p.schedule;
    if (sched == VC_SCHED_AUTO) {
      // a blocked superstep costs a full pass over the edges, so it takes
      // over from push later than the pull form would (scale-26 SSSP: push
      // 1.9 ms vs blocked 4.4 ms at 12 % of the edges, 6.5 vs 4.5 ms at 46 %)
      const bool blocked = min_blocked(g);
      const double thr = (p.pull_fraction > 0.0f || !blocked) ? pull_threshold(p) : kBlockedFraction;
      if ((double)edges >= thr * (double)m)
        sched = blocked ? VC_SCHED_BLOCKED : VC_SCHED_PULL;
      else
        sched = edges <= 256 ? VC_SCHED_VERTEX : VC_SCHED_EDGE;
    }
    if (arena && m > 0) {
      // only forms whose read-only structures the graph already holds (an
      // explicit PULL was checked before the run); the blocked form would
      // need message slots per edge
      if (sched == VC_SCHED_BLOCKED || sched == VC_SCHED_PULL)
        sched = vc::have_csc_partition(g, vc::pull_tile(tile)) ? VC_SCHED_PULL : VC_SCHED_EDGE;
      if (sched == VC_SCHED_EDGE && dense && !vc::have_dense_partition(g, tile)) sched = VC_SCHED_VERTEX;
    }
    rec.step(step, frontier, edges, sched);
    const bool timed = rec.want_time(step);
    if (timed) VC_TRY(hipEventRecord(g->events[0], s));
    uint32_t* improved = bits[cur];
    if (sched == VC_SCHED_BLOCKED) {
      vc_status st = use_pb(g, s);
      if (st != VC_OK) return st;
      const vc::PbShared& pb = g->pb;
      uint32_t* slot_msg = g->pb_vals.as<uint32_t>();
      if (timed) VC_TRY(hipEventRecord(g->events[1], s));
      // single-source SSSP: a value set at superstep t is a path of at most t
      // edges, so superstep `step` sends messages of at most (step + 1) *
      // wmax; below 0xFFFF they travel in 2-byte slots
      const bool narrow = kind != vc::kCC && !seed && (double)(step + 1) * (double)pb.wmax < 65535.0;
      VC_TRY(vc::launch_pb_spread_min(kind, pb.spread, pb.nspread, n, pb.shift, pb.srcl, pb.w, pb.wbytes, vm,
                                      dense ? nullptr : bits[1 - cur], slot_msg, narrow, nullptr, s));
      VC_TRY(vc::launch_pb_fold_min(pb.fold, pb.nfold, pb.run_off, pb.rpre, pb.btotal, pb.chunk_off, pb.chunks,
                                    pb.rbase, n, slot_msg, narrow, pb.dstl, vm, improved, nullptr, s));
    } else if (sched == VC_SCHED_PULL) {
      vc_status st = ensure_csc(g, s);
      if (st == VC_OK) st = csc_partition(g, vc::pull_tile(tile), s);
      if (st != VC_OK) return st;
      if (timed) VC_TRY(hipEventRecord(g->events[1], s));
      VC_TRY(vc::launch_min_pull(kind, g->csc_off_p, g->in_src, g->in_w, n, m, g->csc_tiles_p,
                                 g->csc_tile, g->csc_ntiles, vm, dense ? nullptr : bits[1 - cur], improved, nullptr,
                                 s));
    } else if (sched == VC_SCHED_EDGE) {
      if (dense) {
        vc_status st = dense_partition(g, tile, s);
        if (st != VC_OK) return st;
        if (timed) VC_TRY(hipEventRecord(g->events[1], s));
        VC_TRY(vc::launch_min_scatter_mp(kind, false, tba, g->off, g->off64, g->dst, g->w, n, n, n + m, nullptr,
                                         nullptr, g->dense_tiles_p, tile, g->dense_ntiles, vm, improved, hub, s));
      } else {
        if (!prefix_ready) VC_TRY(vc::launch_exclusive_scan(P, listed, wk.scan, s));
        const int64_t total = listed + edges;
        const int64_t ntiles = (total + tile - 1) / tile;
        VC_TRY(vc::launch_mp_partition(P, true, listed, total, tile, ntiles, list_tiles, s));
        if (timed) VC_TRY(hipEventRecord(g->events[1], s));
        VC_TRY(vc::launch_min_scatter_mp(kind, true, tba, g->off, g->off64, g->dst, g->w, n, listed, total, P, fq,
                                         list_tiles, tile, ntiles, vm, improved, hub, s));
      }
    } else {
      if (timed) VC_TRY(hipEventRecord(g->events[1], s));
      VC_TRY(vc::launch_min_scatter_vertex(kind, !dense, tba, g->off, g->off64, g->dst, g->w, n, dense ? n : listed,
                                           fq, vm, improved, hub, s));
    }
    if (timed) VC_TRY(hipEventRecord(g->events[2], s));
    VC_TRY(vc::launch_min_compact(g->off, g->off64, n, vm, improved, bits[1 - cur], fq, P, ctr, false, nullptr, s));
    if (timed) VC_TRY(hipEventRecord(g->events[3], s));
    VC_TRY(hipMemcpyAsync(hc, ctr, sizeof(vc::Counters), hipMemcpyDeviceToHost, s));
    VC_TRY(vc::launch_zero_counters(ctr, s));
    VC_TRY(hipStreamSynchronize(s));
    if (timed) {
      float a = 0, b = 0;
      VC_TRY(hipEventElapsedTime(&a, g->events[1], g->events[2]));
      VC_TRY(hipEventElapsedTime(&b, g->events[0], g->events[3]));
      rec.times(step, a, b);
    }
    frontier = (int64_t)hc->active;
    listed = (int64_t)hc->listed;
    edges = (int64_t)hc->edges;
    dense = false;
    prefix_ready = false;
    cur = 1 - cur;
    ++step;
    if (step >= cap) {
      *supersteps = (int32_t)step;
      status = fail(VC_ERR_NOT_CONVERGED, "superstep cap reached before quiescence");
      break;
    }
  }
  if (g->relabeled)
    VC_TRY(vc::launch_unpermute(reinterpret_cast<const uint32_t*>(vm), 2, g->perm_p, n, out, s));
  else
    VC_TRY(vc::launch_min_output(n, vm, out, s));
  VC_TRY(hipStreamSynchronize(s));
  return status;
}

// A run that leaves the distribution to the library (AUTO, tile 0, default
// pull threshold) takes the graph's autotuned setting for the program.
void apply_tuned(vc_graph g, vc_program prog, vc_params* p) {
  if (!g->tuned[prog] || p->schedule != VC_SCHED_AUTO || p->tile != 0 || p->pull_fraction != 0.0f) return;
  const vc_params& t = g->tuned_params[prog];
  p->schedule = t.schedule;
  p->tile = t.tile;
  p->pull_fraction = t.pull_fraction;
  p->options |= t.options & VC_OPT_GRAPH_CAPTURE;
}

}  // namespace

namespace vc {

bool valid_params(const vc_params& p, vc_program prog, int64_t n, std::string* why) {
  if (p.struct_size != sizeof(vc_params)) return *why = "vc_params.struct_size mismatch", false;
  if (p.schedule < VC_SCHED_AUTO || p.schedule > VC_SCHED_BLOCKED) return *why = "bad schedule", false;

  if (p.tile < 0) return *why = "negative tile", false;
  if (!(p.pull_fraction >= 0.0f)) return *why = "negative pull_fraction", false;
  if ((p.options & VC_OPT_F32_ACCUMULATE) && (p.options & VC_OPT_F32_MESSAGES))
    return *why = "VC_OPT_F32_ACCUMULATE and VC_OPT_F32_MESSAGES exclude each other", false;
  if (prog == VC_PAGERANK || prog == VC_PPR) {
    if (p.max_supersteps < 0) return *why = "PageRank needs T >= 0", false;
    if (!(p.damping >= 0.0 && p.damping <= 1.0)) return *why = "damping outside [0, 1]", false;
  } else if (p.max_supersteps < 0) {
    return *why = "negative superstep cap", false;
  }
  if ((prog == VC_SSSP || prog == VC_PPR) && (int64_t)p.source >= n) return *why = "source >= N", false;
  return true;
}


vc_status prepare_shared(vc_graph base, hipStream_t s) {
  if (!base || base->is_view) return fail(VC_ERR_INVALID_ARG, "not a graph handle");
  vc_params p;
  vc_params_default(&p);
  const int64_t tile = pick_tile(p, base);
  vc_status st = ensure_csc(base, s);
  if (st == VC_OK) st = csc_partition(base, pull_tile(tile), s);
  if (st == VC_OK) st = dense_partition(base, tile, s);
  if (st != VC_OK) return st;
  VC_TRY(hipStreamSynchronize(s));
  return VC_OK;
}

vc_status make_view(vc_graph base, hipStream_t s, vc_graph* out) {
  if (!base || !out) return fail(VC_ERR_INVALID_ARG, "null graph or out");
  if (base->is_view) return fail(VC_ERR_INVALID_ARG, "a view cannot serve as the base of another view");
  vc_status st = prepare_shared(base, s);
  if (st != VC_OK) return st;
  vc_graph v = new (std::nothrow) vc_graph_s();
  if (!v) return fail(VC_ERR_OUT_OF_MEMORY, "host allocation failed");
  v->n = base->n;
  v->m = base->m;
  v->off64 = base->off64;
  v->flags = base->flags | VC_GRAPH_BORROW;
  v->device = base->device;
  v->off = base->off;
  v->dst = base->dst;
  v->w = base->w;
  v->relabeled = base->relabeled;
  v->perm_p = base->perm_p;
  v->inv_p = base->inv_p;
  v->csc_off_p = base->csc_off_p;
  v->csc_tiles_p = base->csc_tiles_p;
  v->csc_tile = base->csc_tile;
  v->csc_ntiles = base->csc_ntiles;
  v->dense_tiles_p = base->dense_tiles_p;
  v->dense_tile = base->dense_tile;
  v->dense_ntiles = base->dense_ntiles;
  v->in_src = base->in_src;
  v->in_w = base->in_w;
  v->csc_ready = base->csc_ready;
  v->max_lds = base->max_lds;
  v->base = base;
  v->pb = base->pb;  // if built; else the view's first blocked run builds it on the base
  for (int i = 0; i < 4; ++i) {
    v->tuned[i] = base->tuned[i];
    v->tuned_params[i] = base->tuned_params[i];
  }
  v->is_view = true;
  *out = v;
  return VC_OK;
}

vc_status run_entry(vc_graph g, vc_program program, const vc_params* params, void* out, hipStream_t stream,
                    vc_stats* stats, const Arena* arena) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g) return fail(VC_ERR_INVALID_ARG, "null graph");
  if (!out) return fail(VC_ERR_INVALID_ARG, "null out");
  if ((uintptr_t)out % 4) return fail(VC_ERR_INVALID_ARG, "misaligned out");
  if (program < VC_PAGERANK || program > VC_PPR) return fail(VC_ERR_INVALID_ARG, "bad program");
  vc_params p;
  if (params) {
    p = *params;
  } else {
    vc_params_default(&p);
  }
  std::string why;
  if (!valid_params(p, program, g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  if (stats) {
    if (stats->struct_size != sizeof(vc_stats)) return fail(VC_ERR_INVALID_ARG, "vc_stats.struct_size mismatch");
    if (stats->capacity < 0) return fail(VC_ERR_INVALID_ARG, "negative stats capacity");
  }
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != g->device) return fail(VC_ERR_INVALID_ARG, "graph lives on another device than the current one");
  if (arena) {
    // everything that would allocate is refused here, before any device work
    if (p.options & VC_OPT_GRAPH_CAPTURE)
      return fail(VC_ERR_UNSUPPORTED, "a captured loop needs buffers of its own; drop VC_OPT_GRAPH_CAPTURE");
    if (p.schedule == VC_SCHED_BLOCKED)
      return fail(VC_ERR_UNSUPPORTED, "the blocked form needs 8 bytes of message slots per edge");
    if (p.schedule == VC_SCHED_PULL && g->m > 0 && !have_csc_partition(g, pull_tile(pick_tile(p, g))))
      return fail(VC_ERR_UNSUPPORTED, "the pull form needs the transpose and its partition: "
                                      "call vc_graph_prepare with the same params first");
    const size_t need = arena_need(g, program, p);
    if (need > arena->bytes)
      return fail(VC_ERR_INVALID_ARG, "the run needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                          std::to_string(arena->bytes) + " the fixed workspace holds");
  } else {
    apply_tuned(g, program, &p);
  }
  if (stats) {
    stats->supersteps = 0;
    stats->edges_relaxed = 0;
    stats->elapsed_ms = 0;
  }
  Recorder rec(stats);
  if (arena) rec.timed = false;  // events would have to be created
  int32_t supersteps = 0;
  vc_status st;
  if (program == VC_PAGERANK || program == VC_PPR)
    st = run_rank(g, p, program == VC_PPR, static_cast<float*>(out), stream, rec, &supersteps, arena);
  else
    st = run_min(g, p, program == VC_CC_HASHMIN ? kCC : (g->w ? kSsspWeighted : kSsspUnit), nullptr,
                 static_cast<uint32_t*>(out), stream, rec, &supersteps, arena);
  if (stats) {
    stats->supersteps = supersteps;
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // namespace vc

extern "C" {

int vc_abi_version(void) { return VC_ABI_VERSION; }

const char* vc_last_error(void) { return vc::t_last_error.c_str(); }

const char* vc_status_string(vc_status s) {
  switch (s) {
    case VC_OK: return "ok";
    case VC_ERR_INVALID_ARG: return "invalid argument";
    case VC_ERR_BAD_GRAPH: return "bad graph";
    case VC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case VC_ERR_HIP: return "HIP runtime error";
    case VC_ERR_UNSUPPORTED: return "unsupported";
    case VC_ERR_NOT_CONVERGED: return "superstep cap reached";
  }
  return "unknown status";
}

void vc_params_default(vc_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof(vc_params);
  p->max_supersteps = 10;
  p->damping = 0.85;
  p->source = 0;
  p->schedule = VC_SCHED_AUTO;
  p->tile = 0;
  p->options = 0;
  p->pull_fraction = 0.0f;
}

vc_status vc_graph_create(const vc_graph_desc* d, hipStream_t stream, vc_graph* out) {
  if (!d || !out) return fail(VC_ERR_INVALID_ARG, "null desc or out");
  if (d->struct_size != sizeof(vc_graph_desc)) return fail(VC_ERR_INVALID_ARG, "vc_graph_desc.struct_size mismatch");
  if (d->num_vertices < 1 || d->num_vertices > 2147483647LL)
    return fail(VC_ERR_INVALID_ARG, "num_vertices must be in [1, 2^31 - 1]");
  if (d->num_edges < 0) return fail(VC_ERR_INVALID_ARG, "negative num_edges");
  if (d->offset_type != VC_IDX_I32 && d->offset_type != VC_IDX_I64) return fail(VC_ERR_INVALID_ARG, "bad offset_type");
  if (d->offset_type == VC_IDX_I32 && d->num_edges >= 2147483648LL)
    return fail(VC_ERR_INVALID_ARG, "int32 offsets need num_edges < 2^31");
  if (!d->offsets || (d->num_edges > 0 && !d->dst)) return fail(VC_ERR_INVALID_ARG, "null offsets or dst");
  const size_t ow = d->offset_type == VC_IDX_I64 ? 8 : 4;
  if (((uintptr_t)d->offsets % ow) || ((uintptr_t)d->dst % 4) || ((uintptr_t)d->weights % 4))
    return fail(VC_ERR_INVALID_ARG, "misaligned array");

  vc_graph g = new (std::nothrow) vc_graph_s();
  if (!g) return fail(VC_ERR_OUT_OF_MEMORY, "host allocation failed");
  auto cleanup = [g](vc_status st) {
    vc_graph_destroy(g);
    return st;
  };
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipDeviceGetAttribute"));
  if (lds > 0) g->max_lds = (size_t)lds;
  g->n = d->num_vertices;
  g->m = d->num_edges;
  g->off64 = d->offset_type == VC_IDX_I64;
  g->flags = d->flags;
  if (d->flags & VC_GRAPH_BORROW) {
    g->off = d->offsets;
    g->dst = d->dst;
    g->w = d->weights;
  } else {
    const size_t ob = (size_t)(g->n + 1) * ow, eb = (size_t)g->m * 4;
    if ((e = g->own_off.ensure(ob)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc offsets"));
    if ((e = hipMemcpyAsync(g->own_off.p, d->offsets, ob, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
      return cleanup(hip_fail(e, "copy offsets"));
    g->off = g->own_off.p;
    if (eb) {
      if ((e = g->own_dst.ensure(eb)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc dst"));
      if ((e = hipMemcpyAsync(g->own_dst.p, d->dst, eb, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
        return cleanup(hip_fail(e, "copy dst"));
      g->dst = g->own_dst.as<int32_t>();
      if (d->weights) {
        if ((e = g->own_w.ensure(eb)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc weights"));
        if ((e = hipMemcpyAsync(g->own_w.p, d->weights, eb, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
          return cleanup(hip_fail(e, "copy weights"));
        g->w = g->own_w.as<uint32_t>();
      }
    }
  }
  if (d->flags & VC_GRAPH_VALIDATE) {
    if ((e = g->counters.ensure(sizeof(vc::Counters))) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
    vc::Counters h{};
    if ((e = vc::launch_zero_counters(g->counters.as<vc::Counters>(), stream)) != hipSuccess ||
        (e = vc::launch_validate(g->off, g->off64, g->dst, g->n, g->m, g->counters.as<vc::Counters>(), stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(&h, g->counters.p, sizeof h, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
      return cleanup(hip_fail(e, "validation"));
    if (h.flags) {
      std::string why;
      if (h.flags & 1) why += " offsets[0] != 0;";
      if (h.flags & 2) why += " offsets[N] != num_edges;";
      if (h.flags & 4) why += " offsets decrease;";
      if (h.flags & 8) why += " dst out of range;";
      return cleanup(fail(VC_ERR_BAD_GRAPH, "CSR validation failed:" + why));
    }
    if ((d->flags & VC_GRAPH_SYMMETRIC) && g->m > 0) {
      // the edge multiset against the reversed one, by multiset hashes
      unsigned long long acc[2] = {1, 1};
      auto* dacc = reinterpret_cast<unsigned long long*>(g->counters.p);
      if ((e = vc::launch_fill_u32(reinterpret_cast<uint32_t*>(dacc), 4, 0u, stream)) != hipSuccess ||
          (e = vc::launch_sym_hash(g->off, g->off64, g->dst, g->w, g->n, dacc, stream)) != hipSuccess ||
          (e = hipMemcpyAsync(acc, dacc, sizeof acc, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
          (e = hipStreamSynchronize(stream)) != hipSuccess)
        return cleanup(hip_fail(e, "symmetry validation"));
      if (acc[0] != 0 || acc[1] != 0)
        return cleanup(fail(VC_ERR_BAD_GRAPH,
                            "graph declared VC_GRAPH_SYMMETRIC differs from its transpose (edge multisets, weights "
                            "included, do not match)"));
    }
  }
  if (!(d->flags & VC_GRAPH_NO_RELABEL)) {
    vc_status st = relabel(g, stream);
    if (st != VC_OK) return cleanup(st);
  }
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return cleanup(hip_fail(e, "graph create"));
  *out = g;
  return VC_OK;
}

vc_status vc_graph_destroy(vc_graph g) {
  if (!g) return VC_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  for (DevBuf* b : {&g->own_off, &g->own_dst, &g->own_w, &g->perm, &g->inv, &g->rel_off, &g->rel_dst, &g->rel_w,
                    &g->contrib, &g->mb, &g->vm, &g->bitmap, &g->bitmap2,
                    &g->fq, &g->prefix, &g->scan_blocks, &g->list_tiles, &g->csc_off, &g->csc_src,
                    &g->csc_w, &g->ms_src, &g->counters, &g->pb_srcl, &g->pb_dstl, &g->pb_w, &g->pb_vals,
                    &g->pb_run_off, &g->pb_btotal, &g->pb_rpre, &g->pb_rbase, &g->pb_chunk_off, &g->pb_chunks,
                    &g->pb_spread, &g->pb_fold})
    b->release();
  g->ms.release();
  g->dense_parts.release();
  g->csc_parts.release();
  g->loop_state.release();
  g->loop_steps.release();
  if (g->host_ctr) (void)hipHostFree(g->host_ctr);
  if (g->host_loop) (void)hipHostFree(g->host_loop);
  for (auto& row : g->min_exec)
    for (hipGraphExec_t& e : row)
      if (e) (void)hipGraphExecDestroy(e);
  if (g->pr_exec) (void)hipGraphExecDestroy(g->pr_exec);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  for (hipEvent_t e : g->events) (void)hipEventDestroy(e);
  (void)hipSetDevice(prev);
  delete g;
  return VC_OK;
}

vc_status vc_graph_footprint(vc_graph g, vc_program program, size_t* bytes_held, size_t* bytes_run) {
  if (!g) return fail(VC_ERR_INVALID_ARG, "null graph");
  if (program < VC_PAGERANK || program > VC_PPR) return fail(VC_ERR_INVALID_ARG, "bad program");
  size_t held = g->own_off.bytes + g->own_dst.bytes + g->own_w.bytes + g->perm.bytes + g->inv.bytes +
                g->rel_off.bytes + g->rel_dst.bytes + g->rel_w.bytes;
  for (const DevBuf* b : {&g->contrib, &g->mb, &g->vm, &g->bitmap, &g->bitmap2, &g->fq, &g->prefix, &g->scan_blocks,
                          &g->list_tiles, &g->csc_off, &g->csc_src, &g->csc_w,
                          &g->ms_src, &g->counters, &g->pb_srcl, &g->pb_dstl, &g->pb_w, &g->pb_vals, &g->pb_run_off,
                          &g->pb_btotal, &g->pb_rpre, &g->pb_rbase, &g->pb_chunk_off, &g->pb_chunks,
                          &g->pb_spread, &g->pb_fold})
    held += b->bytes;
  held += g->ms.bytes();
  held += g->dense_parts.bytes() + g->csc_parts.bytes();
  if (bytes_held) *bytes_held = held;
  if (bytes_run) {
    // workspace of the program plus the transpose the pull form reads
    const size_t want = workspace_bytes(g->n, g->m, program, vc::kDefaultTile);
    size_t have = 0;
    if (program == VC_PAGERANK || program == VC_PPR)
      have = g->contrib.bytes + g->mb.bytes + g->dense_parts.bytes();
    else
      have = g->vm.bytes + g->bitmap.bytes + g->bitmap2.bytes + g->fq.bytes + g->prefix.bytes +
             g->scan_blocks.bytes + g->list_tiles.bytes + g->dense_parts.bytes() + g->counters.bytes;
    const size_t csc_want = (size_t)(g->n + 1) * 8 + (size_t)((g->n + g->m) / vc::kDefaultTile + 2) * 4 +
                            ((g->flags & VC_GRAPH_SYMMETRIC) ? 0 : (size_t)g->m * (g->w ? 8 : 4));
    const size_t csc_have = g->csc_off.bytes + g->csc_src.bytes + g->csc_w.bytes + g->csc_parts.bytes();
    size_t csc_need = g->csc_ready ? 0 : (csc_want > csc_have ? csc_want - csc_have : 0);
    // the blocked layout (shared with the base of a view) and this object's
    // message slots, where AUTO would take the blocked form; CC / SSSP keep
    // the transpose too (a captured loop pulls)
    size_t pb_need = 0;
    const vc_graph owner = g->is_view ? g->base : g;
    const size_t pb_more = (owner->pb.ready ? 0 : pb_layout_bytes(g) + pb_build_transient_bytes(g)) +
                           (g->pb_vals.bytes >= (size_t)g->m * 8 ? 0 : (size_t)g->m * 8 + 8);
    if (program == VC_PAGERANK || program == VC_PPR) {
      vc_params dp;
      vc_params_default(&dp);
      if (rank_schedule(g, dp, true) == VC_SCHED_BLOCKED) {
        csc_need = 0;  // the blocked schedule reads its own layout, not the transpose
        pb_need = pb_more;
      }
    } else if (min_blocked(g)) {
      pb_need = pb_more;
    }
    *bytes_run = (want > have ? want - have : 0) + csc_need + pb_need;
  }
  return VC_OK;
}

vc_status vc_run(vc_graph g, vc_program program, const vc_params* params, void* out, hipStream_t stream,
                 vc_stats* stats) {
  return vc::run_entry(g, program, params, out, stream, stats, nullptr);
}

vc_status vc_graph_prepare(vc_graph g, vc_program program, const vc_params* params, hipStream_t stream) {
  if (!g) return fail(VC_ERR_INVALID_ARG, "null graph");
  if (program < VC_PAGERANK || program > VC_PPR) return fail(VC_ERR_INVALID_ARG, "bad program");
  vc_params p;
  if (params)
    p = *params;
  else
    vc_params_default(&p);
  std::string why;
  if (!valid_params(p, program, g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  apply_tuned(g, program, &p);
  int cur = 0;
  VC_TRY(hipGetDevice(&cur));
  if (cur != g->device) return fail(VC_ERR_INVALID_ARG, "graph lives on another device than the current one");
  if (g->m == 0) return VC_OK;
  const int64_t tile = pick_tile(p, g);
  const bool capture = (p.options & VC_OPT_GRAPH_CAPTURE) != 0;
  auto pull = [&]() {
    vc_status st = ensure_csc(g, stream);
    return st == VC_OK ? csc_partition(g, vc::pull_tile(tile), stream) : st;
  };
  vc_status st = VC_OK;
  if (program == VC_PAGERANK || program == VC_PPR) {
    const bool fx = !(p.options & VC_OPT_F32_ACCUMULATE);
    const int sched = rank_schedule(g, p, fx);
    if (sched == VC_SCHED_BLOCKED && !fx)
      return fail(VC_ERR_UNSUPPORTED, "the blocked schedule sums in fixed point; drop VC_OPT_F32_ACCUMULATE");
    if (sched == VC_SCHED_PULL) st = pull();
    else if (sched == VC_SCHED_EDGE) st = dense_partition(g, tile, stream);
    else if (sched == VC_SCHED_BLOCKED) st = use_pb(g, stream);
  } else {
    switch (p.schedule) {
      case VC_SCHED_BLOCKED: st = use_pb(g, stream); break;
      case VC_SCHED_PULL: st = pull(); break;
      case VC_SCHED_EDGE: st = dense_partition(g, tile, stream); break;
      case VC_SCHED_VERTEX: break;
      default:  // AUTO: the dense form its dense supersteps take, the partition of a dense push
        st = min_blocked(g) ? use_pb(g, stream) : pull();
        if (st == VC_OK) st = dense_partition(g, tile, stream);
    }
    (void)capture;  // a captured loop takes the same forms
  }
  if (st != VC_OK) return st;
  VC_TRY(hipStreamSynchronize(stream));
  return VC_OK;
}

vc_status vc_combine(vc_graph g, vc_combiner op, const uint64_t* msg, const uint8_t* active, uint64_t* mailbox,
                     uint32_t* has, hipStream_t stream) {
  if (!g || !msg || !mailbox || !has) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (op < VC_COMBINE_SUM_U64 || op > VC_COMBINE_SUM_F64) return fail(VC_ERR_INVALID_ARG, "bad combiner");
  if ((uintptr_t)msg % 8 || (uintptr_t)mailbox % 8 || (uintptr_t)has % 4)
    return fail(VC_ERR_INVALID_ARG, "misaligned array");
  int cur = 0;
  VC_TRY(hipGetDevice(&cur));
  if (cur != g->device) return fail(VC_ERR_INVALID_ARG, "graph lives on another device than the current one");
  const int64_t n = g->n, m = g->m;
  const int32_t* inv = g->relabeled ? g->inv_p : nullptr;
  const auto* words = reinterpret_cast<const unsigned long long*>(msg);
  auto* box = reinterpret_cast<unsigned long long*>(mailbox);
  VC_TRY(vc::launch_fill_u32(has, n, 0u, stream));
  VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(mailbox), 2 * n, 0u, stream));
  if (m == 0) {
    VC_TRY(hipStreamSynchronize(stream));
    return VC_OK;
  }
  vc_params p;
  vc_params_default(&p);
  // Direction: push (contention only at the few receivers of a sparse set of
  // senders) when the senders' out-edges are under the pull threshold, else
  // pull (receivers fold their in-edges; no contention).
  bool pull = true;
  if (active) {
    VC_TRY(g->counters.ensure(sizeof(vc::Counters)));
    if (!g->host_ctr) VC_TRY(hipHostMalloc((void**)&g->host_ctr, sizeof(vc::Counters), hipHostMallocDefault));
    VC_TRY(vc::launch_zero_counters(g->counters.as<vc::Counters>(), stream));
    VC_TRY(vc::launch_active_edges(g->off, g->off64, n, inv, active, g->counters.as<vc::Counters>(), stream));
    VC_TRY(hipMemcpyAsync(g->host_ctr, g->counters.p, sizeof(vc::Counters), hipMemcpyDeviceToHost, stream));
    VC_TRY(hipStreamSynchronize(stream));
    pull = (double)g->host_ctr->edges >= pull_threshold(p) * (double)m;
    if (g->host_ctr->edges == 0) return VC_OK;
  }
  if (pull) {
    int64_t tile = vc::pull_tile(pick_tile(p, g));
    while (tile > 256 && vc::combine_pull_lds_bytes(tile) > g->max_lds) tile /= 2;
    vc_status st = ensure_csc(g, stream);
    if (st == VC_OK) st = csc_partition(g, tile, stream);
    if (st != VC_OK) return st;
    VC_TRY(vc::launch_combine_pull((int)op, g->csc_off_p, g->in_src, n, m, g->csc_tiles_p, g->csc_tile,
                                   g->csc_ntiles, inv, words, active, box, has, stream));
  } else {
    int64_t tile = pick_tile(p, g);
    while (tile > 64 && vc::combine_lds_bytes(tile) > g->max_lds) tile -= 64;
    vc_status st = dense_partition(g, tile, stream);
    if (st != VC_OK) return st;
    VC_TRY(vc::launch_combine((int)op, g->off, g->off64, g->dst, n, m, g->dense_tiles_p, tile, g->dense_ntiles, inv,
                              words, active, box, has, stream));
  }
  VC_TRY(hipStreamSynchronize(stream));
  return VC_OK;
}

// ---------------------------------------------------------------- batches

struct vc_batch_s {
  vc_graph g = nullptr;             // the disjoint union of the members
  std::vector<int64_t> vbase;       // member i owns union vertices [vbase[i], vbase[i+1])
  DevBuf u_off, u_dst, u_w;         // union CSR in member order (kept only without relabelling)
  DevBuf init;                      // initial values, internal order
};

vc_status vc_batch_create(const vc_graph_desc* members, const vc_batch_query* queries, int32_t count, uint32_t flags,
                          hipStream_t stream, vc_batch* out) {
  if (!members || !queries || !out || count < 1) return fail(VC_ERR_INVALID_ARG, "null argument or count < 1");
  int64_t n = 0, m = 0;
  for (int32_t i = 0; i < count; ++i) {
    const vc_graph_desc& d = members[i];
    const vc_batch_query& q = queries[i];
    if (d.struct_size != sizeof(vc_graph_desc) || q.struct_size != sizeof(vc_batch_query))
      return fail(VC_ERR_INVALID_ARG, "struct_size mismatch in member " + std::to_string(i));
    if (d.num_vertices < 1 || d.num_edges < 0 || !d.offsets || (d.num_edges > 0 && !d.dst))
      return fail(VC_ERR_INVALID_ARG, "bad member graph " + std::to_string(i));
    if (d.offset_type != VC_IDX_I32 && d.offset_type != VC_IDX_I64)
      return fail(VC_ERR_INVALID_ARG, "bad offset_type in member " + std::to_string(i));
    if (q.program != VC_CC_HASHMIN && q.program != VC_SSSP)
      return fail(VC_ERR_UNSUPPORTED, "batched members run VC_CC_HASHMIN or VC_SSSP");
    if (q.program == VC_SSSP && (int64_t)q.source >= d.num_vertices)
      return fail(VC_ERR_INVALID_ARG, "source >= N in member " + std::to_string(i));
    n += d.num_vertices;
    m += d.num_edges;
  }
  if (n > 2147483647LL) return fail(VC_ERR_INVALID_ARG, "the union exceeds 2^31 - 1 vertices");
  vc_batch b = new (std::nothrow) vc_batch_s();
  if (!b) return fail(VC_ERR_OUT_OF_MEMORY, "host allocation failed");
  auto cleanup = [b](vc_status st) {
    vc_batch_destroy(b);
    return st;
  };
  hipError_t e;
  if ((e = b->u_off.ensure((size_t)(n + 1) * 8)) != hipSuccess || (e = b->u_dst.ensure((size_t)m * 4 + 4)) != hipSuccess ||
      (e = b->u_w.ensure((size_t)m * 4 + 4)) != hipSuccess || (e = b->init.ensure((size_t)n * 4)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc union"));
  b->vbase.assign((size_t)count + 1, 0);
  int64_t vb = 0, eb = 0;
  for (int32_t i = 0; i < count; ++i) {
    const vc_graph_desc& d = members[i];
    const vc_batch_query& q = queries[i];
    b->vbase[i] = vb;
    const int wmode = q.program == VC_CC_HASHMIN ? 0 : (d.weights ? 1 : 2);
    if ((e = vc::launch_union_member(d.offsets, d.offset_type == VC_IDX_I64, d.dst, d.weights, d.num_vertices,
                                     d.num_edges, vb, eb, wmode, b->u_off.as<int64_t>(), b->u_dst.as<int32_t>(),
                                     b->u_w.as<uint32_t>(), stream)) != hipSuccess ||
        (e = vc::launch_union_init(d.num_vertices, vb, q.program == VC_CC_HASHMIN ? 0 : 1, (int64_t)q.source,
                                   b->init.as<uint32_t>(), stream)) != hipSuccess)
      return cleanup(hip_fail(e, "union member"));
    vb += d.num_vertices;
    eb += d.num_edges;
  }
  b->vbase[count] = vb;
  if ((e = hipMemcpyAsync(b->u_off.as<int64_t>() + n, &m, 8, hipMemcpyHostToDevice, stream)) != hipSuccess ||
      (e = hipStreamSynchronize(stream)) != hipSuccess)
    return cleanup(hip_fail(e, "union offsets"));
  vc_graph_desc ud;
  std::memset(&ud, 0, sizeof ud);
  ud.struct_size = sizeof ud;
  ud.flags = VC_GRAPH_BORROW | (flags & (VC_GRAPH_VALIDATE | VC_GRAPH_NO_RELABEL));
  ud.num_vertices = n;
  ud.num_edges = m;
  ud.offset_type = VC_IDX_I64;
  ud.offsets = b->u_off.p;
  ud.dst = b->u_dst.as<int32_t>();
  ud.weights = b->u_w.as<uint32_t>();
  vc_status st = vc_graph_create(&ud, stream, &b->g);
  if (st != VC_OK) return cleanup(st);
  if (b->g->relabeled) {
    DevBuf tmp;
    if ((e = tmp.ensure((size_t)n * 4)) != hipSuccess ||
        (e = vc::launch_permute(b->init.as<uint32_t>(), b->g->perm_p, n, tmp.as<uint32_t>(), stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
      return cleanup(hip_fail(e, "permute initial values"));
    std::swap(b->init.p, tmp.p);
    std::swap(b->init.bytes, tmp.bytes);
    b->u_off.release();
    b->u_dst.release();
    b->u_w.release();
  }
  *out = b;
  return VC_OK;
}

vc_status vc_batch_layout(vc_batch b, int64_t* vertex_base) {
  if (!b || !vertex_base) return fail(VC_ERR_INVALID_ARG, "null argument");
  std::memcpy(vertex_base, b->vbase.data(), b->vbase.size() * sizeof(int64_t));
  return VC_OK;
}

vc_status vc_batch_run(vc_batch b, const vc_params* params, uint32_t* out, hipStream_t stream, vc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!b) return fail(VC_ERR_INVALID_ARG, "null batch");
  if (!out || ((uintptr_t)out % 4)) return fail(VC_ERR_INVALID_ARG, "null or misaligned out");
  vc_params p;
  if (params)
    p = *params;
  else
    vc_params_default(&p);
  p.source = 0;
  std::string why;
  if (!valid_params(p, VC_SSSP, b->g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  apply_tuned(b->g, VC_SSSP, &p);
  if (stats) {
    if (stats->struct_size != sizeof(vc_stats) || stats->capacity < 0)
      return fail(VC_ERR_INVALID_ARG, "bad vc_stats");
    stats->supersteps = 0;
    stats->edges_relaxed = 0;
  }
  Recorder rec(stats);
  int32_t supersteps = 0;
  vc_status st = run_min(b->g, p, vc::kSsspWeighted, b->init.as<uint32_t>(), out, stream, rec, &supersteps);
  if (stats) {
    stats->supersteps = supersteps;
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

vc_status vc_batch_destroy(vc_batch b) {
  if (!b) return VC_OK;
  vc_graph_destroy(b->g);
  b->u_off.release();
  b->u_dst.release();
  b->u_w.release();
  b->init.release();
  delete b;
  return VC_OK;
}

vc_status vc_run_multi_source(vc_graph g, const uint32_t* sources, int32_t k, const vc_params* params, uint32_t* out,
                              hipStream_t s, vc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g || !sources || !out) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (k < 1 || k > 256) return fail(VC_ERR_INVALID_ARG, "need 1 <= k <= 256 sources");
  if ((uintptr_t)out % 4) return fail(VC_ERR_INVALID_ARG, "misaligned out");
  for (int32_t i = 0; i < k; ++i)
    if ((int64_t)sources[i] >= g->n) return fail(VC_ERR_INVALID_ARG, "source >= N");
  vc_params p;
  if (params)
    p = *params;
  else
    vc_params_default(&p);
  p.source = 0;
  std::string why;
  if (!valid_params(p, VC_SSSP, g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  if (p.schedule == VC_SCHED_BLOCKED)
    return fail(VC_ERR_UNSUPPORTED, "many-source runs choose push or pull per superstep; the blocked form is not one");
  if (stats) {
    if (stats->struct_size != sizeof(vc_stats) || stats->capacity < 0) return fail(VC_ERR_INVALID_ARG, "bad vc_stats");
    stats->supersteps = 0;
    stats->edges_relaxed = 0;
  }
  Recorder rec(stats);
  const int64_t n = g->n;
  const int C = vc::ms_chunks(k);
  const int64_t nwords = (n + 31) / 32;
  VC_TRY(g->ms_src.ensure((size_t)k * 4));
  // the pull reads a 2-byte copy of the distances while they cannot reach
  // 0xFFFF: after superstep s they are at most s times the largest weight
  uint32_t wmax = 1;
  {
    vc_status st = ensure_csc(g, s);
    if (st == VC_OK) st = weight_max(g, s, &wmax);
    if (st == VC_OK) st = vc::ms_reset(g->ms, g, C, s, wmax < 0xFFFFu);
    if (st != VC_OK) return st;
  }
  vc::MsState& ms = g->ms;
  vc::Counters* ctr = ms.ctr.as<vc::Counters>();
  VC_TRY(vc::launch_zero_counters(ctr, s));
  VC_TRY(hipMemcpyAsync(g->ms_src.p, sources, (size_t)k * 4, hipMemcpyHostToDevice, s));
  VC_TRY(vc::launch_ms_seed(g->ms_src.as<int32_t>(), g->relabeled ? g->perm_p : nullptr, k, n, ms.D.as<uint32_t>(),
                            ms.shadow ? ms.D16.as<uint16_t>() : nullptr, ms.A[0].as<unsigned long long>(),
                            ms.bits.as<uint32_t>(), s));
  VC_TRY(vc::launch_ms_count(g->off, g->off64, n, ms.bits.as<uint32_t>(), ctr, s));
  VC_TRY(vc::launch_fill_u32(ms.bits.as<uint32_t>(), nwords, 0u, s));
  VC_TRY(hipMemcpyAsync(ms.host, ctr, sizeof(vc::Counters), hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  if (rec.timed) VC_TRY(ensure_events(g, 4));
  int64_t frontier = (int64_t)ms.host[0].active, edges = (int64_t)ms.host[0].edges;
  const int64_t cap = p.max_supersteps > 0 ? (int64_t)p.max_supersteps : n + 1;
  vc_status status = VC_OK;
  int cur = 0;
  int64_t step = 0;
  int32_t supersteps = 0;
  for (;;) {
    if (frontier == 0 || edges == 0) {
      rec.step(step, frontier, edges, 0);
      supersteps = (int32_t)(step + 1);
      break;
    }
    if (ms.shadow && (double)(step + 1) * (double)wmax >= 65535.0) ms.shadow = false;
    const bool timed = rec.want_time(step);
    if (timed) VC_TRY(hipEventRecord(g->events[0], s));
    bool pushed = false;
    vc_status st = vc::ms_superstep(ms, g, cur, C, edges, false, vc::LaneMask{}, nullptr, &pushed, s);
    if (st != VC_OK) return st;
    if (timed) VC_TRY(hipEventRecord(g->events[2], s));
    VC_TRY(hipStreamSynchronize(s));
    rec.step(step, frontier, edges, pushed ? VC_SCHED_EDGE : VC_SCHED_PULL);
    if (timed) {
      float b = 0;
      VC_TRY(hipEventElapsedTime(&b, g->events[0], g->events[2]));
      rec.times(step, b, b);
    }
    frontier = (int64_t)ms.host[0].active;
    edges = (int64_t)ms.host[0].edges;
    cur = 1 - cur;
    ++step;
    if (step >= cap) {
      supersteps = (int32_t)step;
      status = fail(VC_ERR_NOT_CONVERGED, "superstep cap reached before quiescence");
      break;
    }
  }
  VC_TRY(vc::launch_ms_output(ms.D.as<uint32_t>(), g->relabeled ? g->perm_p : nullptr, n, k, out, s));
  VC_TRY(hipStreamSynchronize(s));
  if (stats) {
    stats->supersteps = supersteps;
    stats->elapsed_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return status;
}

}  // extern "C"

namespace {

// Candidate distributions for a program: PageRank / PPR vary schedule, tile
// and capture; CC / SSSP vary the pull threshold, tile and capture.
std::vector<vc_params> tune_candidates(vc_program program, const vc_params& base, bool blocked_ok) {
  std::vector<vc_params> out;
  const int32_t tiles[] = {1024, 2048, 4096};
  for (uint32_t capture : {0u, (uint32_t)VC_OPT_GRAPH_CAPTURE})
    for (int32_t tile : tiles) {
      if (program == VC_PAGERANK || program == VC_PPR) {
        for (vc_schedule sc : {VC_SCHED_PULL, VC_SCHED_EDGE, VC_SCHED_BLOCKED}) {
          // the blocked form has no tile, and sums in fixed point only
          if (sc == VC_SCHED_BLOCKED && (!blocked_ok || tile != tiles[0] || (base.options & VC_OPT_F32_ACCUMULATE)))
            continue;
          vc_params p = base;
          p.schedule = sc;
          p.tile = tile;
          p.options = (base.options & ~(uint32_t)VC_OPT_GRAPH_CAPTURE) | capture;
          out.push_back(p);
        }
      } else {
        for (float frac : {0.0f, 0.03f, 0.1f, 0.3f, 2.0f}) {  // 0: the library default
          vc_params p = base;
          p.schedule = VC_SCHED_AUTO;
          p.tile = tile;
          p.pull_fraction = frac;
          p.options = (base.options & ~(uint32_t)VC_OPT_GRAPH_CAPTURE) | capture;
          out.push_back(p);
        }
      }
    }
  return out;
}

template <class Run>
vc_status pick_fastest(const std::vector<vc_params>& cands, Run run, vc_params* best) {
  double best_ms = 1e300;
  for (const vc_params& c : cands) {
    vc_status st = run(c);  // warm-up: workspace, transpose, captured graph
    if (st != VC_OK) return st;
    const auto t0 = std::chrono::steady_clock::now();
    st = run(c);
    if (st != VC_OK) return st;
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (ms < best_ms) {
      best_ms = ms;
      *best = c;
    }
  }
  return VC_OK;
}

}  // namespace

extern "C" {

vc_status vc_graph_autotune(vc_graph g, vc_program program, const vc_params* base, hipStream_t stream,
                            vc_params* best) {
  if (!g || !best) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (program < VC_PAGERANK || program > VC_PPR) return fail(VC_ERR_INVALID_ARG, "bad program");
  vc_params b;
  if (base)
    b = *base;
  else
    vc_params_default(&b);
  std::string why;
  if (!valid_params(b, program, g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  DevBuf out;
  VC_TRY(out.ensure((size_t)g->n * 4));
  vc_params pick = b;
  vc_status st = pick_fastest(tune_candidates(program, b, g->m > 0 && pb_supported(g)),
                              [&](const vc_params& c) { return vc_run(g, program, &c, out.p, stream, nullptr); }, &pick);
  if (st != VC_OK) return st;
  g->tuned[program] = true;
  g->tuned_params[program] = pick;
  *best = pick;
  return VC_OK;
}

vc_status vc_batch_autotune(vc_batch b, const vc_params* base, hipStream_t stream, vc_params* best) {
  if (!b || !best) return fail(VC_ERR_INVALID_ARG, "null argument");
  vc_params p;
  if (base)
    p = *base;
  else
    vc_params_default(&p);
  p.source = 0;
  std::string why;
  if (!valid_params(p, VC_SSSP, b->g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  DevBuf out;
  VC_TRY(out.ensure((size_t)b->g->n * 4));
  vc_params pick = p;
  vc_status st = pick_fastest(
      tune_candidates(VC_SSSP, p, false),
      [&](const vc_params& c) { return vc_batch_run(b, &c, out.as<uint32_t>(), stream, nullptr); }, &pick);
  if (st != VC_OK) return st;
  b->g->tuned[VC_SSSP] = true;
  b->g->tuned_params[VC_SSSP] = pick;
  *best = pick;
  return VC_OK;
}

}  // extern "C"

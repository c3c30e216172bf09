// Host-side internals of libvc shared by the API and server translation
// units: device buffers, the graph object, error reporting and the graph
// preparation steps.  Not part of the public ABI (include/vc.h is).
#pragma once

#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "vc_internal.h"

namespace vc {

// Records `msg` as this thread's last error (vc_last_error) and returns st.
vc_status fail(vc_status st, const std::string& msg);
vc_status hip_fail(hipError_t e, const char* what);

#define VC_TRY(call)                                      \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::vc::hip_fail(e_, #call); \
  } while (0)

// A device buffer, grown on demand and kept across runs; freed when its
// owner goes away (graph, batch, or a temporary of a build step).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  hipError_t ensure(size_t want) {
    if (want <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      bytes = 0;
    }
    if (want == 0) return hipSuccess;
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) bytes = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};


// Merge-path partitions by tile size.  Entries live until the owning graph
// is destroyed, so views may keep pointers into them.
struct PartCache {
  std::vector<std::pair<int64_t, std::unique_ptr<DevBuf>>> parts;
  DevBuf* find(int64_t tile) const {
    for (const auto& e : parts)
      if (e.first == tile) return e.second.get();
    return nullptr;
  }
  DevBuf* add(int64_t tile) {
    parts.emplace_back(tile, std::unique_ptr<DevBuf>(new DevBuf()));
    return parts.back().second.get();
  }
  size_t bytes() const {
    size_t b = 0;
    for (const auto& e : parts) b += e.second->bytes;
    return b;
  }
  void release() { parts.clear(); }
};

// Device state of a many-lane min-plus superstep loop (many-source SSSP,
// request-server lane tables): lanes form cs chunks of 64, and every array
// is chunk-major (chunk c of vertex v at c * n + v; a value row is 64
// lanes), so a loop whose busy lanes sit in the first ceff chunks touches
// only a prefix of each array.
struct MsState {
  int64_t n = 0, m = 0;
  int cs = 0;
  DevBuf D, MB, A[2], bits, list, P, scan_blocks, push_tiles, ctr;
  DevBuf D16;                        // 2-byte copy of D read by the pull (while `shadow`)
  bool shadow = false;
  DevBuf pull_tiles[4];              // pull partitions for 1..4 chunks
  int64_t pull_ntiles[4] = {0, 0, 0, 0};
  int dirty[2] = {0, 0};             // chunks of A[b] that may hold set bits
  Counters* host = nullptr;          // pinned: [0] apply counters, [1] broadcast-list counters
  MsState() = default;
  MsState(const MsState&) = delete;
  MsState& operator=(const MsState&) = delete;
  ~MsState() { release(); }
  void release();
  size_t bytes() const;
};

// Lane-step tiles: a pull tile of 512 items per chunk keeps the LDS of one
// wavefront at 4 KiB; push tiles are small so a sparse frontier still
// spreads over many wavefronts.
constexpr int64_t kMsPullTilePerChunk = 512;
constexpr int64_t kMsPushTile = 256;
// A superstep is pushed from a broadcast list while its active vertices'
// out-edges stay below this fraction of all edges, else pulled.
constexpr double kMsPullFraction = 0.05;

// Allocates st for (g, cs) and resets every lane to unreached with no
// active vertex.  Needs g's transpose.  shadow: also keep a 2-byte copy of
// the values (0xFFFF: unreached) for the pull to read; valid while every
// distance stays below 0xFFFF, and the caller clears st.shadow before the
// first superstep where one might not.
vc_status ms_reset(MsState& st, vc_graph g, int cs, hipStream_t s, bool shadow = false);
// One superstep over the first ceff chunks (seeds already in A[cur]): push
// from a compacted broadcast list when force_pull is false and the active
// vertices' out-edges (next_edges estimates them; counted exactly before a
// push) stay below kMsPullFraction * m, else pull; then apply into
// A[1 - cur].  The apply counters are copied to st.host[0] on s; the caller
// synchronises s before reading them.
vc_status ms_superstep(MsState& st, vc_graph g, int cur, int ceff, int64_t next_edges, bool force_pull,
                       const LaneMask& zero, unsigned long long* live, bool* pushed, hipStream_t s);

// Read-only part of the blocked PageRank layout (see vc_blocked.hip); a
// view copies its base's once the base has built it.
struct PbShared {
  const uint16_t* srcl = nullptr;
  const uint16_t* dstl = nullptr;
  const void* w = nullptr;  // edge weights in slot order (weighted graphs), wbytes each
  int wbytes = 4;
  uint32_t wmax = 1;        // largest edge weight (1 when unweighted)
  const int64_t* run_off = nullptr;
  const int64_t* btotal = nullptr;
  const int64_t* rpre = nullptr;
  const int64_t* rbase = nullptr;
  const int64_t* chunk_off = nullptr;
  const PbChunk* chunks = nullptr;
  const PbSpreadItem* spread = nullptr;
  const PbFoldItem* fold = nullptr;
  const uint8_t* kinds = nullptr;  // PbBinKind of every destination bin
  int64_t nspread = 0, nfold = 0, tiles = 0;
  int shift = 0;
  bool ready = false;
};

}  // namespace vc

struct vc_graph_s {
  int64_t n = 0, m = 0;
  bool off64 = false;
  uint32_t flags = 0;
  int device = 0;
  const void* off = nullptr;
  const int32_t* dst = nullptr;
  const uint32_t* w = nullptr;
  vc::DevBuf own_off, own_dst, own_w;  // copies when not borrowed
  // relabelled copy (hot-first vertex order); perm[old] = new, inv[new] = old
  bool relabeled = false;
  vc::DevBuf perm, inv, rel_off, rel_dst, rel_w;
  // read-only arrays shared with views (see make_view): plain pointers to
  // buffers owned by the base graph, or by this object for its own partitions
  const int32_t* perm_p = nullptr;
  const int32_t* inv_p = nullptr;
  const int64_t* csc_off_p = nullptr;
  const int32_t* csc_tiles_p = nullptr;
  const int32_t* dense_tiles_p = nullptr;
  bool is_view = false;
  // workspace
  vc::DevBuf contrib, mb;                             // PageRank / PPR
  vc::DevBuf vm, bitmap, bitmap2, fq, prefix, scan_blocks;  // CC / SSSP (two bitmaps: improved / active)
  vc::DevBuf list_tiles;                              // per-superstep merge-path partition
  vc::PartCache dense_parts;                      // merge-path partitions of the CSR itself
  int64_t dense_tile = 0, dense_ntiles = 0;
  // transpose (CSC) for the pull form; for symmetric graphs only csc_off is
  // owned (int64 copy of the offsets) and csc_src / csc_w alias the CSR
  vc::DevBuf csc_off, csc_src, csc_w;
  vc::PartCache csc_parts;
  const int32_t* in_src = nullptr;
  const uint32_t* in_w = nullptr;
  bool csc_ready = false;
  int64_t csc_tile = 0, csc_ntiles = 0;
  vc::MsState ms;                                 // many-source SSSP
  // propagation-blocking layout (PageRank / PPR, built on first use): the
  // read-only part in buffers owned by the base graph, referenced by `pb`
  // in the base and in its views; each object owns its message slots
  vc::DevBuf pb_srcl, pb_dstl, pb_w, pb_run_off, pb_btotal, pb_rpre, pb_rbase, pb_chunk_off, pb_chunks, pb_spread,
      pb_fold, pb_kinds;
  vc::PbShared pb;
  vc::DevBuf pb_vals;
  uint32_t wmax = 0;        // largest edge weight once computed (0: not yet)
  std::mutex pb_mu;         // base: serialises the layout build between views
  vc_graph base = nullptr;  // views: the graph they share arrays with
  vc::DevBuf ms_src;
  // captured superstep loops (HIP graphs), replayed on the caller's stream
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t min_exec[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};
  std::string min_exec_key[3][2];  // device addresses and tile each captured loop was recorded with
  hipGraphExec_t pr_exec = nullptr;
  std::string pr_exec_key;
  vc::DevBuf loop_state, loop_steps;
  vc::LoopState* host_loop = nullptr;  // pinned
  // autotuned settings per program (used by VC_SCHED_AUTO runs with tile 0)
  bool tuned[4] = {false, false, false, false};
  vc_params tuned_params[4];
  vc::DevBuf counters;
  size_t max_lds = 65536;            // dynamic LDS limit per workgroup on the graph's device
  vc::Counters* host_ctr = nullptr;  // pinned
  std::vector<hipEvent_t> events;
};

namespace vc {

// A fixed device region that holds a run's workspace in place of the graph's
// own buffers, so that the run allocates nothing (vc_run_noalloc).  Pieces are
// carved from it at 256-byte boundaries, in a fixed order per program.
struct Arena {
  unsigned char* base = nullptr;
  size_t bytes = 0;
};

// Bytes of fixed workspace a run of `program` on g needs (merge-path tile as
// the run would pick it from p).
size_t arena_need(vc_graph g, vc_program program, const vc_params& p);

// The body of vc_run.  With arena != nullptr the run allocates nothing: its
// workspace comes from the arena, it reads only the read-only structures the
// graph already holds (a form whose structure is missing is replaced by one
// that needs none, or refused), per-superstep timings are not recorded, and
// the graph's autotuned setting is not applied.
vc_status run_entry(vc_graph g, vc_program program, const vc_params* params, void* out, hipStream_t stream,
                    vc_stats* stats, const Arena* arena);

// Transpose (CSC) of the graph, built once; in_src / in_w / csc_off_p set.
vc_status ensure_csc(vc_graph g, hipStream_t s);
// Merge-path partition of the transpose for pull tiles of `tile` items.
vc_status csc_partition(vc_graph g, int64_t tile, hipStream_t s);
// Requested merge-path tile clamped to what the device's LDS can stage.
int64_t pick_tile(const vc_params& p, vc_graph g);
// Checks params for a run of prog on a graph of n vertices; *why on failure.
bool valid_params(const vc_params& p, vc_program prog, int64_t n, std::string* why);
// Builds base's transpose and default partitions (on s, synchronised), the
// read-only arrays views share.
vc_status prepare_shared(vc_graph base, hipStream_t s);
// A graph object that shares every read-only array of `base` (structure,
// relabelling, transpose, partitions) and owns only its own workspace,
// events and streams.  The base must outlive the view.  The base's transpose
// and default partitions are built first (on stream s) so views never build
// their own.
vc_status make_view(vc_graph base, hipStream_t s, vc_graph* out);

}  // namespace vc

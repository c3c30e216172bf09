// Request server: many independent program runs (paper, Section I) arriving
// over time on resident graphs.
//
// Min programs on a graph with a lane table are served by continuous
// batching: one thread per table runs the table's superstep loop, every
// occupied lane side by side (the many-source pull of the min combiner,
// paper, Sections III and VI-C).  Between supersteps it retires lanes whose
// program has quiesced, copying their column to the request's output, and
// seeds waiting requests into the freed lanes, so requests join and leave
// the running batch at superstep granularity.
//
// Everything else runs on worker threads, one request at a time each, on a
// private workspace ("view") that shares the graph's read-only arrays.  A
// worker admits the oldest request once the workspace it needs fits the HBM
// budget next to the lane tables and the other workers' workspaces.
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "vc_graph.h"

using vc::DevBuf;
using vc::fail;
using vc::hip_fail;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Job {
  uint64_t ticket = 0;
  vc_request req{};
  Clock::time_point submitted, started;
  double est_ms = 0;     // expected worker service time, counted in the worker backlog
  bool movable = false;  // routed automatically: may move from the worker queue to a lane table
};

// Running estimate (exponentially weighted mean).
struct Ema {
  double v = 0;
  int64_t n = 0;
  void add(double x) {
    v = n ? 0.75 * v + 0.25 * x : x;
    ++n;
  }
};

constexpr int kMaxLanes = 256;

// Per-superstep control block of a lane table: a device copy and a pinned
// host mirror.  The first part is written by the host, the rest (from
// `live`) by the device after being cleared.
struct LaneCtl {
  int32_t seeds[2 * kMaxLanes];  // (lane, source) of SSSP lanes seeded this superstep
  int32_t cc_lanes[kMaxLanes];   // CC lanes seeded this superstep
  int32_t ret_lanes[kMaxLanes];  // lanes retired after this superstep
  uint32_t* outs[kMaxLanes];     // their requests' outputs
  unsigned long long live[64 * 4];
  unsigned long long stillborn[4];
};
constexpr size_t kCtlIn = offsetof(LaneCtl, live);
static_assert(kCtlIn % 8 == 0 && (sizeof(LaneCtl) - kCtlIn) % 4 == 0, "control block layout");

struct Lane {
  bool busy = false;
  bool cc = false;
  bool fresh = false;  // seeded, first superstep not yet evaluated
  int64_t age = 0;     // supersteps run since seeding
  int64_t cap = 0;
  Job job;
};

struct LaneTable {
  vc_graph g = nullptr;
  int C = 1, K = 64;     // C chunks of 64 lanes
  vc::MsState ms;        // values, mailboxes, masks, broadcast list
  DevBuf ctl;
  int64_t next_edges = 0;  // out-edges of the vertices the last apply activated
  Ema step_ms, steps;      // superstep wall time, supersteps per request
  LaneCtl* host = nullptr;  // pinned
  hipStream_t stream = nullptr;
  std::thread th;
  std::deque<Job> queue;  // guarded by the server mutex
  std::vector<Lane> lanes;
  int busy = 0;
  bool broken = false;
  std::string broken_why;
  size_t bytes = 0;
};

// PageRank / PPR lanes: every busy lane takes one rank update per
// superstep; a lane retires after its T-th.
struct RankSlot {
  bool busy = false;
  int64_t age = 0;  // updates done
  int64_t T = 0;
  Job job;
};

struct RankTable {
  vc_graph g = nullptr;
  int C = 1, K = 64;
  DevBuf contrib, mb, params, seeds;
  DevBuf pull_tiles[4];
  int64_t pull_ntiles[4] = {0, 0, 0, 0};
  vc::RankLane* hparams = nullptr;  // pinned, kMaxLanes entries
  int32_t* hseeds = nullptr;        // pinned, 2 * kMaxLanes entries
  hipStream_t stream = nullptr;
  std::thread th;
  std::deque<Job> queue;  // guarded by the server mutex
  std::vector<RankSlot> lanes;
  int busy = 0;
  bool broken = false;
  std::string broken_why;
  size_t bytes = 0;
  Ema step_ms;
};

struct GraphEntry {
  vc_graph g = nullptr;
  std::unique_ptr<LaneTable> lanes;
  std::unique_ptr<RankTable> ranks;
  Ema alone[4];  // worker service time per program
};

size_t rank_table_bytes(int64_t n, int64_t m, int K) {
  const int C = K / 64;
  size_t b = (size_t)n * K * 16 + kMaxLanes * sizeof(vc::RankLane) + 2 * kMaxLanes * 4;
  for (int c = 1; c <= C; ++c) b += (size_t)((n + m + vc::kMsPullTilePerChunk * c - 1) / (vc::kMsPullTilePerChunk * c) + 1) * 4;
  return b;
}

struct View {
  int32_t graph = -1;
  vc_graph g = nullptr;
  size_t held = 0;
  Clock::time_point used;
};

struct Worker {
  std::thread th;
  hipStream_t stream = nullptr;
  std::vector<View> views;  // touched only by this worker's thread
};

size_t lane_table_bytes(int64_t n, int64_t m, int K) {
  const int C = K / 64;
  size_t b = (size_t)n * K * 8 + (size_t)n * C * 16 + (size_t)((n + 31) / 32) * 4 + sizeof(LaneCtl) +
             (size_t)n * 4 + 4 + (size_t)(n + 1) * 8 + (size_t)vc::scan_scratch_entries(n) * 8 +
             (size_t)((n + m) / vc::kMsPushTile + 2) * 4 + 2 * sizeof(vc::Counters);
  for (int c = 1; c <= C; ++c) b += (size_t)((n + m + vc::kMsPullTilePerChunk * c - 1) / (vc::kMsPullTilePerChunk * c) + 1) * 4;
  return b;
}

}  // namespace

struct vc_server_s {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work;  // workers and lane threads: new work, memory or stop
  std::condition_variable cv_done;  // pollers and drain
  bool stopping = false;
  uint64_t epoch = 0;               // bumped whenever admission could change
  std::vector<GraphEntry> graphs;
  std::deque<Job> queue;            // worker path, arrival order
  std::deque<vc_completion> done;
  uint64_t next_ticket = 1, submitted = 0, completed = 0;
  size_t reserved = 0;              // lane tables
  size_t held = 0;                  // worker workspaces (incl. admitted reservations)
  int running = 0;                  // worker jobs in progress
  double backlog_ms = 0;            // expected service time of the queued worker jobs
  double running_ms = 0;            // and of the running ones
  int64_t lane_steps = 0, lane_requests = 0, lane_push_steps = 0;
  int64_t rank_steps = 0, rank_requests = 0;
  std::vector<std::unique_ptr<Worker>> workers;
};

namespace {

// Caller holds s->mu.
void complete(vc_server s, const Job& j, vc_status st, int32_t supersteps, int lane, const std::string& msg) {
  vc_completion c;
  std::memset(&c, 0, sizeof c);
  c.ticket = j.ticket;
  c.tag = j.req.tag;
  c.status = st;
  c.supersteps = supersteps;
  c.lane = lane;
  const Clock::time_point end = Clock::now();
  c.queue_ms = ms_between(j.submitted, j.started);
  c.service_ms = ms_between(j.started, end);
  if (st != VC_OK) std::strncpy(c.message, msg.c_str(), sizeof c.message - 1);
  s->done.push_back(c);
  ++s->completed;
  ++s->epoch;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// ---------------------------------------------------------------- workers

void worker_main(vc_server s, Worker* w) {
  (void)hipSetDevice(s->device);
  std::vector<vc_graph> drop;
  std::unique_lock<std::mutex> lk(s->mu);
  uint64_t seen = ~0ull;
  for (;;) {
    s->cv_work.wait(lk, [&] { return (s->stopping && s->queue.empty()) || (!s->queue.empty() && s->epoch != seen); });
    if (s->queue.empty()) break;  // stopping
    seen = s->epoch;
    Job& head = s->queue.front();
    const int32_t gid = head.req.graph;
    auto find = [&]() -> int {
      for (size_t i = 0; i < w->views.size(); ++i)
        if (w->views[i].graph == gid) return (int)i;
      return -1;
    };
    int vi = find();
    if (vi < 0) {
      vc_graph v = nullptr;
      if (vc::make_view(s->graphs[gid].g, w->stream, &v) != VC_OK) {
        Job j = std::move(head);
        s->queue.pop_front();
        s->backlog_ms -= j.est_ms;
        j.started = Clock::now();
        complete(s, j, VC_ERR_OUT_OF_MEMORY, 0, -1, std::string("workspace view: ") + vc_last_error());
        continue;
      }
      w->views.push_back(View{gid, v, 0, Clock::now()});
      vi = (int)w->views.size() - 1;
    }
    size_t need = 0;
    (void)vc_graph_footprint(w->views[vi].g, head.req.program, nullptr, &need);
    auto fits = [&](size_t want) { return s->reserved + s->held + want <= s->budget; };
    // drop this worker's other workspaces, least recently used first
    while (!fits(need)) {
      int victim = -1;
      for (size_t i = 0; i < w->views.size(); ++i)
        if (w->views[i].graph != gid && (victim < 0 || w->views[i].used < w->views[victim].used)) victim = (int)i;
      if (victim < 0) break;
      s->held -= w->views[victim].held;
      drop.push_back(w->views[victim].g);
      w->views.erase(w->views.begin() + victim);
      ++s->epoch;
      vi = find();
    }
    // then this graph's own workspace, if it holds buffers of other programs
    if (!fits(need) && w->views[vi].held > 0) {
      vc_graph v = nullptr;
      if (vc::make_view(s->graphs[gid].g, w->stream, &v) == VC_OK) {
        s->held -= w->views[vi].held;
        drop.push_back(w->views[vi].g);
        w->views[vi].g = v;
        w->views[vi].held = 0;
        (void)vc_graph_footprint(v, head.req.program, nullptr, &need);
        ++s->epoch;
      }
    }
    if (!fits(need)) {
      if (s->running == 0 && s->held == 0) {
        Job j = std::move(head);
        s->queue.pop_front();
        s->backlog_ms -= j.est_ms;
        j.started = Clock::now();
        complete(s, j, VC_ERR_OUT_OF_MEMORY, 0, -1,
                 "request needs " + std::to_string(need) + " bytes of workspace; budget left after lane tables: " +
                     std::to_string(s->budget - s->reserved));
      } else if (!drop.empty()) {
        s->cv_work.notify_all();  // freed memory may let another worker proceed
      }
      if (!drop.empty()) {
        std::vector<vc_graph> d;
        d.swap(drop);
        lk.unlock();
        for (vc_graph v : d) vc_graph_destroy(v);
        lk.lock();
      }
      continue;  // wait for the next completion or eviction
    }
    Job job = std::move(head);
    s->queue.pop_front();
    ++s->epoch;
    job.started = Clock::now();
    s->held += need;
    ++s->running;
    s->backlog_ms -= job.est_ms;
    s->running_ms += job.est_ms;
    View& view = w->views[vi];
    view.used = job.started;
    vc_graph vg = view.g;
    const size_t before = view.held;
    lk.unlock();
    for (vc_graph v : drop) vc_graph_destroy(v);
    drop.clear();
    vc_stats st;
    std::memset(&st, 0, sizeof st);
    st.struct_size = sizeof(vc_stats);
    vc_status rc = vc_run(vg, job.req.program, &job.req.params, job.req.out, w->stream, &st);
    std::string msg = rc == VC_OK ? std::string() : std::string(vc_last_error());
    size_t after = 0;
    (void)vc_graph_footprint(vg, job.req.program, &after, nullptr);
    lk.lock();
    s->held = s->held - need - before + after;
    w->views[vi].held = after;
    --s->running;
    s->running_ms -= job.est_ms;
    if (rc == VC_OK) s->graphs[gid].alone[job.req.program].add(ms_between(job.started, Clock::now()));
    complete(s, job, rc, st.supersteps, -1, msg);
  }
  lk.unlock();
  for (View& v : w->views) vc_graph_destroy(v.g);
  w->views.clear();
}

// ---------------------------------------------------------------- lanes

// One superstep of a lane table over its first ceff chunks: seeds the
// listed lanes, runs the superstep (pulled when a CC lane was seeded, which
// activates every vertex) and reads back which lanes are still live.  Runs
// without the server lock.
vc_status lane_superstep(LaneTable* t, int cur, int ceff, const std::vector<int>& sssp, const std::vector<int>& cc,
                         const vc::LaneMask& zero, bool* pushed) {
  vc_graph g = t->g;
  const int64_t n = g->n;
  hipStream_t s = t->stream;
  LaneCtl* h = t->host;
  LaneCtl* d = t->ctl.as<LaneCtl>();
  vc::MsState& ms = t->ms;
  for (size_t j = 0; j < sssp.size(); ++j) {
    h->seeds[2 * j] = sssp[j];
    h->seeds[2 * j + 1] = (int32_t)t->lanes[sssp[j]].job.req.params.source;
  }
  for (size_t j = 0; j < cc.size(); ++j) h->cc_lanes[j] = cc[j];
  if (!sssp.empty() || !cc.empty())
    VC_TRY(hipMemcpyAsync(d, h, offsetof(LaneCtl, ret_lanes), hipMemcpyHostToDevice, s));
  VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(d->live), (int64_t)(sizeof(LaneCtl) - kCtlIn) / 4, 0u, s));
  VC_TRY(vc::launch_lane_seed_cc(g->off, g->off64, g->relabeled ? g->inv_p : nullptr, n, d->cc_lanes, (int)cc.size(),
                                 ms.D.as<uint32_t>(), ms.A[cur].as<unsigned long long>(), s));
  VC_TRY(vc::launch_lane_seed_sssp(g->off, g->off64, g->relabeled ? g->perm_p : nullptr, n, d->seeds,
                                   (int)sssp.size(), ms.D.as<uint32_t>(), ms.A[cur].as<unsigned long long>(),
                                   d->stillborn, s));
  vc_status st = vc::ms_superstep(ms, g, cur, ceff, t->next_edges, !cc.empty(), zero, d->live, pushed, s);
  if (st != VC_OK) return st;
  VC_TRY(hipMemcpyAsync(&h->live, &d->live, sizeof(LaneCtl) - kCtlIn, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
  t->next_edges = (int64_t)ms.host[0].edges;
  return VC_OK;
}

struct Retired {
  int lane;
  vc_status status;
  int32_t supersteps;
};

// Copies the retired lanes' columns to their outputs and resets them;
// lanes in `drop` (stopped at the cap while active) leave the active masks.
vc_status lane_retire(LaneTable* t, int next, const std::vector<Retired>& r, const vc::LaneMask& drop, bool any_drop) {
  vc_graph g = t->g;
  hipStream_t s = t->stream;
  LaneCtl* h = t->host;
  LaneCtl* d = t->ctl.as<LaneCtl>();
  for (size_t j = 0; j < r.size(); ++j) {
    h->ret_lanes[j] = r[j].lane;
    h->outs[j] = static_cast<uint32_t*>(t->lanes[r[j].lane].job.req.out);
  }
  VC_TRY(hipMemcpyAsync(d->ret_lanes, h->ret_lanes, kCtlIn - offsetof(LaneCtl, ret_lanes), hipMemcpyHostToDevice, s));
  if (any_drop) VC_TRY(vc::launch_lane_clear(t->ms.A[next].as<unsigned long long>(), g->n, t->C, drop, s));
  VC_TRY(vc::launch_lane_retire(t->ms.D.as<uint32_t>(), g->relabeled ? g->perm_p : nullptr, g->n, d->ret_lanes,
                                d->outs, (int)r.size(), s));
  VC_TRY(hipStreamSynchronize(s));
  return VC_OK;
}

void lane_main(vc_server s, LaneTable* t) {
  (void)hipSetDevice(s->device);
  const int64_t n = t->g->n, m = t->g->m;
  int cur = 0;
  std::vector<int> sssp, cc;
  std::vector<Retired> retired;
  for (;;) {
    sssp.clear();
    cc.clear();
    vc::LaneMask zero{};
    int ceff = 1;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stopping || t->busy > 0 || !t->queue.empty(); });
      if (t->busy == 0 && t->queue.empty()) break;  // stopping
      if (t->broken) {
        while (!t->queue.empty()) {
          Job j = std::move(t->queue.front());
          t->queue.pop_front();
          j.started = Clock::now();
          complete(s, j, VC_ERR_HIP, 0, -1, t->broken_why);
        }
        continue;
      }
      for (int l = 0; l < t->K && !t->queue.empty(); ++l) {
        Lane& ln = t->lanes[l];
        if (ln.busy) continue;
        ln.job = std::move(t->queue.front());
        t->queue.pop_front();
        ln.job.started = Clock::now();
        ln.busy = true;
        ln.fresh = true;
        ln.age = 0;
        ln.cc = ln.job.req.program == VC_CC_HASHMIN;
        ln.cap = ln.job.req.params.max_supersteps > 0 ? (int64_t)ln.job.req.params.max_supersteps : n + 1;
        ++t->busy;
        (ln.cc ? cc : sssp).push_back(l);
      }
      for (int l = 0; l < t->K; ++l)
        if (t->lanes[l].busy) {
          if (t->lanes[l].cc) zero.bits[l >> 6] |= 1ull << (l & 63);
          ceff = (l >> 6) + 1;  // busy lanes fill the table from the front
        }
    }
    bool pushed = false;
    const Clock::time_point t_step = Clock::now();
    vc_status st = lane_superstep(t, cur, ceff, sssp, cc, zero, &pushed);
    retired.clear();
    vc::LaneMask drop{};
    bool any_drop = false;
    if (st == VC_OK) {
      unsigned long long live[4] = {0, 0, 0, 0};
      for (int w = 0; w < 64; ++w)
        for (int c = 0; c < t->C; ++c) live[c] |= t->host->live[w * t->C + c];
      for (int l = 0; l < t->K; ++l) {
        Lane& ln = t->lanes[l];
        if (!ln.busy) continue;
        const unsigned long long bit = 1ull << (l & 63);
        ++ln.age;
        const bool is_live = (live[l >> 6] & bit) != 0;
        // a program that could not send at its first superstep ends there
        const bool stillborn = ln.fresh && (ln.cc ? m == 0 : (t->host->stillborn[l >> 6] & bit) != 0);
        ln.fresh = false;
        if (stillborn) {
          retired.push_back({l, VC_OK, 1});
        } else if (ln.age >= ln.cap) {
          retired.push_back({l, VC_ERR_NOT_CONVERGED, (int32_t)ln.age});
          if (is_live) {
            drop.bits[l >> 6] |= bit;
            any_drop = true;
          }
        } else if (!is_live) {
          retired.push_back({l, VC_OK, (int32_t)(ln.age + 1)});
        }
      }
      if (!retired.empty()) st = lane_retire(t, 1 - cur, retired, drop, any_drop);
    }
    std::string why = st == VC_OK ? std::string() : std::string(vc_last_error());
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->lane_steps;
    if (pushed) ++s->lane_push_steps;
    t->step_ms.add(ms_between(t_step, Clock::now()));
    if (st != VC_OK) {
      // a failed launch or copy leaves the table unusable: fail its requests
      t->broken = true;
      t->broken_why = why;
      for (Lane& ln : t->lanes)
        if (ln.busy) {
          complete(s, ln.job, st, 0, -1, why);
          ln.busy = false;
        }
      t->busy = 0;
      continue;
    }
    for (const Retired& r : retired) {
      Lane& ln = t->lanes[r.lane];
      complete(s, ln.job, r.status, r.supersteps, r.lane,
               r.status == VC_OK ? std::string() : std::string("superstep cap reached before quiescence"));
      t->steps.add(r.supersteps);
      ln.busy = false;
      --t->busy;
      ++s->lane_requests;
    }
    cur = 1 - cur;
  }
}

vc_status lane_table_init(LaneTable* t, vc_graph g, int K) {
  t->g = g;
  t->K = K;
  t->C = K / 64;
  VC_TRY(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
  VC_TRY(t->ctl.ensure(sizeof(LaneCtl)));
  VC_TRY(hipHostMalloc((void**)&t->host, sizeof(LaneCtl), hipHostMallocDefault));
  std::memset(t->host, 0, sizeof(LaneCtl));
  vc_status st = vc::ms_reset(t->ms, g, t->C, t->stream);
  if (st != VC_OK) return st;
  VC_TRY(hipStreamSynchronize(t->stream));
  t->lanes.resize(K);
  t->bytes = lane_table_bytes(g->n, g->m, K);
  return VC_OK;
}

void lane_table_free(LaneTable* t) {
  t->ms.release();
  t->ctl.release();
  if (t->host) (void)hipHostFree(t->host);
  t->host = nullptr;
  if (t->stream) (void)hipStreamDestroy(t->stream);
  t->stream = nullptr;
}

// ---------------------------------------------------------------- rank lanes

void rank_main(vc_server s, RankTable* t) {
  (void)hipSetDevice(s->device);
  vc_graph g = t->g;
  const int64_t n = g->n;
  std::vector<int> seeded;
  std::vector<int> finished;
  for (;;) {
    seeded.clear();
    finished.clear();
    int ceff = 1;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stopping || t->busy > 0 || !t->queue.empty(); });
      if (t->busy == 0 && t->queue.empty()) break;  // stopping
      if (t->broken) {
        while (!t->queue.empty()) {
          Job j = std::move(t->queue.front());
          t->queue.pop_front();
          j.started = Clock::now();
          complete(s, j, VC_ERR_HIP, 0, -1, t->broken_why);
        }
        continue;
      }
      for (int l = 0; l < t->K && !t->queue.empty(); ++l) {
        RankSlot& sl = t->lanes[l];
        if (sl.busy) continue;
        sl.job = std::move(t->queue.front());
        t->queue.pop_front();
        sl.job.started = Clock::now();
        sl.busy = true;
        sl.age = 0;
        sl.T = sl.job.req.params.max_supersteps;
        ++t->busy;
        seeded.push_back(l);
      }
      for (int l = 0; l < t->K; ++l)
        if (t->lanes[l].busy) ceff = (l >> 6) + 1;
    }
    const Clock::time_point t0 = Clock::now();
    for (size_t j = 0; j < seeded.size(); ++j) {
      const vc_request& r = t->lanes[seeded[j]].job.req;
      t->hseeds[2 * j] = seeded[j];
      t->hseeds[2 * j + 1] = r.program == VC_PPR ? (int32_t)r.params.source : -1;
    }
    for (int l = 0; l < 64 * ceff; ++l) {
      const RankSlot& sl = t->lanes[l];
      vc::RankLane& P = t->hparams[l];
      if (!sl.busy) {
        P.state = 0;
        continue;
      }
      const vc_request& r = sl.job.req;
      const double d = r.params.damping;
      P.damping = d;
      P.teleport = r.program == VC_PPR ? (1.0 - d) : (1.0 - d) / (double)n;
      P.out = static_cast<float*>(r.out);
      P.source = r.program == VC_PPR ? (int32_t)r.params.source : -1;
      P.state = sl.age + 1 == sl.T ? 2 : 1;
    }
    hipError_t e = hipMemcpyAsync(t->params.p, t->hparams, sizeof(vc::RankLane) * 64 * ceff, hipMemcpyHostToDevice,
                                  t->stream);
    if (e == hipSuccess && !seeded.empty())
      e = hipMemcpyAsync(t->seeds.p, t->hseeds, seeded.size() * 8, hipMemcpyHostToDevice, t->stream);
    const int32_t* ids = g->relabeled ? g->inv_p : nullptr;
    if (e == hipSuccess)
      e = vc::launch_rl_seed(g->off, g->off64, ids, n, t->seeds.as<int32_t>(), (int)seeded.size(),
                             t->contrib.as<unsigned long long>(), t->stream);
    if (e == hipSuccess)
      e = vc::launch_rl_pull(ceff, g->csc_off_p, g->in_src, n, g->m, t->pull_tiles[ceff - 1].as<int32_t>(),
                             vc::kMsPullTilePerChunk * ceff, t->pull_ntiles[ceff - 1],
                             t->contrib.as<unsigned long long>(), t->mb.as<unsigned long long>(), t->stream);
    if (e == hipSuccess)
      e = vc::launch_rl_apply(g->off, g->off64, ids, n, ceff, t->params.as<vc::RankLane>(),
                              t->contrib.as<unsigned long long>(), t->mb.as<unsigned long long>(), t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->rank_steps;
    t->step_ms.add(ms_between(t0, Clock::now()));
    if (e != hipSuccess) {
      hip_fail(e, "rank lane superstep");
      t->broken = true;
      t->broken_why = vc_last_error();
      for (RankSlot& sl : t->lanes)
        if (sl.busy) {
          complete(s, sl.job, VC_ERR_HIP, 0, -1, t->broken_why);
          sl.busy = false;
        }
      t->busy = 0;
      continue;
    }
    for (int l = 0; l < t->K; ++l) {
      RankSlot& sl = t->lanes[l];
      if (!sl.busy || ++sl.age < sl.T) continue;
      complete(s, sl.job, VC_OK, (int32_t)(sl.T + 1), l, std::string());
      sl.busy = false;
      --t->busy;
      ++s->rank_requests;
    }
  }
}

vc_status rank_table_init(RankTable* t, vc_graph g, int K) {
  t->g = g;
  t->K = K;
  t->C = K / 64;
  const int64_t n = g->n, m = g->m;
  if ((size_t)(4 * vc::kMsPullTilePerChunk + 2) * 8 > g->max_lds) return fail(VC_ERR_UNSUPPORTED, "pull tile exceeds LDS");
  VC_TRY(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
  VC_TRY(t->contrib.ensure((size_t)n * K * 8));
  VC_TRY(t->mb.ensure((size_t)n * K * 8));
  VC_TRY(t->params.ensure(kMaxLanes * sizeof(vc::RankLane)));
  VC_TRY(t->seeds.ensure(2 * kMaxLanes * 4));
  VC_TRY(hipHostMalloc((void**)&t->hparams, kMaxLanes * sizeof(vc::RankLane), hipHostMallocDefault));
  VC_TRY(hipHostMalloc((void**)&t->hseeds, 2 * kMaxLanes * 4, hipHostMallocDefault));
  std::memset(t->hparams, 0, kMaxLanes * sizeof(vc::RankLane));
  for (int c = 1; c <= t->C; ++c) {
    const int64_t tile = vc::kMsPullTilePerChunk * c;
    const int64_t ntiles = (n + m + tile - 1) / tile;
    VC_TRY(t->pull_tiles[c - 1].ensure((size_t)(ntiles + 1) * 4));
    VC_TRY(vc::launch_mp_partition(g->csc_off_p, true, n, n + m, tile, ntiles, t->pull_tiles[c - 1].as<int32_t>(),
                                   t->stream));
    t->pull_ntiles[c - 1] = ntiles;
  }
  VC_TRY(vc::launch_fill_u32(t->contrib.as<uint32_t>(), n * K * 2, 0u, t->stream));
  VC_TRY(vc::launch_fill_u32(t->mb.as<uint32_t>(), n * K * 2, 0u, t->stream));
  VC_TRY(hipStreamSynchronize(t->stream));
  t->lanes.resize(K);
  t->bytes = rank_table_bytes(n, m, K);
  return VC_OK;
}

void rank_table_free(RankTable* t) {
  for (DevBuf* b : {&t->contrib, &t->mb, &t->params, &t->seeds, &t->pull_tiles[0], &t->pull_tiles[1],
                    &t->pull_tiles[2], &t->pull_tiles[3]})
    b->release();
  if (t->hparams) (void)hipHostFree(t->hparams);
  if (t->hseeds) (void)hipHostFree(t->hseeds);
  t->hparams = nullptr;
  t->hseeds = nullptr;
  if (t->stream) (void)hipStreamDestroy(t->stream);
  t->stream = nullptr;
}

// Expected worker service time of a request: the mean of the graph's past
// worker runs of the program, before any a prior from the edge count (about
// 0.1 ns per edge for a min program, 12 ps per edge and iteration for a
// rank program, as measured on R-MAT graphs).
double worker_estimate(const GraphEntry& ge, const vc_request& r) {
  if (ge.alone[r.program].n) return ge.alone[r.program].v;
  const double m = (double)ge.g->m;
  if (r.program == VC_PAGERANK || r.program == VC_PPR) return (double)r.params.max_supersteps * (0.05 + m * 1.2e-8);
  return 0.5 + m * 1e-7;
}

// Workers share one GPU: bandwidth-bound runs overlap little, so the
// backlog drains at about this many runs' worth at a time, however many
// worker threads there are.
constexpr double kWorkerOverlap = 2.0;
// Lanes trade latency for throughput (a lane waits for whole-graph
// supersteps), so they are chosen only when clearly ahead.
constexpr double kLaneMargin = 2.0;

double worker_wait(vc_server s) {
  const double w = s->workers.size() < kWorkerOverlap ? (double)s->workers.size() : kWorkerOverlap;
  return (s->backlog_ms + 0.5 * s->running_ms) / w;
}

// Routing of a request on a graph with a lane table: the lane table when its
// expected completion time is shorter than the worker path's.  Worker path:
// the queued and running worker jobs' expected service times, drained
// kWorkerOverlap at a time, plus this request's.  Lane table (counted
// kLaneMargin times): supersteps per request times superstep time (means of its past runs; before any, 20
// supersteps of a model time that reads every edge and the value rows of
// the chunks in use once), once more for every table-full of requests
// queued ahead.  Rank lanes: T updates of the table's superstep time (model
// before any run: every edge's message row and every value row of the
// chunks in use read once).  Caller holds s->mu.
bool rank_lane_is_faster(vc_server s, const GraphEntry& ge, const vc_request& r) {
  const RankTable& t = *ge.ranks;
  const double worker = worker_wait(s) + worker_estimate(ge, r);
  const int64_t want = t.busy + (int64_t)t.queue.size() + 1;
  const double c = (double)(want >= t.K ? t.C : (want + 63) / 64);
  const double step = t.step_ms.n ? t.step_ms.v : ((double)t.g->m * 512.0 * c + (double)t.g->n * c * 64.0 * 24.0) / 3e9;
  const int64_t ahead = (int64_t)t.queue.size() - (t.K - t.busy);
  const double rounds = 1.0 + (ahead >= 0 ? (double)(ahead / t.K + 1) : 0.0);
  return kLaneMargin * rounds * (double)r.params.max_supersteps * step < worker;
}

bool lane_is_faster(vc_server s, const GraphEntry& ge, const vc_request& r) {
  const LaneTable& t = *ge.lanes;
  const double worker = worker_wait(s) + worker_estimate(ge, r);
  const int64_t want = t.busy + (int64_t)t.queue.size() + 1;
  const double c = (double)(want >= t.K ? t.C : (want + 63) / 64);
  const double step = t.step_ms.n ? t.step_ms.v : ((double)t.g->m * 64.0 + (double)t.g->n * c * 1024.0) / 2e9;
  const double steps = t.steps.n ? t.steps.v : 20.0;
  const int64_t ahead = (int64_t)t.queue.size() - (t.K - t.busy);
  const double rounds = 1.0 + (ahead >= 0 ? (double)(ahead / t.K + 1) : 0.0);
  return kLaneMargin * rounds * steps * step < worker;
}

bool lane_eligible(const GraphEntry& ge, const vc_request& r, bool rank) {
  if (rank)
    return ge.ranks && (r.program == VC_PAGERANK || r.program == VC_PPR) && r.params.max_supersteps > 0 &&
           !(r.params.options & (VC_OPT_F32_ACCUMULATE | VC_OPT_F32_MESSAGES));
  return ge.lanes && (r.program == VC_CC_HASHMIN || r.program == VC_SSSP);
}

// Batching trigger.  A lane generation costs about the same GPU time however
// many lanes are busy, so it pays once the requests it would serve would cost
// more run alone: when the automatically routed, lane-eligible requests of
// graph gid waiting in the worker queue add up (in expected worker time) to
// kLaneMargin generations' time (supersteps per request times superstep
// time for the lane chunks they fill; T updates for rank lanes), they move
// to the lane table together.  The margin covers what the estimates miss:
// a generation shares the GPU with the workers' runs.  Caller holds s->mu.
void batch_from_queue(vc_server s, int32_t gid, bool rank) {
  GraphEntry& ge = s->graphs[gid];
  int64_t count = 0, max_t = 0;
  double alone = 0;
  for (const Job& j : s->queue)
    if (j.movable && j.req.graph == gid && lane_eligible(ge, j.req, rank)) {
      ++count;
      alone += j.est_ms;
      if (j.req.params.max_supersteps > max_t) max_t = j.req.params.max_supersteps;
    }
  if (count < 2) return;
  double generation;
  if (rank) {
    const RankTable& t = *ge.ranks;
    const int64_t want = count < t.K ? count : t.K;
    const double c = (double)((want + 63) / 64);
    const double step = t.step_ms.n ? t.step_ms.v
                                    : ((double)t.g->m * 512.0 * c + (double)t.g->n * c * 64.0 * 24.0) / 3e9;
    generation = (double)max_t * step * (double)((count + t.K - 1) / t.K);
  } else {
    const LaneTable& t = *ge.lanes;
    const int64_t want = count < t.K ? count : t.K;
    const double c = (double)((want + 63) / 64);
    const double step = t.step_ms.n ? t.step_ms.v : ((double)t.g->m * 64.0 + (double)t.g->n * c * 1024.0) / 2e9;
    const double steps = t.steps.n ? t.steps.v : 20.0;
    generation = steps * step * (double)((count + t.K - 1) / t.K);
  }
  if (alone < kLaneMargin * generation) return;
  std::deque<Job>& dest = rank ? ge.ranks->queue : ge.lanes->queue;
  for (auto it = s->queue.begin(); it != s->queue.end();) {
    if (it->movable && it->req.graph == gid && lane_eligible(ge, it->req, rank)) {
      s->backlog_ms -= it->est_ms;
      it->est_ms = 0;
      dest.push_back(std::move(*it));
      it = s->queue.erase(it);
    } else {
      ++it;
    }
  }
  ++s->epoch;
  s->cv_work.notify_all();
}

}  // namespace

extern "C" {

vc_status vc_server_create(const vc_server_config* config, vc_server* out) {
  if (!out) return fail(VC_ERR_INVALID_ARG, "null out");
  vc_server_config cfg;
  std::memset(&cfg, 0, sizeof cfg);
  cfg.struct_size = sizeof cfg;
  if (config) {
    if (config->struct_size != sizeof(vc_server_config))
      return fail(VC_ERR_INVALID_ARG, "vc_server_config.struct_size mismatch");
    cfg = *config;
  }
  if (cfg.workers == 0) cfg.workers = 2;
  if (cfg.workers < 1 || cfg.workers > 64) return fail(VC_ERR_INVALID_ARG, "workers must be in 1..64");
  int dev = 0;
  VC_TRY(hipGetDevice(&dev));
  size_t budget = cfg.hbm_budget;
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    VC_TRY(hipMemGetInfo(&free_b, &total_b));
    budget = free_b / 5 * 4;
  }
  vc_server s = new (std::nothrow) vc_server_s();
  if (!s) return fail(VC_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->device = dev;
  s->budget = budget;
  for (int i = 0; i < cfg.workers; ++i) {
    std::unique_ptr<Worker> w(new Worker());
    hipError_t e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      vc_server_destroy(s);
      return hip_fail(e, "worker stream");
    }
    s->workers.push_back(std::move(w));
  }
  for (auto& w : s->workers) w->th = std::thread(worker_main, s, w.get());
  *out = s;
  return VC_OK;
}

vc_status vc_server_add_graph(vc_server s, vc_graph g, int32_t lanes, int32_t rank_lanes, int32_t* id) {
  if (!s || !g || !id) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (lanes < 0 || lanes > kMaxLanes || lanes % 64) return fail(VC_ERR_INVALID_ARG, "lanes must be 0, 64, 128, 192 or 256");
  if (rank_lanes < 0 || rank_lanes > kMaxLanes || rank_lanes % 64)
    return fail(VC_ERR_INVALID_ARG, "rank_lanes must be 0, 64, 128, 192 or 256");
  if (g->is_view) return fail(VC_ERR_INVALID_ARG, "not a graph handle");
  if (g->device != s->device) return fail(VC_ERR_INVALID_ARG, "graph lives on another device than the server");
  // the shared read-only arrays (transpose, default partitions) are built
  // before the graph is registered, outside the lock: nothing else uses it yet
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  VC_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  vc_status rc = vc::prepare_shared(g, st);
  (void)hipStreamDestroy(st);
  if (rc != VC_OK) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail(VC_ERR_INVALID_ARG, "server is shutting down");
  GraphEntry e;
  e.g = g;
  if (lanes > 0) {
    const size_t need = lane_table_bytes(g->n, g->m, lanes);
    if (s->reserved + s->held + need > s->budget)
      return fail(VC_ERR_OUT_OF_MEMORY, "lane table of " + std::to_string(need) + " bytes exceeds the budget left");
    std::unique_ptr<LaneTable> t(new LaneTable());
    rc = lane_table_init(t.get(), g, lanes);
    if (rc != VC_OK) {
      lane_table_free(t.get());
      return rc;
    }
    s->reserved += t->bytes;
    e.lanes = std::move(t);
  }
  if (rank_lanes > 0) {
    const size_t need = rank_table_bytes(g->n, g->m, rank_lanes);
    if (s->reserved + s->held + need > s->budget) {
      if (e.lanes) {
        lane_table_free(e.lanes.get());
        s->reserved -= e.lanes->bytes;
      }
      return fail(VC_ERR_OUT_OF_MEMORY, "rank lane table of " + std::to_string(need) + " bytes exceeds the budget left");
    }
    std::unique_ptr<RankTable> t(new RankTable());
    rc = rank_table_init(t.get(), g, rank_lanes);
    if (rc != VC_OK) {
      rank_table_free(t.get());
      if (e.lanes) {
        lane_table_free(e.lanes.get());
        s->reserved -= e.lanes->bytes;
      }
      return rc;
    }
    s->reserved += t->bytes;
    e.ranks = std::move(t);
  }
  if (e.lanes) e.lanes->th = std::thread(lane_main, s, e.lanes.get());
  if (e.ranks) e.ranks->th = std::thread(rank_main, s, e.ranks.get());
  s->graphs.push_back(std::move(e));
  *id = (int32_t)s->graphs.size() - 1;
  return VC_OK;
}

vc_status vc_server_submit(vc_server s, const vc_request* req, uint64_t* ticket) {
  if (!s || !req) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (req->struct_size != sizeof(vc_request)) return fail(VC_ERR_INVALID_ARG, "vc_request.struct_size mismatch");
  if (req->program < VC_PAGERANK || req->program > VC_PPR) return fail(VC_ERR_INVALID_ARG, "bad program");
  if (!req->out || (uintptr_t)req->out % 4) return fail(VC_ERR_INVALID_ARG, "null or misaligned out");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail(VC_ERR_INVALID_ARG, "server is shutting down");
  if (req->graph < 0 || req->graph >= (int32_t)s->graphs.size()) return fail(VC_ERR_INVALID_ARG, "unknown graph id");
  GraphEntry& ge = s->graphs[req->graph];
  std::string why;
  if (!vc::valid_params(req->params, req->program, ge.g->n, &why)) return fail(VC_ERR_INVALID_ARG, why);
  Job j;
  j.ticket = s->next_ticket++;
  j.req = *req;
  j.submitted = Clock::now();
  if (req->route < VC_ROUTE_AUTO || req->route > VC_ROUTE_WORKER) return fail(VC_ERR_INVALID_ARG, "bad route");
  // Automatic routing: join a lane table's running generation when that
  // finishes sooner than the worker path; otherwise queue for a worker,
  // where the batching trigger may gather it into a new generation.  Rank
  // lanes sum in exact fixed point: binary32 requests and T = 0 stay on
  // workers.
  bool lane = req->route != VC_ROUTE_WORKER && lane_eligible(ge, *req, false);
  bool rank = req->route != VC_ROUTE_WORKER && lane_eligible(ge, *req, true);
  if (req->route == VC_ROUTE_AUTO) {
    lane = lane && ge.lanes->busy > 0 && lane_is_faster(s, ge, *req);
    rank = rank && ge.ranks->busy > 0 && rank_lane_is_faster(s, ge, *req);
  }
  if (lane) {
    ge.lanes->queue.push_back(j);
  } else if (rank) {
    ge.ranks->queue.push_back(j);
  } else {
    j.est_ms = worker_estimate(ge, *req);
    j.movable = req->route == VC_ROUTE_AUTO && (lane_eligible(ge, *req, false) || lane_eligible(ge, *req, true));
    s->backlog_ms += j.est_ms;
    s->queue.push_back(j);
    if (j.movable) batch_from_queue(s, req->graph, lane_eligible(ge, *req, true));
  }
  ++s->submitted;
  ++s->epoch;
  s->cv_work.notify_all();
  if (ticket) *ticket = j.ticket;
  return VC_OK;
}

vc_status vc_server_poll(vc_server s, vc_completion* done, int32_t cap, int32_t timeout_ms, int32_t* count) {
  if (!s || !count || (cap > 0 && !done) || cap < 0) return fail(VC_ERR_INVALID_ARG, "bad argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_ms != 0) {
    auto ready = [&] { return !s->done.empty(); };
    if (timeout_ms < 0)
      s->cv_done.wait(lk, ready);
    else
      s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  }
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    done[k++] = s->done.front();
    s->done.pop_front();
  }
  *count = k;
  return VC_OK;
}

vc_status vc_server_drain(vc_server s) {
  if (!s) return fail(VC_ERR_INVALID_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  const uint64_t target = s->submitted;
  s->cv_done.wait(lk, [&] { return s->completed >= target; });
  return VC_OK;
}

vc_status vc_server_info_get(vc_server s, vc_server_info* info) {
  if (!s || !info) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (info->struct_size != sizeof(vc_server_info)) return fail(VC_ERR_INVALID_ARG, "vc_server_info.struct_size mismatch");
  std::lock_guard<std::mutex> lk(s->mu);
  info->graphs = (int32_t)s->graphs.size();
  info->hbm_budget = s->budget;
  info->bytes_reserved = s->reserved;
  info->bytes_held = s->held;
  info->submitted = s->submitted;
  info->completed = s->completed;
  info->lane_supersteps = s->lane_steps;
  info->lane_requests = s->lane_requests;
  info->lane_push_supersteps = s->lane_push_steps;
  info->rank_supersteps = s->rank_steps;
  info->rank_requests = s->rank_requests;
  return VC_OK;
}

vc_status vc_server_destroy(vc_server s) {
  if (!s) return VC_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed >= s->submitted; });
    s->stopping = true;
    ++s->epoch;
    s->cv_work.notify_all();
  }
  for (auto& w : s->workers)
    if (w->th.joinable()) w->th.join();
  for (GraphEntry& e : s->graphs) {
    if (e.lanes && e.lanes->th.joinable()) e.lanes->th.join();
    if (e.ranks && e.ranks->th.joinable()) e.ranks->th.join();
  }
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (auto& w : s->workers)
    if (w->stream) (void)hipStreamDestroy(w->stream);
  for (GraphEntry& e : s->graphs) {
    if (e.lanes) lane_table_free(e.lanes.get());
    if (e.ranks) rank_table_free(e.ranks.get());
  }
  (void)hipSetDevice(prev);
  delete s;
  return VC_OK;
}

}  // extern "C"

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
  vc::Counters ctr;
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
  int C = 1, K = 64;
  DevBuf D, MB, A0, A1, bits, ctl;
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

struct GraphEntry {
  vc_graph g = nullptr;
  std::unique_ptr<LaneTable> lanes;
};

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

size_t lane_table_bytes(int64_t n, int K) {
  const int C = K / 64;
  return (size_t)n * K * 8 + (size_t)n * C * 16 + (size_t)((n + 31) / 32) * 4 + sizeof(LaneCtl);
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
  int64_t lane_steps = 0, lane_requests = 0;
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
    complete(s, job, rc, st.supersteps, -1, msg);
  }
  lk.unlock();
  for (View& v : w->views) vc_graph_destroy(v.g);
  w->views.clear();
}

// ---------------------------------------------------------------- lanes

// One superstep of a lane table: seeds the listed lanes, pulls, applies and
// reads back which lanes are still live.  Runs without the server lock.
vc_status lane_superstep(LaneTable* t, int cur, const std::vector<int>& sssp, const std::vector<int>& cc,
                         const vc::LaneMask& zero) {
  vc_graph g = t->g;
  const int64_t n = g->n, m = g->m;
  hipStream_t s = t->stream;
  LaneCtl* h = t->host;
  LaneCtl* d = t->ctl.as<LaneCtl>();
  unsigned long long* A[2] = {t->A0.as<unsigned long long>(), t->A1.as<unsigned long long>()};
  for (size_t j = 0; j < sssp.size(); ++j) {
    h->seeds[2 * j] = sssp[j];
    h->seeds[2 * j + 1] = (int32_t)t->lanes[sssp[j]].job.req.params.source;
  }
  for (size_t j = 0; j < cc.size(); ++j) h->cc_lanes[j] = cc[j];
  if (!sssp.empty() || !cc.empty())
    VC_TRY(hipMemcpyAsync(d, h, offsetof(LaneCtl, ret_lanes), hipMemcpyHostToDevice, s));
  VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(d->live), (int64_t)(sizeof(LaneCtl) - kCtlIn) / 4, 0u, s));
  VC_TRY(vc::launch_lane_seed_cc(t->C, g->off, g->off64, g->relabeled ? g->inv_p : nullptr, n, d->cc_lanes,
                                 (int)cc.size(), t->D.as<uint32_t>(), A[cur], s));
  VC_TRY(vc::launch_lane_seed_sssp(t->C, g->off, g->off64, g->relabeled ? g->perm_p : nullptr, d->seeds,
                                   (int)sssp.size(), t->D.as<uint32_t>(), A[cur], d->stillborn, s));
  VC_TRY(vc::launch_ms_pull(t->C, g->w != nullptr, g->csc_off_p, g->in_src, g->in_w, n, m, g->csc_tiles_p,
                            g->csc_tile, g->csc_ntiles, t->D.as<uint32_t>(), t->MB.as<uint32_t>(), A[cur],
                            t->bits.as<uint32_t>(), zero, s));
  VC_TRY(vc::launch_fill_u32(reinterpret_cast<uint32_t*>(A[1 - cur]), 2 * n * t->C, 0u, s));
  VC_TRY(vc::launch_ms_apply(t->C, g->off, g->off64, n, t->D.as<uint32_t>(), t->MB.as<uint32_t>(), A[1 - cur],
                             t->bits.as<uint32_t>(), &d->ctr, d->live, s));
  VC_TRY(hipMemcpyAsync(&h->live, &d->live, sizeof(LaneCtl) - kCtlIn, hipMemcpyDeviceToHost, s));
  VC_TRY(hipStreamSynchronize(s));
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
  if (any_drop)
    VC_TRY(vc::launch_lane_clear(t->C, next ? t->A1.as<unsigned long long>() : t->A0.as<unsigned long long>(), g->n,
                                 drop, s));
  VC_TRY(vc::launch_lane_retire(t->C, t->D.as<uint32_t>(), g->relabeled ? g->perm_p : nullptr, g->n, d->ret_lanes,
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
        if (t->lanes[l].busy && t->lanes[l].cc) zero.bits[l >> 6] |= 1ull << (l & 63);
    }
    vc_status st = lane_superstep(t, cur, sssp, cc, zero);
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
      ln.busy = false;
      --t->busy;
      ++s->lane_requests;
    }
    cur = 1 - cur;
  }
}

vc_status lane_table_init(vc_server s, LaneTable* t, vc_graph g, int K) {
  t->g = g;
  t->K = K;
  t->C = K / 64;
  const int64_t n = g->n;
  VC_TRY(hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking));
  VC_TRY(t->D.ensure((size_t)n * K * 4));
  VC_TRY(t->MB.ensure((size_t)n * K * 4));
  VC_TRY(t->A0.ensure((size_t)n * t->C * 8));
  VC_TRY(t->A1.ensure((size_t)n * t->C * 8));
  VC_TRY(t->bits.ensure((size_t)((n + 31) / 32) * 4));
  VC_TRY(t->ctl.ensure(sizeof(LaneCtl)));
  VC_TRY(hipHostMalloc((void**)&t->host, sizeof(LaneCtl), hipHostMallocDefault));
  std::memset(t->host, 0, sizeof(LaneCtl));
  VC_TRY(vc::launch_fill_u32(t->D.as<uint32_t>(), n * K, vc::kInf, t->stream));
  VC_TRY(vc::launch_fill_u32(t->MB.as<uint32_t>(), n * K, vc::kInf, t->stream));
  VC_TRY(vc::launch_fill_u32(t->A0.as<uint32_t>(), 2 * n * t->C, 0u, t->stream));
  VC_TRY(vc::launch_fill_u32(t->A1.as<uint32_t>(), 2 * n * t->C, 0u, t->stream));
  VC_TRY(vc::launch_fill_u32(t->bits.as<uint32_t>(), (n + 31) / 32, 0u, t->stream));
  VC_TRY(hipStreamSynchronize(t->stream));
  t->lanes.resize(K);
  t->bytes = lane_table_bytes(n, K);
  (void)s;
  return VC_OK;
}

void lane_table_free(LaneTable* t) {
  for (DevBuf* b : {&t->D, &t->MB, &t->A0, &t->A1, &t->bits, &t->ctl}) b->release();
  if (t->host) (void)hipHostFree(t->host);
  t->host = nullptr;
  if (t->stream) (void)hipStreamDestroy(t->stream);
  t->stream = nullptr;
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

vc_status vc_server_add_graph(vc_server s, vc_graph g, int32_t lanes, int32_t* id) {
  if (!s || !g || !id) return fail(VC_ERR_INVALID_ARG, "null argument");
  if (lanes < 0 || lanes > kMaxLanes || lanes % 64) return fail(VC_ERR_INVALID_ARG, "lanes must be 0, 64, 128, 192 or 256");
  if (g->is_view) return fail(VC_ERR_INVALID_ARG, "not a graph handle");
  if (g->device != s->device) return fail(VC_ERR_INVALID_ARG, "graph lives on another device than the server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return fail(VC_ERR_INVALID_ARG, "server is shutting down");
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  VC_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  // builds the shared read-only arrays once (transpose, default partitions)
  vc_graph probe = nullptr;
  vc_status rc = vc::make_view(g, st, &probe);
  (void)hipStreamDestroy(st);
  if (rc != VC_OK) return rc;
  vc_graph_destroy(probe);
  GraphEntry e;
  e.g = g;
  if (lanes > 0) {
    const size_t need = lane_table_bytes(g->n, lanes);
    if (s->reserved + s->held + need > s->budget)
      return fail(VC_ERR_OUT_OF_MEMORY, "lane table of " + std::to_string(need) + " bytes exceeds the budget left");
    std::unique_ptr<LaneTable> t(new LaneTable());
    rc = lane_table_init(s, t.get(), g, lanes);
    if (rc != VC_OK) {
      lane_table_free(t.get());
      return rc;
    }
    s->reserved += t->bytes;
    t->th = std::thread(lane_main, s, t.get());
    e.lanes = std::move(t);
  }
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
  const bool lane = ge.lanes && (req->program == VC_CC_HASHMIN || req->program == VC_SSSP);
  if (lane)
    ge.lanes->queue.push_back(j);
  else
    s->queue.push_back(j);
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
  for (GraphEntry& e : s->graphs)
    if (e.lanes && e.lanes->th.joinable()) e.lanes->th.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  for (auto& w : s->workers)
    if (w->stream) (void)hipStreamDestroy(w->stream);
  for (GraphEntry& e : s->graphs)
    if (e.lanes) lane_table_free(e.lanes.get());
  (void)hipSetDevice(prev);
  delete s;
  return VC_OK;
}

}  // extern "C"

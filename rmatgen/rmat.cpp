// Seeded synthetic graph inputs: an R-MAT edge sampler and a CSR builder.
//
// This module produces INPUTS only.  It is shared by the CPU oracle and the
// GPU path and holds none of the vertex-centric method's arithmetic (no
// messages, no combiners, no supersteps).
//
// R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each sampled edge descends
// `scale` levels of the adjacency matrix, most significant bit first; at every
// level it picks one quadrant with probabilities a (src bit 0, dst bit 0),
// b (0,1), c (1,0), d = 1-a-b-c (1,1).  No noise and no vertex relabelling are
// applied, so low-popcount ids (vertex 0 first) are the hubs.
//
// Randomness is counter based: draw j of a stream keyed by `seed` is
// splitmix64_mix(key + (j+1) * GAMMA), i.e. the j-th output of Steele, Lea and
// Flood's SplitMix64 generator (OOPSLA 2014) started at state `key`.  Every
// sample is a pure function of (seed, sample index), so the graph does not
// depend on the number of threads.
//
// CSR build: self-loops are dropped, every adjacency list is sorted and
// de-duplicated; for an undirected graph both directions of every sample are
// inserted before de-duplication (so the result is symmetric).  Optional edge
// weights are 1 + (draw k of the weight stream mod 255) for edge k in final
// CSR order, i.e. uniform on [1, 255].
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t draw(uint64_t key, uint64_t j) { return mix64(key + (j + 1) * GAMMA); }

struct Sampler {
  int scale;
  uint64_t key;
  uint32_t ta, tab, tabc;  // cumulative quadrant thresholds on a 32-bit uniform
  int draws_per_sample;    // two 32-bit uniforms per 64-bit draw

  void sample(uint64_t i, uint32_t* src, uint32_t* dst) const {
    uint32_t s = 0, d = 0;
    uint64_t r = 0;
    for (int l = 0; l < scale; ++l) {
      uint32_t u;
      if ((l & 1) == 0) {
        r = draw(key, i * (uint64_t)draws_per_sample + (uint64_t)(l >> 1));
        u = (uint32_t)r;
      } else {
        u = (uint32_t)(r >> 32);
      }
      uint32_t sb, db;
      if (u < ta) { sb = 0; db = 0; }
      else if (u < tab) { sb = 0; db = 1; }
      else if (u < tabc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    *src = s;
    *dst = d;
  }
};

uint32_t threshold(double p) {
  double t = p * 4294967296.0;
  if (t <= 0.0) return 0;
  if (t >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)t;
}

struct Csr {
  int64_t n = 0, m = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> dst;
  std::vector<uint32_t> w;
};

// Builds a CSR from `count` samples produced by `gen(i, &s, &d)`.
template <class Gen>
int build_csr(int64_t n, uint64_t count, bool directed, Gen gen, Csr* out) {
  // Pass 1: per-source insertion counts (both directions when undirected).
  std::vector<uint32_t> cnt((size_t)n, 0u);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    uint32_t s, d;
    gen((uint64_t)i, &s, &d);
    if (s == d) continue;
    __atomic_fetch_add(&cnt[s], 1u, __ATOMIC_RELAXED);
    if (!directed) __atomic_fetch_add(&cnt[d], 1u, __ATOMIC_RELAXED);
  }
  std::vector<int64_t> start((size_t)n + 1);
  start[0] = 0;
  for (int64_t v = 0; v < n; ++v) start[v + 1] = start[v] + cnt[v];
  const int64_t raw = start[n];
  // Pass 2: regenerate the samples and place them in their source's bucket.
  std::vector<int32_t> tmp;
  try { tmp.resize((size_t)raw); } catch (...) { return -2; }
  std::vector<int64_t> cur(start.begin(), start.end() - 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    uint32_t s, d;
    gen((uint64_t)i, &s, &d);
    if (s == d) continue;
    int64_t p = __atomic_fetch_add(&cur[s], (int64_t)1, __ATOMIC_RELAXED);
    tmp[(size_t)p] = (int32_t)d;
    if (!directed) {
      int64_t q = __atomic_fetch_add(&cur[d], (int64_t)1, __ATOMIC_RELAXED);
      tmp[(size_t)q] = (int32_t)s;
    }
  }
  cur.clear();
  cur.shrink_to_fit();
  // Sort + de-duplicate every bucket; the bucket order within is irrelevant
  // afterwards, so the result is deterministic.
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* b = tmp.data() + start[v];
    int32_t* e = tmp.data() + start[v + 1];
    std::sort(b, e);
    cnt[v] = (uint32_t)(std::unique(b, e) - b);
  }
  out->n = n;
  out->off.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) out->off[v + 1] = out->off[v] + cnt[v];
  out->m = out->off[n];
  try { out->dst.resize((size_t)out->m); } catch (...) { return -2; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v) {
    std::memcpy(out->dst.data() + out->off[v], tmp.data() + start[v], sizeof(int32_t) * cnt[v]);
  }
  return 0;
}

void add_weights(Csr* g, uint64_t wseed) {
  const uint64_t key = mix64(wseed ^ 0x5745494748545321ull);
  g->w.resize((size_t)g->m);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < g->m; ++k) g->w[(size_t)k] = 1u + (uint32_t)(draw(key, (uint64_t)k) % 255u);
}

}  // namespace

extern "C" {

// Opaque handle to a generated CSR kept in host memory until rmat_free.
typedef struct rmat_graph_s rmat_graph;
struct rmat_graph_s {
  Csr csr;
  int weighted = 0;
};

// Generates an R-MAT graph with 2^scale vertices from edge_factor * 2^scale
// samples.  Returns NULL on invalid arguments or allocation failure.
rmat_graph* rmat_generate(int scale, double edge_factor, double a, double b, double c, uint64_t seed,
                          int directed, int weighted, uint64_t weight_seed, int threads) {
  if (scale < 1 || scale > 30 || edge_factor < 0.0) return nullptr;
  if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0 + 1e-12) return nullptr;
  if (threads > 0) omp_set_num_threads(threads);
  Sampler smp;
  smp.scale = scale;
  smp.key = mix64(seed ^ 0x524D4154474E5230ull);
  smp.ta = threshold(a);
  smp.tab = threshold(a + b);
  smp.tabc = threshold(a + b + c);
  smp.draws_per_sample = (scale + 1) / 2;
  const int64_t n = (int64_t)1 << scale;
  const uint64_t count = (uint64_t)(edge_factor * (double)n + 0.5);
  rmat_graph* g = new (std::nothrow) rmat_graph();
  if (!g) return nullptr;
  auto gen = [&smp](uint64_t i, uint32_t* s, uint32_t* d) { smp.sample(i, s, d); };
  if (build_csr(n, count, directed != 0, gen, &g->csr) != 0) {
    delete g;
    return nullptr;
  }
  if (weighted) add_weights(&g->csr, weight_seed);
  g->weighted = weighted != 0;
  return g;
}

// Builds a CSR from an explicit edge list (the same self-loop removal, sort
// and de-duplication as rmat_generate).  Used for small hand-shaped graphs.
rmat_graph* rmat_from_edges(int64_t n, int64_t count, const int64_t* src, const int64_t* dst, int directed,
                            int weighted, uint64_t weight_seed) {
  if (n <= 0 || n > ((int64_t)1 << 31) - 1 || count < 0) return nullptr;
  for (int64_t i = 0; i < count; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return nullptr;
  rmat_graph* g = new (std::nothrow) rmat_graph();
  if (!g) return nullptr;
  auto gen = [src, dst](uint64_t i, uint32_t* s, uint32_t* d) {
    *s = (uint32_t)src[i];
    *d = (uint32_t)dst[i];
  };
  if (build_csr(n, (uint64_t)count, directed != 0, gen, &g->csr) != 0) {
    delete g;
    return nullptr;
  }
  if (weighted) add_weights(&g->csr, weight_seed);
  g->weighted = weighted != 0;
  return g;
}

int64_t rmat_num_vertices(const rmat_graph* g) { return g->csr.n; }
int64_t rmat_num_edges(const rmat_graph* g) { return g->csr.m; }
int rmat_has_weights(const rmat_graph* g) { return g->weighted; }

// Copies the CSR out: off[n+1] as int64 (or int32 when off32 != NULL and
// m < 2^31), dst[m], and w[m] when weights were generated and w != NULL.
int rmat_copy_out(const rmat_graph* g, int64_t* off64, int32_t* off32, int32_t* dst, uint32_t* w) {
  const Csr& c = g->csr;
  if (off64) std::memcpy(off64, c.off.data(), sizeof(int64_t) * (size_t)(c.n + 1));
  if (off32) {
    if (c.m >= ((int64_t)1 << 31)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v <= c.n; ++v) off32[v] = (int32_t)c.off[(size_t)v];
  }
  if (dst) {
    const int64_t chunk = 1 << 22;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < c.m; b += chunk) {
      const int64_t e = std::min(c.m, b + chunk);
      std::memcpy(dst + b, c.dst.data() + b, sizeof(int32_t) * (size_t)(e - b));
    }
  }
  if (w) {
    if (c.w.size() != (size_t)c.m) return -2;
    const int64_t chunk = 1 << 22;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < c.m; b += chunk) {
      const int64_t e = std::min(c.m, b + chunk);
      std::memcpy(w + b, c.w.data() + b, sizeof(uint32_t) * (size_t)(e - b));
    }
  }
  return 0;
}

void rmat_free(rmat_graph* g) { delete g; }

// Raw sampler access for tests of the sampling distribution: writes the
// (src, dst) pair of samples [first, first + count) before any clean-up.
void rmat_samples(int scale, double a, double b, double c, uint64_t seed, uint64_t first, uint64_t count,
                  uint32_t* src, uint32_t* dst) {
  Sampler smp;
  smp.scale = scale;
  smp.key = mix64(seed ^ 0x524D4154474E5230ull);
  smp.ta = threshold(a);
  smp.tab = threshold(a + b);
  smp.tabc = threshold(a + b + c);
  smp.draws_per_sample = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)count; ++i) smp.sample(first + (uint64_t)i, &src[i], &dst[i]);
}

}  // extern "C"

/*
 * Sequential CPU oracle of the vertex-centric (Pregel) superstep.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or helper with the GPU library; it is deliberately plain and slow:
 * one thread, one vertex at a time, in ascending id order.
 *
 * Execution model (paper, Section I): every vertex starts active; in each
 * superstep a user function runs once on every active vertex; it may send
 * messages along its out-edges and may vote to halt; messages sent in
 * superstep s are delivered at superstep s+1, where receiving a message
 * re-activates a halted vertex; execution ends when every vertex has halted
 * and no message is in flight.
 *
 * Mailboxes (paper, Section III): each vertex keeps the message for the next
 * superstep together with an explicit "has a message" flag.  The first
 * message that reaches a mailbox is stored as is; every later one is merged
 * into it with the program's combiner (sum for PageRank, min for hash-min
 * connected components and SSSP).  Because the flag is explicit, no neutral
 * value is ever assumed, which is what lets this oracle check the GPU path's
 * neutral-value mailboxes independently (paper, Section III, on the
 * empty-mailbox ambiguity of compare-and-swap combiners).
 *
 * Programs (paper, Section VI-C, "Benchmarks"):
 *   PageRank  rank^(0) = 1/N; for s = 1..T: rank = (1-d)/N + d * (sum of the
 *             messages received); a vertex with out-degree k > 0 sends
 *             rank/k to each out-neighbour for s < T; a vertex with no
 *             out-edge sends nothing, so its mass is dropped.  The result is
 *             rank after superstep T (T rank updates).
 *   PPR       as PageRank with the teleport restricted to one source:
 *             rank^(0) = [v == src], rank = (1-d)*[v == src] + d * sum.
 *   CC        hash-min label propagation: label^(0) = v and every vertex
 *             sends its label; afterwards a vertex whose smallest received
 *             label is below its own adopts it and sends it on; all vote to
 *             halt after computing.
 *   SSSP      dist^(0) = 0 at the source and "unreached" elsewhere; the
 *             source sends dist + w(e) along each out-edge e; afterwards a
 *             vertex whose smallest received distance is below its own adopts
 *             it and sends dist + w(e) along each out-edge; all halt.  With no
 *             weight array every edge weighs 1 (the paper's unweighted SSSP).
 *
 * Arithmetic: PageRank and PPR in IEEE binary64; labels and distances in
 * uint64, with UINT64_MAX as "unreached" while running.  The result of CC and
 * SSSP is returned as uint32 with 0xFFFFFFFF as "unreached"; a finite distance
 * that does not fit below 0xFFFFFFFF is reported as ORACLE_EOVERFLOW rather
 * than silently truncated.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PAGERANK 0
#define ORACLE_CC 1
#define ORACLE_SSSP 2
#define ORACLE_PPR 3

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)
#define ORACLE_EOVERFLOW (-3)
#define ORACLE_ECAP (-4)

#define UNREACHED_U32 0xFFFFFFFFull /* "unreached" in the uint32 result */
#define INF_U64 UINT64_MAX              /* "unreached" while running */

/* Per-superstep statistics, filled for s = 0 .. supersteps-1. */
typedef struct {
  int64_t senders;   /* vertices that broadcast in superstep s */
  int64_t messages;  /* messages sent in superstep s (out-edges of the senders) */
  int64_t receivers; /* vertices holding at least one message after superstep s */
} oracle_step;

typedef struct {
  /* graph (CSR, out-edges) */
  int64_t n;
  const int64_t* off;
  const int32_t* dst;
  const uint32_t* w;
  /* program and parameters */
  int program;
  int32_t T;
  double d;
  int64_t src;
  /* vertex values */
  double* rank;
  uint64_t* label;
  unsigned char* halted;
  /* mailboxes: message + explicit flag, for this superstep and the next */
  double* fmsg_cur;
  double* fmsg_next;
  uint64_t* umsg_cur;
  uint64_t* umsg_next;
  unsigned char* has_cur;
  unsigned char* has_next;
  /* counters of the running superstep */
  int64_t senders;
  int64_t messages;
} engine;

/* Delivery with the sum combiner. */
static void deliver_sum(engine* g, int64_t u, double m) {
  if (g->has_next[u]) {
    g->fmsg_next[u] = g->fmsg_next[u] + m;
  } else {
    g->fmsg_next[u] = m;
    g->has_next[u] = 1;
  }
}

/* Delivery with the min combiner. */
static void deliver_min(engine* g, int64_t u, uint64_t m) {
  if (g->has_next[u]) {
    if (m < g->umsg_next[u]) g->umsg_next[u] = m;
  } else {
    g->umsg_next[u] = m;
    g->has_next[u] = 1;
  }
}

/* Sends the same floating-point message to every out-neighbour of v. */
static void broadcast_sum(engine* g, int64_t v, double m) {
  g->senders++;
  for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
    deliver_sum(g, g->dst[e], m);
    g->messages++;
  }
}

/* Sends the same integer message to every out-neighbour of v. */
static void broadcast_min(engine* g, int64_t v, uint64_t m) {
  g->senders++;
  for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
    deliver_min(g, g->dst[e], m);
    g->messages++;
  }
}

/* Sends base + w(e) along every out-edge e of v (unit weights when absent). */
static void broadcast_dist(engine* g, int64_t v, uint64_t base) {
  g->senders++;
  for (int64_t e = g->off[v]; e < g->off[v + 1]; ++e) {
    uint64_t we = g->w ? (uint64_t)g->w[e] : 1u;
    deliver_min(g, g->dst[e], base + we);
    g->messages++;
  }
}

static void compute_rank(engine* g, int64_t v, int64_t s) {
  const int64_t deg = g->off[v + 1] - g->off[v];
  const int personal = g->program == ORACLE_PPR;
  if (s == 0) {
    g->rank[v] = personal ? (v == g->src ? 1.0 : 0.0) : 1.0 / (double)g->n;
  } else {
    const double sum = g->has_cur[v] ? g->fmsg_cur[v] : 0.0;
    const double teleport = personal ? (v == g->src ? 1.0 - g->d : 0.0) : (1.0 - g->d) / (double)g->n;
    g->rank[v] = teleport + g->d * sum;
  }
  if (s < g->T) {
    if (deg > 0)
      broadcast_sum(g, v, g->rank[v] / (double)deg);
    else
      g->senders++; /* a broadcast over no out-edge: the mass is dropped */
  } else {
    g->halted[v] = 1;
  }
}

static void compute_cc(engine* g, int64_t v, int64_t s) {
  if (s == 0) {
    g->label[v] = (uint64_t)v;
    broadcast_min(g, v, g->label[v]);
  } else if (g->has_cur[v] && g->umsg_cur[v] < g->label[v]) {
    g->label[v] = g->umsg_cur[v];
    broadcast_min(g, v, g->label[v]);
  }
  g->halted[v] = 1;
}

static void compute_sssp(engine* g, int64_t v, int64_t s) {
  if (s == 0) {
    g->label[v] = (v == g->src) ? 0u : INF_U64;
    if (v == g->src) broadcast_dist(g, v, 0u);
  } else if (g->has_cur[v] && g->umsg_cur[v] < g->label[v]) {
    g->label[v] = g->umsg_cur[v];
    broadcast_dist(g, v, g->label[v]);
  }
  g->halted[v] = 1;
}

static void release(engine* g) {
  free(g->rank);
  free(g->label);
  free(g->halted);
  free(g->fmsg_cur);
  free(g->fmsg_next);
  free(g->umsg_cur);
  free(g->umsg_next);
  free(g->has_cur);
  free(g->has_next);
}

/*
 * Runs one program to completion.
 *   off[n+1], dst[m]   CSR out-edges (host memory); w[m] or NULL
 *   T                  PageRank / PPR: number of rank updates (>= 0)
 *   d                  damping factor (PageRank / PPR)
 *   src                SSSP / PPR source vertex
 *   max_supersteps     <= 0 selects T + 1 for PageRank / PPR and n + 1 for
 *                      CC / SSSP, enough for any run
 *   out                double[n] for PageRank / PPR, uint32[n] for CC / SSSP
 *   steps[cap]         per-superstep statistics (may be NULL when cap == 0)
 *   supersteps         number of supersteps executed
 * Returns ORACLE_OK or a negative ORACLE_E* code.
 */
int oracle_run(int program, int64_t n, const int64_t* off, const int32_t* dst, const uint32_t* w, int32_t T,
               double d, int64_t src, int64_t max_supersteps, void* out, oracle_step* steps, int64_t cap,
               int64_t* supersteps) {
  if (n < 0 || !off || !out || !supersteps || (cap > 0 && !steps)) return ORACLE_EINVAL;
  if (program < ORACLE_PAGERANK || program > ORACLE_PPR) return ORACLE_EINVAL;
  if ((program == ORACLE_SSSP || program == ORACLE_PPR) && (src < 0 || src >= n)) return ORACLE_EINVAL;
  if ((program == ORACLE_PAGERANK || program == ORACLE_PPR) && T < 0) return ORACLE_EINVAL;
  if (off[n] > 0 && !dst) return ORACLE_EINVAL;
  const int is_rank = program == ORACLE_PAGERANK || program == ORACLE_PPR;
  engine g;
  memset(&g, 0, sizeof g);
  g.n = n;
  g.off = off;
  g.dst = dst;
  g.w = program == ORACLE_SSSP ? w : NULL;
  g.program = program;
  g.T = T;
  g.d = d;
  g.src = src;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  g.halted = calloc(nn, 1);
  g.has_cur = calloc(nn, 1);
  g.has_next = calloc(nn, 1);
  if (is_rank) {
    g.rank = calloc(nn, sizeof(double));
    g.fmsg_cur = calloc(nn, sizeof(double));
    g.fmsg_next = calloc(nn, sizeof(double));
  } else {
    g.label = calloc(nn, sizeof(uint64_t));
    g.umsg_cur = calloc(nn, sizeof(uint64_t));
    g.umsg_next = calloc(nn, sizeof(uint64_t));
  }
  if (!g.halted || !g.has_cur || !g.has_next || (is_rank && (!g.rank || !g.fmsg_cur || !g.fmsg_next)) ||
      (!is_rank && (!g.label || !g.umsg_cur || !g.umsg_next))) {
    release(&g);
    return ORACLE_ENOMEM;
  }
  /* default cap: PageRank / PPR run exactly T + 1 supersteps; CC / SSSP need at most n + 1 */
  if (max_supersteps <= 0) max_supersteps = is_rank ? (int64_t)T + 1 : n + 1;

  int64_t s = 0;
  for (;; ++s) {
    if (s >= max_supersteps) {
      release(&g);
      *supersteps = s;
      return ORACLE_ECAP;
    }
    g.senders = 0;
    g.messages = 0;
    for (int64_t v = 0; v < n; ++v) {
      if (g.halted[v] && !g.has_cur[v]) continue; /* halted and no message: stays asleep */
      g.halted[v] = 0;                            /* a message re-activates */
      if (is_rank)
        compute_rank(&g, v, s);
      else if (program == ORACLE_CC)
        compute_cc(&g, v, s);
      else
        compute_sssp(&g, v, s);
    }
    /* message exchange: next-superstep mailboxes become current */
    int64_t receivers = 0;
    for (int64_t v = 0; v < n; ++v) receivers += g.has_next[v];
    if (s < cap) {
      steps[s].senders = g.senders;
      steps[s].messages = g.messages;
      steps[s].receivers = receivers;
    }
    if (is_rank) {
      double* t = g.fmsg_cur;
      g.fmsg_cur = g.fmsg_next;
      g.fmsg_next = t;
    } else {
      uint64_t* t = g.umsg_cur;
      g.umsg_cur = g.umsg_next;
      g.umsg_next = t;
    }
    unsigned char* t = g.has_cur;
    g.has_cur = g.has_next;
    g.has_next = t;
    memset(g.has_next, 0, nn);
    int any = 0;
    for (int64_t v = 0; v < n && !any; ++v) any = !g.halted[v] || g.has_cur[v];
    if (!any) break;
  }
  *supersteps = s + 1;

  int status = ORACLE_OK;
  if (is_rank) {
    memcpy(out, g.rank, sizeof(double) * (size_t)n);
  } else {
    uint32_t* o = (uint32_t*)out;
    for (int64_t v = 0; v < n; ++v) {
      if (g.label[v] == INF_U64) {
        o[v] = (uint32_t)UNREACHED_U32;
      } else {
        if (g.label[v] >= UNREACHED_U32) status = ORACLE_EOVERFLOW; /* not representable */
        o[v] = (uint32_t)g.label[v];
      }
    }
  }
  release(&g);
  return status;
}

/*
 * One superstep of message passing with a chosen combiner (paper, Section
 * III, and its hybrid combiner of Figure 1): every active vertex v sends
 * msg[v] along each of its out-edges; v = 0, 1, ... in turn, edges in CSR
 * order.  A receiver's first message is stored as is and its flag set;
 * every later one is merged into the stored message with the combiner.  No
 * neutral value is assumed.  Messages are 8-byte words:
 *   ORACLE_COMBINE_SUM_U64   wrapping sum of uint64
 *   ORACLE_COMBINE_PROD_U64  wrapping product of uint64
 *   ORACLE_COMBINE_MAX_F64   maximum of binary64 (inputs without NaN)
 *   ORACLE_COMBINE_MINARG    pair (value: binary32 in the low word, id:
 *                            uint32 in the high word); the smaller value
 *                            wins, equal values go to the smaller id
 *                            (inputs without NaN)
 *   ORACLE_COMBINE_SUM_F64   binary64 sum, added in the order above
 * active may be NULL (every vertex sends).  Results: mailbox[u] (undefined
 * where has[u] == 0) and has[u] in {0, 1}.
 */
#define ORACLE_COMBINE_SUM_U64 0
#define ORACLE_COMBINE_PROD_U64 1
#define ORACLE_COMBINE_MAX_F64 2
#define ORACLE_COMBINE_MINARG 3
#define ORACLE_COMBINE_SUM_F64 4

static double word_f64(uint64_t x) {
  double d;
  memcpy(&d, &x, sizeof d);
  return d;
}

static uint64_t f64_word(double d) {
  uint64_t x;
  memcpy(&x, &d, sizeof x);
  return x;
}

static float word_f32_lo(uint64_t x) {
  uint32_t lo = (uint32_t)(x & 0xFFFFFFFFu);
  float f;
  memcpy(&f, &lo, sizeof f);
  return f;
}

static uint64_t combine_words(int op, uint64_t stored, uint64_t msg) {
  switch (op) {
    case ORACLE_COMBINE_SUM_U64: return stored + msg;
    case ORACLE_COMBINE_PROD_U64: return stored * msg;
    case ORACLE_COMBINE_MAX_F64: return word_f64(msg) > word_f64(stored) ? msg : stored;
    case ORACLE_COMBINE_MINARG: {
      const float a = word_f32_lo(stored), b = word_f32_lo(msg);
      const uint32_t ia = (uint32_t)(stored >> 32), ib = (uint32_t)(msg >> 32);
      return (b < a || (b == a && ib < ia)) ? msg : stored;
    }
    default: return f64_word(word_f64(stored) + word_f64(msg));
  }
}

int oracle_combine(int op, int64_t n, const int64_t* off, const int32_t* dst, const uint64_t* msg,
                   const uint8_t* active, uint64_t* mailbox, uint8_t* has) {
  if (op < ORACLE_COMBINE_SUM_U64 || op > ORACLE_COMBINE_SUM_F64) return ORACLE_EINVAL;
  if (n < 0 || !off || !msg || !mailbox || !has || off[0] != 0) return ORACLE_EINVAL;
  for (int64_t v = 0; v < n; ++v) {
    if (off[v + 1] < off[v]) return ORACLE_EINVAL;
  }
  if (off[n] > 0 && !dst) return ORACLE_EINVAL;
  for (int64_t e = 0; e < off[n]; ++e) {
    if (dst[e] < 0 || dst[e] >= n) return ORACLE_EINVAL;
  }
  for (int64_t u = 0; u < n; ++u) {
    has[u] = 0;
    mailbox[u] = 0;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (active && !active[v]) continue;
    for (int64_t e = off[v]; e < off[v + 1]; ++e) {
      const int64_t u = dst[e];
      if (!has[u]) {
        mailbox[u] = msg[v]; /* first message: stored, flag set */
        has[u] = 1;
      } else {
        mailbox[u] = combine_words(op, mailbox[u], msg[v]);
      }
    }
  }
  return ORACLE_OK;
}

/* Library version tag, so a stale build is detected by its loader. */
int oracle_version(void) { return 2; }

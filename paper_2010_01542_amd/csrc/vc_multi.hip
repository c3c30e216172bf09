// Many min-plus programs on one graph in one superstep loop.
//
// Up to 256 lanes (SSSP sources, or the requests of a server lane table)
// run side by side, one wavefront lane each, in cs chunks of 64 lanes.
// Values, mailboxes and per-vertex active masks are chunk-major: chunk c of
// vertex v sits at c * n + v (a value row holds the chunk's 64 lanes, 256
// bytes), so loops over the first ceff chunks touch array prefixes only.
// Each superstep applies the min combiner (paper, Section III) to all lanes
// at once, either in the pull form (paper, Section VI-C: a receiver's row
// takes, lane by lane, the minimum of dist(u) + w(u, v) over in-neighbours u
// whose lane improved in the previous superstep) or, when few vertices are
// active, in the push form (each active vertex broadcasts along its
// out-edges, paper, Section I).  Every lane of a wavefront handles the same
// edge, so row loads are coalesced.  Values and mailboxes are separate
// arrays, so the superstep stays bulk-synchronous.
//
// A lane may run hash-min CC instead of SSSP (paper, Section VI: CC is the
// min combiner over labels with no edge cost): its column starts at the
// vertex labels with every vertex active, and a per-lane mask zeroes the
// edge weight.
#include "vc_device.h"
#include "vc_graph.h"

namespace vc {
namespace {

using namespace dev;


// Row of chunk c of vertex v in a chunk-major value array.
__device__ __forceinline__ int64_t row(int c, int64_t n, int64_t v) { return ((int64_t)c * n + v) * 64; }

// Source k (internal id src[k]) starts at distance 0 with lane k active.
__global__ void k_ms_seed(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int k_real, int64_t n,
                          uint32_t* __restrict__ D, uint16_t* __restrict__ D16, unsigned long long* __restrict__ A,
                          uint32_t* __restrict__ bits) {
  const int k = threadIdx.x + blockIdx.x * blockDim.x;
  if (k >= k_real) return;
  const int64_t x = perm ? (int64_t)perm[src[k]] : (int64_t)src[k];
  D[row(k >> 6, n, x) + (k & 63)] = 0u;
  if (D16) D16[row(k >> 6, n, x) + (k & 63)] = 0;
  atomicOr(&A[(int64_t)(k >> 6) * n + x], 1ull << (k & 63));
  atomicOr(&bits[x >> 5], 1u << (x & 31));
}

// Pull: per receiver v and lane, best = min over in-neighbours of D[u] + w;
// written to the mailbox when it beats the current value.  One wavefront
// per chunk walks the tile's in-edges.  Every in-neighbour is read, active
// or not: an inactive u's value has not changed since it last sent, and
// that message already took each receiver's value to D[u] + w or lower,
// so sending it again improves nothing and every superstep's outcome is
// the one the active senders alone give.  Skipping the per-edge load of
// u's active mask (a random 8-byte read, a whole line) saves more than the
// rows of inactive lanes cost (dense superstep 16.7 -> 11.6 ms, 256 lanes,
// scale 22).  Lanes without a program hold the unreached value everywhere.
template <int C, bool WEIGHTED>
__global__ __launch_bounds__(64 * C) void k_ms_pull(const int64_t* __restrict__ in_off,
                                                    const int32_t* __restrict__ in_src,
                                                    const uint32_t* __restrict__ in_w, int64_t n, int64_t m,
                                                    const int32_t* __restrict__ tile_v, int64_t tile,
                                                    const uint32_t* __restrict__ D, uint32_t* __restrict__ MB,
                                                    uint32_t* __restrict__ improved, LaneMask zero) {
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  Tile tl;
  if (!tile_bounds(tile_v, tile, n, m, &tl)) return;
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);
  for (int x = threadIdx.x; x <= tl.cnt; x += 64 * C) s_off[x] = in_off[tl.i0 + x];
  __syncthreads();
  const int c = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool zero_w = (zero.bits[c] >> lane) & 1ull;  // CC lane: labels travel without cost
  const uint32_t* Dc = D + row(c, n, 0) + lane;
  int x = owner_of(s_off, tl.cnt, tl.j0);
  int64_t next = s_off[x + 1];
  uint32_t run = kInf;
  auto flush = [&](int xo, uint32_t best) {
    const int64_t v = tl.i0 + xo;
    bool imp = false;
    if (best != kInf) {
      const int64_t idx = row(c, n, v) + lane;
      if (best < D[idx]) {
        if (s_off[xo] >= tl.j0 && s_off[xo + 1] <= tl.j1) {
          MB[idx] = best;  // every in-edge of v is in this tile
          imp = true;
        } else if (best < MB[idx]) {
          atomicMin(&MB[idx], best);
          imp = true;
        }
      }
    }
    if (__ballot(imp) && lane == 0) atomicOr(&improved[v >> 5], 1u << (v & 31));
  };
  for (int64_t e0 = tl.j0; e0 < tl.j1; e0 += U) {
    int32_t u[U];
    uint32_t val[U], wv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) u[k] = e0 + k < tl.j1 ? in_src[e0 + k] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      wv[k] = (WEIGHTED && e0 + k < tl.j1) ? in_w[e0 + k] : 1u;
      val[k] = e0 + k < tl.j1 ? Dc[(int64_t)u[k] * 64] : kInf;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t e = e0 + k;
      if (e < tl.j1) {
        while (e >= next) {  // receiver changes (uniform over the wavefront)
          flush(x, run);
          run = kInf;
          ++x;
          next = s_off[x + 1];
        }
        if (val[k] != kInf) {
          const uint32_t cand = zero_w ? val[k] : sat_add(val[k], wv[k]);
          run = cand < run ? cand : run;
        }
      }
    }
  }
  flush(x, run);
}

// 2-byte copies of R consecutive lane values, and 4-byte lane values, as
// one load each (R = 1, 2, 4).
template <int R>
struct LanePart;
template <>
struct LanePart<1> {
  using T16 = uint16_t;
  using T32 = uint32_t;
  __device__ __forceinline__ static uint32_t h(const T16& x, int) { return x; }
  __device__ __forceinline__ static uint32_t w(const T32& x, int) { return x; }
  __device__ __forceinline__ static void setw(T32& x, int, uint32_t v) { x = v; }
};
template <>
struct LanePart<2> {
  using T16 = uint32_t;
  using T32 = uint2;
  __device__ __forceinline__ static uint32_t h(const T16& x, int j) { return j ? x >> 16 : x & 0xFFFFu; }
  __device__ __forceinline__ static uint32_t w(const T32& x, int j) { return j ? x.y : x.x; }
  __device__ __forceinline__ static void setw(T32& x, int j, uint32_t v) {
    if (j) x.y = v; else x.x = v;
  }
};
template <>
struct LanePart<4> {
  using T16 = uint2;
  using T32 = uint4;
  __device__ __forceinline__ static uint32_t h(const T16& x, int j) {
    const uint32_t q = j < 2 ? x.x : x.y;
    return (j & 1) ? q >> 16 : q & 0xFFFFu;
  }
  __device__ __forceinline__ static uint32_t w(const T32& x, int j) {
    return j == 0 ? x.x : j == 1 ? x.y : j == 2 ? x.z : x.w;
  }
  __device__ __forceinline__ static void setw(T32& x, int j, uint32_t v) {
    if (j == 0) x.x = v; else if (j == 1) x.y = v; else if (j == 2) x.z = v; else x.w = v;
  }
};

// Pull from the 2-byte copy D16 of the lane values (every value below
// 0xFFFF, which stands for unreached; the host uses this form only while
// no distance can reach it).  One wavefront per tile covers every chunk:
// chunk r's row is read by lanes r * 64 / R .. (r + 1) * 64 / R - 1, R
// values each, so one load instruction per in-edge brings the 2-byte rows
// of all R chunks (R = 4: 8 bytes per lane, 512 bytes per edge).  A row
// gather is bounded by the load pipeline's bytes per instruction, not by
// HBM (the 4-byte rows: 11 % L2 hits and ~7 TB/s from the memory side at
// 69 % texture-addresser busy), so half the bytes per edge is the point.
// Receivers are compared with, and written to, the 4-byte D and MB as in
// k_ms_pull.  Chunks at or past ceff are left alone.
template <int R, bool WEIGHTED>
__global__ __launch_bounds__(64) void k_ms_pull16(const int64_t* __restrict__ in_off,
                                                  const int32_t* __restrict__ in_src,
                                                  const uint32_t* __restrict__ in_w, int64_t n, int64_t m,
                                                  const int32_t* __restrict__ tile_v, int64_t tile,
                                                  const uint16_t* __restrict__ D16, const uint32_t* __restrict__ D,
                                                  uint32_t* __restrict__ MB, uint32_t* __restrict__ improved,
                                                  LaneMask zero, int ceff) {
  using P = LanePart<R>;
  using T16 = typename P::T16;
  using T32 = typename P::T32;
  constexpr int L = 64 / R;  // lanes per row
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  Tile tl;
  if (!tile_bounds(tile_v, tile, n, m, &tl)) return;
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);
  for (int x = threadIdx.x; x <= tl.cnt; x += 64) s_off[x] = in_off[tl.i0 + x];
  __syncthreads();
  const int lane = threadIdx.x;
  const int r = lane / L, q = lane % L;
  const bool on = r < ceff;
  const int rr = on ? r : 0;  // rows past ceff read chunk 0 (in bounds) and are never used
  unsigned zmask = 0;         // values of this lane that travel without cost (CC lanes)
#pragma unroll
  for (int j = 0; j < R; ++j) zmask |= (unsigned)((zero.bits[rr] >> (q * R + j)) & 1ull) << j;
  const T16* Hr = reinterpret_cast<const T16*>(D16 + row(rr, n, 0)) + q;
  const T32* Dr = reinterpret_cast<const T32*>(D + row(rr, n, 0)) + q;
  T32* MBr = reinterpret_cast<T32*>(MB + row(rr, n, 0)) + q;
  int x = owner_of(s_off, tl.cnt, tl.j0);
  int64_t next = s_off[x + 1];
  uint32_t run[R];
#pragma unroll
  for (int j = 0; j < R; ++j) run[j] = kInf;
  auto flush = [&](int xo) {  // uniform over the wavefront
    const int64_t v = tl.i0 + xo;
    bool any = false;
#pragma unroll
    for (int j = 0; j < R; ++j) any |= run[j] != kInf;
    bool imp = false;
    if (on && any) {
      const T32 d = Dr[v * L];
      if (s_off[xo] >= tl.j0 && s_off[xo + 1] <= tl.j1) {  // every in-edge of v is in this tile
        T32 nb = d;
        bool lowered = false;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const bool lower = run[j] < P::w(d, j);
          P::setw(nb, j, lower ? run[j] : kInf);  // the mailbox was empty
          lowered |= lower;
        }
        if (lowered) {
          MBr[v * L] = nb;
          imp = true;
        }
      } else {
        const T32 mb = MBr[v * L];
        uint32_t* mp = reinterpret_cast<uint32_t*>(MBr + v * L);
#pragma unroll
        for (int j = 0; j < R; ++j)
          if (run[j] < P::w(d, j) && run[j] < P::w(mb, j)) {
            atomicMin(mp + j, run[j]);
            imp = true;
          }
      }
    }
    if (__ballot(imp) && lane == 0) atomicOr(&improved[v >> 5], 1u << (v & 31));
  };
  for (int64_t e0 = tl.j0; e0 < tl.j1; e0 += U) {
    int32_t u[U];
    uint32_t wv[U];
    T16 val[U];
#pragma unroll
    for (int k = 0; k < U; ++k) u[k] = e0 + k < tl.j1 ? in_src[e0 + k] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) {  // unconditional (vertex 0's rows past the end): all loads issue first
      wv[k] = (WEIGHTED && e0 + k < tl.j1) ? in_w[e0 + k] : 1u;
      val[k] = Hr[(int64_t)u[k] * L];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t e = e0 + k;
      if (e < tl.j1) {
        if (e >= next) {  // receiver changes (uniform over the wavefront)
          flush(x);
#pragma unroll
          for (int j = 0; j < R; ++j) run[j] = kInf;
          ++x;
          next = s_off[x + 1];
          while (e >= next) {  // receivers without in-edges here
            ++x;
            next = s_off[x + 1];
          }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t dv = P::h(val[k], j);
          if (dv != 0xFFFFu) {
            const uint32_t cand = ((zmask >> j) & 1u) ? dv : dv + wv[k];
            run[j] = cand < run[j] ? cand : run[j];
          }
        }
      }
    }
  }
  flush(x);
}

// Push: the listed vertices (list[0..items), out-degree prefix P) broadcast
// along their out-edges, lane by lane, with a test-before-atomic min into
// the receiver's mailbox.  Edge-balanced merge-path tiles over (list, P);
// one wavefront per chunk; the loads of U edges are issued together.
template <int C, bool WEIGHTED, class OffT>
__global__ __launch_bounds__(64 * C) void k_ms_push(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                    const uint32_t* __restrict__ w, int64_t n,
                                                    const int32_t* __restrict__ list, const int64_t* __restrict__ P,
                                                    int64_t items, int64_t edges, const int32_t* __restrict__ tile_v,
                                                    int64_t tile, const uint32_t* __restrict__ D,
                                                    uint32_t* __restrict__ MB, const unsigned long long* __restrict__ A,
                                                    uint32_t* __restrict__ improved, LaneMask zero) {
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  Tile tl;
  if (!tile_bounds(tile_v, tile, items, edges, &tl)) return;
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);                                      // cnt + 1 <= tile + 2
  int64_t* s_base = reinterpret_cast<int64_t*>(smem + align16((size_t)(tile + 2) * 8));   // cnt <= tile + 1
  int32_t* s_u = reinterpret_cast<int32_t*>(smem + align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8));
  for (int x = threadIdx.x; x <= tl.cnt; x += 64 * C) {
    const int64_t p = P[tl.i0 + x];
    s_off[x] = p;
    if (x < tl.cnt) {
      const int32_t u = list[tl.i0 + x];
      s_u[x] = u;
      s_base[x] = (int64_t)off[u] - p;  // CSR position of the owner's edge e is e + base
    }
  }
  __syncthreads();
  const int c = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool zero_w = (zero.bits[c] >> lane) & 1ull;
  const unsigned long long* Ac = A + (int64_t)c * n;
  const uint32_t* Dc = D + row(c, n, 0) + lane;
  uint32_t* MBc = MB + row(c, n, 0) + lane;
  int x = owner_of(s_off, tl.cnt, tl.j0) - 1;
  int64_t next = tl.j0, base = 0;
  for (int64_t e0 = tl.j0; e0 < tl.j1; e0 += U) {
    int32_t v[U], u[U];
    uint32_t wv[U], du[U], dv[U], mv[U];
    int64_t eb[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {  // owners of the next U edges (uniform over the wavefront)
      const int64_t e = e0 + k;
      while (e < tl.j1 && e >= next) {
        ++x;
        next = s_off[x + 1];
        base = s_base[x];
      }
      u[k] = s_u[x < 0 ? 0 : x];
      eb[k] = e + base;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = e0 + k < tl.j1 ? dst[eb[k]] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) wv[k] = (WEIGHTED && e0 + k < tl.j1) ? w[eb[k]] : 1u;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const unsigned long long msk = e0 + k < tl.j1 ? Ac[u[k]] : 0ull;
      du[k] = ((msk >> lane) & 1ull) ? Dc[(int64_t)u[k] * 64] : kInf;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      dv[k] = du[k] != kInf ? Dc[(int64_t)v[k] * 64] : 0u;
      mv[k] = du[k] != kInf ? MBc[(int64_t)v[k] * 64] : 0u;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (e0 + k < tl.j1) {
        bool imp = false;
        if (du[k] != kInf) {
          const uint32_t cand = zero_w ? du[k] : sat_add(du[k], wv[k]);
          if (cand < dv[k] && cand < mv[k]) {
            atomicMin(&MBc[(int64_t)v[k] * 64], cand);
            imp = true;
          }
        }
        if (__ballot(imp) && lane == 0) atomicOr(&improved[v[k] >> 5], 1u << (v[k] & 31));
      }
    }
  }
}

// For every improved vertex (one workgroup of four wavefronts per bitmap
// word, each taking (vertex, chunk) pairs in turn): adopt the mailbox lane
// by lane, reset it, record the improved lanes as the vertex's active mask
// for the next superstep, and count |F| and E.  A vertex without out-edges
// keeps an empty mask: it has nobody to broadcast to.  live (may be NULL)
// collects the OR of all masks, spread over 64 words per chunk (stride cs)
// to keep same-address atomics rare: a lane is live while a word holds its
// bit.
template <int C, class OffT>
__global__ __launch_bounds__(kWG) void k_ms_apply(const OffT* __restrict__ off, int64_t n, int64_t nwords, int cs,
                                                  uint32_t* __restrict__ D, uint16_t* __restrict__ D16,
                                                  uint32_t* __restrict__ MB,
                                                  unsigned long long* __restrict__ A_next,
                                                  uint32_t* __restrict__ improved, Counters* __restrict__ ctr,
                                                  unsigned long long* __restrict__ live) {
  const int64_t wi = blockIdx.x;
  if (wi >= nwords) return;
  const uint32_t word = improved[wi];
  if (!word) return;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int cnt = __popc(word);
  unsigned long long any[C];
#pragma unroll
  for (int q = 0; q < C; ++q) any[q] = 0;
  for (int t = wave; t < cnt * C; t += kWG / 64) {
    const int j = t / C, c = t - j * C;
    uint32_t b = word;
    for (int q = 0; q < j; ++q) b &= b - 1;  // j-th set bit
    const int64_t v = wi * 32 + (__ffs(b) - 1);
    const int64_t idx = row(c, n, v) + lane;
    const uint32_t mb = MB[idx];
    const bool act = mb < D[idx];
    if (act) {
      D[idx] = mb;
      if (D16) D16[idx] = (uint16_t)(mb < 0xFFFFu ? mb : 0xFFFFu);
    }
    if (mb != kInf) MB[idx] = kInf;
    const bool sends = off[v + 1] > off[v];
    const unsigned long long mask = sends ? __ballot(act) : 0ull;
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (q == c) any[q] |= mask;
    if (lane == 0) A_next[(int64_t)c * n + v] = mask;
  }
  if (live && lane == 0) {
#pragma unroll
    for (int q = 0; q < C; ++q)
      if (any[q]) atomicOr(&live[(wi & 63) * cs + q], any[q]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long edges = 0;
    for (uint32_t bits = word; bits; bits &= bits - 1) {
      const int64_t v = wi * 32 + (__ffs(bits) - 1);
      edges += (unsigned long long)((int64_t)off[v + 1] - (int64_t)off[v]);
    }
    atomicAdd(&ctr->active, (unsigned long long)cnt);
    if (edges) atomicAdd(&ctr->edges, edges);
    improved[wi] = 0;
  }
}

// Broadcast list of a push superstep: every vertex with an active lane in
// the first ceff chunks, with its out-degree (the prefix is scanned after).
// ctr->listed / ctr->edges receive the list length and its out-edges.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_ms_compact(const OffT* __restrict__ off,
                                                    const unsigned long long* __restrict__ A, int64_t n, int ceff,
                                                    int32_t* __restrict__ list, int64_t* __restrict__ P,
                                                    Counters* __restrict__ ctr) {
  const int64_t x = gid();
  bool act = false;
  int64_t deg = 0;
  if (x < n) {
    for (int c = 0; c < ceff; ++c) act |= A[(int64_t)c * n + x] != 0ull;
    if (act) deg = (int64_t)off[x + 1] - (int64_t)off[x];
  }
  const unsigned long long b = __ballot(act);
  const unsigned lane = lane_id();
  unsigned long long pos = 0;
  if (lane == 0 && b) pos = atomicAdd(&ctr->listed, (unsigned long long)__popcll(b));
  pos = __shfl(pos, 0, 64);
  if (act) {
    const unsigned long long at = pos + __popcll(b & ((1ull << lane) - 1ull));
    list[at] = (int32_t)x;
    P[at] = deg;
  }
  const unsigned long long e = block_sum<unsigned long long>((unsigned long long)deg);
  if (threadIdx.x == 0 && e) atomicAdd(&ctr->edges, e);
}

// |F_0|, E_0 of the seeded sources (bitmap left in place for the first pull).
template <class OffT>
__global__ __launch_bounds__(kWG) void k_ms_count(const OffT* __restrict__ off, const uint32_t* __restrict__ bits,
                                                  int64_t nwords, Counters* __restrict__ ctr) {
  const int64_t wi = gid();
  unsigned long long active = 0, edges = 0;
  if (wi < nwords) {
    const uint32_t word = bits[wi];
    active = __popc(word);
    for (uint32_t b = word; b; b &= b - 1) {
      const int64_t v = wi * 32 + (__ffs(b) - 1);
      edges += (unsigned long long)((int64_t)off[v + 1] - (int64_t)off[v]);
    }
  }
  active = block_sum<unsigned long long>(active);
  edges = block_sum<unsigned long long>(edges);
  if (threadIdx.x == 0) {
    if (active) atomicAdd(&ctr->active, active);
    if (edges) atomicAdd(&ctr->edges, edges);
  }
}

// out[v * k_real + k] = value of lane k at perm[v]
__global__ __launch_bounds__(kWG) void k_ms_output(const uint32_t* __restrict__ D, const int32_t* __restrict__ perm,
                                                   int64_t n, int k_real, uint32_t* __restrict__ out) {
  for (int64_t i = gid(); i < n * k_real; i += grid_threads()) {
    const int64_t v = i / k_real;
    const int k = (int)(i - v * k_real);
    const int64_t x = perm ? (int64_t)perm[v] : v;
    out[i] = D[row(k >> 6, n, x) + (k & 63)];
  }
}

// Lane seeding, CC: every vertex x takes its label ids[x] (x itself when
// ids is NULL) in each listed lane and is active there if it has out-edges.
// One thread per vertex, so the mask update needs no atomic.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_lane_seed_cc(const OffT* __restrict__ off, const int32_t* __restrict__ ids,
                                                      int64_t n, const int32_t* __restrict__ lanes, int r,
                                                      uint32_t* __restrict__ D, unsigned long long* __restrict__ A) {
  const int64_t x = gid();
  if (x >= n) return;
  const uint32_t label = ids ? (uint32_t)ids[x] : (uint32_t)x;
  unsigned long long acc[4] = {0, 0, 0, 0};
  for (int j = 0; j < r; ++j) {
    const int l = lanes[j];
    D[row(l >> 6, n, x) + (l & 63)] = label;
    acc[l >> 6] |= 1ull << (l & 63);
  }
  if (off[x + 1] > off[x]) {
    for (int c = 0; c < 4; ++c)
      if (acc[c]) A[(int64_t)c * n + x] |= acc[c];
  }
}

// Lane seeding, SSSP: seeds[2j] = lane, seeds[2j + 1] = source (caller's
// id).  The source starts at 0 and is active if it has out-edges; a lane
// whose source has none is flagged in stillborn (it ends after one
// superstep with nothing sent).
template <class OffT>
__global__ __launch_bounds__(kWG) void k_lane_seed_sssp(const OffT* __restrict__ off, const int32_t* __restrict__ perm,
                                                        int64_t n, const int32_t* __restrict__ seeds, int r,
                                                        uint32_t* __restrict__ D, unsigned long long* __restrict__ A,
                                                        unsigned long long* __restrict__ stillborn) {
  const int j = (int)gid();
  if (j >= r) return;
  const int l = seeds[2 * j];
  const int64_t src = seeds[2 * j + 1];
  const int64_t x = perm ? (int64_t)perm[src] : src;
  D[row(l >> 6, n, x) + (l & 63)] = 0u;
  if (off[x + 1] > off[x])
    atomicOr(&A[(int64_t)(l >> 6) * n + x], 1ull << (l & 63));
  else
    atomicOr(&stillborn[l >> 6], 1ull << (l & 63));
}

// Lane retirement: outs[j][v] = value of lane lanes[j] at perm[v], and the
// lane is reset to unreached for its next request.
__global__ __launch_bounds__(kWG) void k_lane_retire(uint32_t* __restrict__ D, const int32_t* __restrict__ perm,
                                                     int64_t n, const int32_t* __restrict__ lanes,
                                                     uint32_t* const* __restrict__ outs, int r) {
  for (int64_t i = gid(); i < n * r; i += grid_threads()) {
    const int64_t v = i / r;
    const int j = (int)(i - v * r);
    const int64_t x = perm ? (int64_t)perm[v] : v;
    const int l = lanes[j];
    const int64_t idx = row(l >> 6, n, x) + (l & 63);
    outs[j][v] = D[idx];
    D[idx] = kInf;
  }
}

// Clears the listed lanes from every active mask of the first cs chunks
// (lanes stopped at their superstep cap while still active).
__global__ __launch_bounds__(kWG) void k_lane_clear(unsigned long long* __restrict__ A, int64_t n, int cs,
                                                    LaneMask drop) {
  for (int64_t i = gid(); i < n * cs; i += grid_threads()) {
    const int c = (int)(i / n);
    if (drop.bits[c]) A[i] &= ~drop.bits[c];
  }
}

size_t push_lds_bytes(int64_t tile) {
  return align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8) + (size_t)(tile + 1) * 4;
}

template <int C>
hipError_t ms_pull_launch(bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                          int64_t n, int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles, const uint32_t* D,
                          uint32_t* MB, uint32_t* improved, const LaneMask& zero, hipStream_t s) {
  const size_t lds = (size_t)(tile + 2) * 8;
  if (weighted)
    hipLaunchKernelGGL((k_ms_pull<C, true>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D, MB, improved, zero);
  else
    hipLaunchKernelGGL((k_ms_pull<C, false>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D, MB, improved, zero);
  return hipGetLastError();
}

template <int C, class OffT>
hipError_t ms_push_launch(bool weighted, const OffT* off, const int32_t* dst, const uint32_t* w, int64_t n,
                          const int32_t* list, const int64_t* P, int64_t items, int64_t edges, const int32_t* tile_v,
                          int64_t tile, int64_t ntiles, const uint32_t* D, uint32_t* MB, const unsigned long long* A,
                          uint32_t* improved, const LaneMask& zero, hipStream_t s) {
  const size_t lds = push_lds_bytes(tile);
  if (weighted)
    hipLaunchKernelGGL((k_ms_push<C, true, OffT>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, off, dst, w, n, list,
                       P, items, edges, tile_v, tile, D, MB, A, improved, zero);
  else
    hipLaunchKernelGGL((k_ms_push<C, false, OffT>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, off, dst, w, n,
                       list, P, items, edges, tile_v, tile, D, MB, A, improved, zero);
  return hipGetLastError();
}

template <int C>
hipError_t ms_apply_launch(const void* off, bool off64, int64_t n, int cs, uint32_t* D, uint16_t* D16, uint32_t* MB,
                           unsigned long long* A_next, uint32_t* improved, Counters* ctr, unsigned long long* live,
                           hipStream_t s) {
  const int64_t nwords = (n + 31) / 32;
  if (off64)
    hipLaunchKernelGGL((k_ms_apply<C, int64_t>), dim3((unsigned)nwords), dim3(kWG), 0, s, (const int64_t*)off, n,
                       nwords, cs, D, D16, MB, A_next, improved, ctr, live);
  else
    hipLaunchKernelGGL((k_ms_apply<C, int32_t>), dim3((unsigned)nwords), dim3(kWG), 0, s, (const int32_t*)off, n,
                       nwords, cs, D, D16, MB, A_next, improved, ctr, live);
  return hipGetLastError();
}

template <int R>
hipError_t ms_pull16_launch(bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                            int64_t n, int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles,
                            const uint16_t* D16, const uint32_t* D, uint32_t* MB, uint32_t* improved,
                            const LaneMask& zero, int ceff, hipStream_t s) {
  const size_t lds = (size_t)(tile + 2) * 8;
  if (weighted)
    hipLaunchKernelGGL((k_ms_pull16<R, true>), dim3((unsigned)ntiles), dim3(64), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D16, D, MB, improved, zero, ceff);
  else
    hipLaunchKernelGGL((k_ms_pull16<R, false>), dim3((unsigned)ntiles), dim3(64), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D16, D, MB, improved, zero, ceff);
  return hipGetLastError();
}

// ceff chunks from the 2-byte copy, R = 1, 2 or 4 values per lane (three
// chunks take the four-chunk layout with its last row idle).
hipError_t launch_ms_pull16(int C, bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                            int64_t n, int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles,
                            const uint16_t* D16, const uint32_t* D, uint32_t* MB, uint32_t* improved,
                            const LaneMask& zero, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (C) {
    case 1: return ms_pull16_launch<1>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D16, D, MB, improved, zero, C, s);
    case 2: return ms_pull16_launch<2>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D16, D, MB, improved, zero, C, s);
    case 3:
    case 4: return ms_pull16_launch<4>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D16, D, MB, improved, zero, C, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ms_pull(int C, bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                          int64_t n, int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles,
                          const uint32_t* D, uint32_t* MB, uint32_t* improved, const LaneMask& zero, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (C) {
    case 1: return ms_pull_launch<1>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, improved, zero, s);
    case 2: return ms_pull_launch<2>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, improved, zero, s);
    case 3: return ms_pull_launch<3>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, improved, zero, s);
    case 4: return ms_pull_launch<4>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, improved, zero, s);
  }
  return hipErrorInvalidValue;
}

template <class OffT>
hipError_t launch_ms_push(int C, bool weighted, const OffT* off, const int32_t* dst, const uint32_t* w, int64_t n,
                          const int32_t* list, const int64_t* P, int64_t items, int64_t edges, const int32_t* tile_v,
                          int64_t tile, int64_t ntiles, const uint32_t* D, uint32_t* MB, const unsigned long long* A,
                          uint32_t* improved, const LaneMask& zero, hipStream_t s) {
  if (ntiles <= 0 || edges <= 0) return hipSuccess;
  switch (C) {
    case 1: return ms_push_launch<1>(weighted, off, dst, w, n, list, P, items, edges, tile_v, tile, ntiles, D, MB, A, improved, zero, s);
    case 2: return ms_push_launch<2>(weighted, off, dst, w, n, list, P, items, edges, tile_v, tile, ntiles, D, MB, A, improved, zero, s);
    case 3: return ms_push_launch<3>(weighted, off, dst, w, n, list, P, items, edges, tile_v, tile, ntiles, D, MB, A, improved, zero, s);
    case 4: return ms_push_launch<4>(weighted, off, dst, w, n, list, P, items, edges, tile_v, tile, ntiles, D, MB, A, improved, zero, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ms_apply(int C, int cs, const void* off, bool off64, int64_t n, uint32_t* D, uint16_t* D16,
                           uint32_t* MB, unsigned long long* A_next, uint32_t* improved, Counters* ctr,
                           unsigned long long* live, hipStream_t s) {
  switch (C) {
    case 1: return ms_apply_launch<1>(off, off64, n, cs, D, D16, MB, A_next, improved, ctr, live, s);
    case 2: return ms_apply_launch<2>(off, off64, n, cs, D, D16, MB, A_next, improved, ctr, live, s);
    case 3: return ms_apply_launch<3>(off, off64, n, cs, D, D16, MB, A_next, improved, ctr, live, s);
    case 4: return ms_apply_launch<4>(off, off64, n, cs, D, D16, MB, A_next, improved, ctr, live, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ms_compact(const void* off, bool off64, const unsigned long long* A, int64_t n, int ceff,
                             int32_t* list, int64_t* P, Counters* ctr, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_ms_compact<int64_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, A, n, ceff,
                       list, P, ctr);
  else
    hipLaunchKernelGGL(k_ms_compact<int32_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, A, n, ceff,
                       list, P, ctr);
  return hipGetLastError();
}

}  // namespace

int ms_chunks(int k) { return (k + 63) / 64; }

hipError_t launch_ms_seed(const int32_t* src, const int32_t* perm, int k_real, int64_t n, uint32_t* D, uint16_t* D16,
                          unsigned long long* A, uint32_t* bits, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_seed, dim3(1), dim3(256), 0, s, src, perm, k_real, n, D, D16, A, bits);
  return hipGetLastError();
}

hipError_t launch_ms_count(const void* off, bool off64, int64_t n, const uint32_t* bits, Counters* ctr,
                           hipStream_t s) {
  const int64_t nwords = (n + 31) / 32;
  if (off64)
    hipLaunchKernelGGL(k_ms_count<int64_t>, dim3(grid_for(nwords)), dim3(kWG), 0, s, (const int64_t*)off, bits, nwords,
                       ctr);
  else
    hipLaunchKernelGGL(k_ms_count<int32_t>, dim3(grid_for(nwords)), dim3(kWG), 0, s, (const int32_t*)off, bits, nwords,
                       ctr);
  return hipGetLastError();
}

hipError_t launch_ms_output(const uint32_t* D, const int32_t* perm, int64_t n, int k_real, uint32_t* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_ms_output, dim3(grid_stride_for(n * k_real)), dim3(kWG), 0, s, D, perm, n, k_real, out);
  return hipGetLastError();
}

hipError_t launch_lane_seed_cc(const void* off, bool off64, const int32_t* ids, int64_t n, const int32_t* lanes,
                               int r, uint32_t* D, unsigned long long* A, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  if (off64)
    hipLaunchKernelGGL(k_lane_seed_cc<int64_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, ids, n, lanes,
                       r, D, A);
  else
    hipLaunchKernelGGL(k_lane_seed_cc<int32_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, ids, n, lanes,
                       r, D, A);
  return hipGetLastError();
}

hipError_t launch_lane_seed_sssp(const void* off, bool off64, const int32_t* perm, int64_t n, const int32_t* seeds,
                                 int r, uint32_t* D, unsigned long long* A, unsigned long long* stillborn,
                                 hipStream_t s) {
  if (r <= 0) return hipSuccess;
  if (off64)
    hipLaunchKernelGGL(k_lane_seed_sssp<int64_t>, dim3(grid_for(r)), dim3(kWG), 0, s, (const int64_t*)off, perm, n,
                       seeds, r, D, A, stillborn);
  else
    hipLaunchKernelGGL(k_lane_seed_sssp<int32_t>, dim3(grid_for(r)), dim3(kWG), 0, s, (const int32_t*)off, perm, n,
                       seeds, r, D, A, stillborn);
  return hipGetLastError();
}

hipError_t launch_lane_retire(uint32_t* D, const int32_t* perm, int64_t n, const int32_t* lanes,
                              uint32_t* const* outs, int r, hipStream_t s) {
  if (r <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lane_retire, dim3(grid_stride_for(n * r)), dim3(kWG), 0, s, D, perm, n, lanes, outs, r);
  return hipGetLastError();
}

hipError_t launch_lane_clear(unsigned long long* A, int64_t n, int cs, const LaneMask& drop, hipStream_t s) {
  hipLaunchKernelGGL(k_lane_clear, dim3(grid_stride_for(n * cs)), dim3(kWG), 0, s, A, n, cs, drop);
  return hipGetLastError();
}

// ---------------------------------------------------------------- host loop

void MsState::release() {
  for (DevBuf* b : {&D, &MB, &D16, &A[0], &A[1], &bits, &list, &P, &scan_blocks, &push_tiles, &ctr, &pull_tiles[0],
                    &pull_tiles[1], &pull_tiles[2], &pull_tiles[3]})
    b->release();
  if (host) (void)hipHostFree(host);
  host = nullptr;
  n = m = 0;
  cs = 0;
}

size_t MsState::bytes() const {
  size_t b = 0;
  for (const DevBuf* x : {&D, &MB, &D16, &A[0], &A[1], &bits, &list, &P, &scan_blocks, &push_tiles, &ctr, &pull_tiles[0],
                          &pull_tiles[1], &pull_tiles[2], &pull_tiles[3]})
    b += x->bytes;
  return b;
}

vc_status ms_reset(MsState& st, vc_graph g, int cs, hipStream_t s, bool shadow) {
  if (cs < 1 || cs > 4) return fail(VC_ERR_INVALID_ARG, "lane chunks must be 1..4");
  if (!g->csc_ready) return fail(VC_ERR_INVALID_ARG, "many-lane loop needs the transpose");
  if (push_lds_bytes(kMsPushTile) > g->max_lds || (size_t)(4 * kMsPullTilePerChunk + 2) * 8 > g->max_lds)
    return fail(VC_ERR_UNSUPPORTED, "lane tiles exceed the device's LDS");
  const int64_t n = g->n, m = g->m;
  const size_t rows = (size_t)cs * n;
  VC_TRY(st.D.ensure(rows * 64 * 4));
  VC_TRY(st.MB.ensure(rows * 64 * 4));
  VC_TRY(st.A[0].ensure(rows * 8));
  VC_TRY(st.A[1].ensure(rows * 8));
  VC_TRY(st.bits.ensure((size_t)((n + 31) / 32) * 4));
  VC_TRY(st.list.ensure((size_t)n * 4 + 4));
  VC_TRY(st.P.ensure((size_t)(n + 1) * 8));
  VC_TRY(st.scan_blocks.ensure((size_t)scan_scratch_entries(n) * 8));
  VC_TRY(st.push_tiles.ensure((size_t)((n + m) / kMsPushTile + 2) * 4));
  VC_TRY(st.ctr.ensure(2 * sizeof(Counters)));
  if (!st.host) VC_TRY(hipHostMalloc((void**)&st.host, 2 * sizeof(Counters), hipHostMallocDefault));
  if (st.n != n || st.m != m || st.cs < cs) {
    for (int c = 1; c <= 4; ++c) {
      if (c > cs) {
        st.pull_tiles[c - 1].release();
        st.pull_ntiles[c - 1] = 0;
        continue;
      }
      const int64_t tile = kMsPullTilePerChunk * c;
      const int64_t ntiles = (n + m + tile - 1) / tile;
      VC_TRY(st.pull_tiles[c - 1].ensure((size_t)(ntiles + 1) * 4));
      VC_TRY(launch_mp_partition(g->csc_off_p, true, n, n + m, tile, ntiles, st.pull_tiles[c - 1].as<int32_t>(), s));
      st.pull_ntiles[c - 1] = ntiles;
    }
  }
  st.n = n;
  st.m = m;
  st.cs = cs;
  VC_TRY(launch_fill_u32(st.D.as<uint32_t>(), (int64_t)rows * 64, kInf, s));
  VC_TRY(launch_fill_u32(st.MB.as<uint32_t>(), (int64_t)rows * 64, kInf, s));
  VC_TRY(launch_fill_u32(st.A[0].as<uint32_t>(), (int64_t)rows * 2, 0u, s));
  VC_TRY(launch_fill_u32(st.A[1].as<uint32_t>(), (int64_t)rows * 2, 0u, s));
  VC_TRY(launch_fill_u32(st.bits.as<uint32_t>(), (n + 31) / 32, 0u, s));
  st.dirty[0] = st.dirty[1] = 0;
  st.shadow = shadow;
  if (shadow) {  // 0xFFFF (unreached) in both halves of every word
    VC_TRY(st.D16.ensure(rows * 64 * 2));
    VC_TRY(launch_fill_u32(st.D16.as<uint32_t>(), (int64_t)rows * 32, kInf, s));
  }
  return VC_OK;
}

vc_status ms_superstep(MsState& st, vc_graph g, int cur, int ceff, int64_t next_edges, bool force_pull,
                       const LaneMask& zero, unsigned long long* live, bool* pushed, hipStream_t s) {
  if (ceff < 1 || ceff > st.cs) return fail(VC_ERR_INVALID_ARG, "lane chunks out of range");
  const int64_t n = st.n, m = st.m;
  Counters* dctr = st.ctr.as<Counters>();
  unsigned long long* Acur = st.A[cur].as<unsigned long long>();
  unsigned long long* Anext = st.A[1 - cur].as<unsigned long long>();
  uint32_t* D = st.D.as<uint32_t>();
  uint32_t* MB = st.MB.as<uint32_t>();
  uint32_t* bits = st.bits.as<uint32_t>();
  if (st.dirty[cur] < ceff) st.dirty[cur] = ceff;  // seeds
  const double dense = kMsPullFraction * (double)m;
  bool pull = force_pull || (double)next_edges >= dense;
  *pushed = false;
  if (!pull) {
    VC_TRY(launch_zero_counters(dctr + 1, s));
    VC_TRY(launch_ms_compact(g->off, g->off64, Acur, n, ceff, st.list.as<int32_t>(), st.P.as<int64_t>(), dctr + 1, s));
    VC_TRY(hipMemcpyAsync(st.host + 1, dctr + 1, sizeof(Counters), hipMemcpyDeviceToHost, s));
    VC_TRY(hipStreamSynchronize(s));
    const int64_t items = (int64_t)st.host[1].listed, edges = (int64_t)st.host[1].edges;
    if ((double)edges >= dense) {
      pull = true;
    } else if (edges > 0) {
      int64_t* P = st.P.as<int64_t>();
      const int64_t ntiles = (items + edges + kMsPushTile - 1) / kMsPushTile;
      VC_TRY(launch_exclusive_scan(P, items, st.scan_blocks.as<int64_t>(), s));
      VC_TRY(launch_mp_partition(P, true, items, items + edges, kMsPushTile, ntiles, st.push_tiles.as<int32_t>(), s));
      if (g->off64)
        VC_TRY(launch_ms_push(ceff, g->w != nullptr, (const int64_t*)g->off, g->dst, g->w, n, st.list.as<int32_t>(), P,
                              items, edges, st.push_tiles.as<int32_t>(), kMsPushTile, ntiles, D, MB, Acur, bits, zero,
                              s));
      else
        VC_TRY(launch_ms_push(ceff, g->w != nullptr, (const int32_t*)g->off, g->dst, g->w, n, st.list.as<int32_t>(), P,
                              items, edges, st.push_tiles.as<int32_t>(), kMsPushTile, ntiles, D, MB, Acur, bits, zero,
                              s));
      *pushed = true;
    }
  }
  if (pull && st.shadow)
    VC_TRY(launch_ms_pull16(ceff, g->w != nullptr, g->csc_off_p, g->in_src, g->in_w, n, m,
                            st.pull_tiles[0].as<int32_t>(), kMsPullTilePerChunk, st.pull_ntiles[0],
                            st.D16.as<uint16_t>(), D, MB, bits, zero, s));
  else if (pull)
    VC_TRY(launch_ms_pull(ceff, g->w != nullptr, g->csc_off_p, g->in_src, g->in_w, n, m,
                          st.pull_tiles[ceff - 1].as<int32_t>(), kMsPullTilePerChunk * ceff, st.pull_ntiles[ceff - 1],
                          D, MB, bits, zero, s));
  const int clear = st.dirty[1 - cur] > ceff ? st.dirty[1 - cur] : ceff;
  VC_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(Anext), 2 * n * clear, 0u, s));
  st.dirty[1 - cur] = ceff;
  VC_TRY(launch_zero_counters(dctr, s));
  VC_TRY(launch_ms_apply(ceff, st.cs, g->off, g->off64, n, D, st.shadow ? st.D16.as<uint16_t>() : nullptr, MB, Anext,
                         bits, dctr, live, s));
  VC_TRY(hipMemcpyAsync(st.host, dctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  return VC_OK;
}

}  // namespace vc

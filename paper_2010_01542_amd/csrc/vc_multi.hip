// Many SSSP sources on one graph in one superstep loop.
//
// K <= 256 sources run side by side: distances form an N x K row-major
// matrix (K padded to 64 * C), one wavefront lane per source.  Each superstep
// is the pull form of the min combiner (paper, Section III) applied to all K
// programs at once: a receiver's row takes, lane by lane, the minimum of
// dist(u) + w(u, v) over in-neighbours u whose lane improved in the previous
// superstep (paper, Section I: only vertices that received a better message
// broadcast).  An in-edge moves one 256-byte row chunk per 64 sources, so the
// loads are coalesced and no per-lane atomic is needed for receivers owned by
// one tile.  Per (vertex, chunk) a 64-bit mask records which lanes are
// active.  Values and mailboxes are separate matrices, so the superstep stays
// bulk-synchronous.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

struct Tile {
  int64_t i0, j0, j1;
  int cnt;
};

__device__ __forceinline__ bool tile_bounds(const int32_t* __restrict__ tile_v, int64_t tile, int64_t items,
                                            int64_t edges, Tile* tl) {
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < items + edges) ? k0 + tile : items + edges;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  tl->i0 = i0;
  tl->j0 = k0 - i0;
  tl->j1 = k1 - i1;
  const int64_t ilast = i1 < items ? i1 : items - 1;
  tl->cnt = (int)(ilast - i0 + 1);
  return tl->j1 > tl->j0;
}

__device__ __forceinline__ int owner_of(const int64_t* __restrict__ s_off, int cnt, int64_t e) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// D = MB = unreached; masks and bitmap cleared by the host with fills.
// Source k (internal id src[k]) starts at distance 0 with lane k active.
template <int C>
__global__ void k_ms_seed(const int32_t* __restrict__ src, const int32_t* __restrict__ perm, int k_real,
                          uint32_t* __restrict__ D, unsigned long long* __restrict__ A, uint32_t* __restrict__ bits) {
  constexpr int K = 64 * C;
  const int k = threadIdx.x + blockIdx.x * blockDim.x;
  if (k >= k_real) return;
  const int64_t x = perm ? (int64_t)perm[src[k]] : (int64_t)src[k];
  D[x * K + k] = 0u;
  atomicOr(&A[x * C + (k >> 6)], 1ull << (k & 63));
  atomicOr(&bits[x >> 5], 1u << (x & 31));
}

// Per receiver v and lane: best = min over active in-neighbours of D[u] + w.
template <int C, bool WEIGHTED>
__global__ __launch_bounds__(64 * C) void k_ms_pull(const int64_t* __restrict__ in_off,
                                                    const int32_t* __restrict__ in_src,
                                                    const uint32_t* __restrict__ in_w, int64_t n, int64_t m,
                                                    const int32_t* __restrict__ tile_v, int64_t tile,
                                                    const uint32_t* __restrict__ D, uint32_t* __restrict__ MB,
                                                    const unsigned long long* __restrict__ A,
                                                    uint32_t* __restrict__ improved, LaneMask zero) {
  constexpr int K = 64 * C;
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
  int x = owner_of(s_off, tl.cnt, tl.j0);
  int64_t next = s_off[x + 1];
  uint32_t run = kInf;
  auto flush = [&](int xo, uint32_t best) {
    const int64_t v = tl.i0 + xo;
    bool imp = false;
    if (best != kInf) {
      const int64_t idx = v * K + c * 64 + lane;
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
    unsigned long long msk[U];
    uint32_t val[U], wv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) u[k] = e0 + k < tl.j1 ? in_src[e0 + k] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) msk[k] = e0 + k < tl.j1 ? A[(int64_t)u[k] * C + c] : 0ull;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      wv[k] = (WEIGHTED && e0 + k < tl.j1) ? in_w[e0 + k] : 1u;
      val[k] = ((msk[k] >> lane) & 1ull) ? D[(int64_t)u[k] * K + c * 64 + lane] : kInf;
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

// For every improved vertex (one workgroup per bitmap word): adopt the
// mailbox lane by lane, reset it, record the improved lanes as the vertex's
// active mask for the next superstep, and count |F| and E.  A vertex without
// out-edges keeps an empty mask: it has nobody to broadcast to.  live (may be
// NULL) collects the OR of all masks, spread over 64 words per chunk to keep
// same-address atomics rare: a lane is live while some word holds its bit.
template <int C, class OffT>
__global__ __launch_bounds__(64 * C) void k_ms_apply(const OffT* __restrict__ off, int64_t nwords,
                                                     uint32_t* __restrict__ D, uint32_t* __restrict__ MB,
                                                     unsigned long long* __restrict__ A_next,
                                                     uint32_t* __restrict__ improved, Counters* __restrict__ ctr,
                                                     unsigned long long* __restrict__ live) {
  constexpr int K = 64 * C;
  const int64_t wi = blockIdx.x;
  if (wi >= nwords) return;
  const uint32_t word = improved[wi];
  if (!word) return;
  const int c = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  unsigned long long any = 0;
  for (uint32_t bits = word; bits; bits &= bits - 1) {
    const int64_t v = wi * 32 + (__ffs(bits) - 1);
    const int64_t idx = v * K + c * 64 + lane;
    const uint32_t mb = MB[idx];
    const bool act = mb < D[idx];
    if (act) D[idx] = mb;
    if (mb != kInf) MB[idx] = kInf;
    const bool sends = off[v + 1] > off[v];
    const unsigned long long mask = sends ? __ballot(act) : 0ull;
    any |= mask;
    if (lane == 0) A_next[v * C + c] = mask;
  }
  if (live && any && lane == 0) atomicOr(&live[(wi & 63) * C + c], any);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long edges = 0;
    for (uint32_t bits = word; bits; bits &= bits - 1) {
      const int64_t v = wi * 32 + (__ffs(bits) - 1);
      edges += (unsigned long long)((int64_t)off[v + 1] - (int64_t)off[v]);
    }
    atomicAdd(&ctr->active, (unsigned long long)__popc(word));
    if (edges) atomicAdd(&ctr->edges, edges);
    improved[wi] = 0;
  }
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

// out[v * k_real + k] = D[perm[v] * K + k]
template <int C>
__global__ __launch_bounds__(kWG) void k_ms_output(const uint32_t* __restrict__ D, const int32_t* __restrict__ perm,
                                                   int64_t n, int k_real, uint32_t* __restrict__ out) {
  constexpr int K = 64 * C;
  const int64_t i = gid();
  if (i >= n * k_real) return;
  const int64_t v = i / k_real;
  const int k = (int)(i - v * k_real);
  const int64_t x = perm ? (int64_t)perm[v] : v;
  out[i] = D[x * K + k];
}

// Lane seeding, CC: every vertex x takes its label ids[x] (x itself when
// ids is NULL) in each listed lane and is active there if it has out-edges.
// One thread per vertex, so the mask update needs no atomic.
template <int C, class OffT>
__global__ __launch_bounds__(kWG) void k_lane_seed_cc(const OffT* __restrict__ off, const int32_t* __restrict__ ids,
                                                      int64_t n, const int32_t* __restrict__ lanes, int r,
                                                      uint32_t* __restrict__ D, unsigned long long* __restrict__ A) {
  constexpr int K = 64 * C;
  const int64_t x = gid();
  if (x >= n) return;
  const uint32_t label = ids ? (uint32_t)ids[x] : (uint32_t)x;
  unsigned long long acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0;
  for (int j = 0; j < r; ++j) {
    const int l = lanes[j];
    D[x * K + l] = label;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if ((l >> 6) == c) acc[c] |= 1ull << (l & 63);
  }
  if (off[x + 1] > off[x]) {
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (acc[c]) A[x * C + c] |= acc[c];
  }
}

// Lane seeding, SSSP: seeds[2j] = lane, seeds[2j + 1] = source (caller's
// id).  The source starts at 0 and is active if it has out-edges; a lane
// whose source has none is flagged in stillborn (it ends after one
// superstep with nothing sent).
template <int C, class OffT>
__global__ __launch_bounds__(kWG) void k_lane_seed_sssp(const OffT* __restrict__ off, const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ seeds, int r,
                                                        uint32_t* __restrict__ D, unsigned long long* __restrict__ A,
                                                        unsigned long long* __restrict__ stillborn) {
  constexpr int K = 64 * C;
  const int j = (int)gid();
  if (j >= r) return;
  const int l = seeds[2 * j];
  const int64_t src = seeds[2 * j + 1];
  const int64_t x = perm ? (int64_t)perm[src] : src;
  D[x * K + l] = 0u;
  if (off[x + 1] > off[x])
    atomicOr(&A[x * C + (l >> 6)], 1ull << (l & 63));
  else
    atomicOr(&stillborn[l >> 6], 1ull << (l & 63));
}

// Lane retirement: outs[j][v] = D[perm[v], lanes[j]], and the column is
// reset to unreached for the next request of that lane.
template <int C>
__global__ __launch_bounds__(kWG) void k_lane_retire(uint32_t* __restrict__ D, const int32_t* __restrict__ perm,
                                                     int64_t n, const int32_t* __restrict__ lanes,
                                                     uint32_t* const* __restrict__ outs, int r) {
  constexpr int K = 64 * C;
  const int64_t i = gid();
  if (i >= n * r) return;
  const int64_t v = i / r;
  const int j = (int)(i - v * r);
  const int64_t x = perm ? (int64_t)perm[v] : v;
  const int64_t idx = x * K + lanes[j];
  outs[j][v] = D[idx];
  D[idx] = kInf;
}

// Clears the listed lanes from every active mask (lanes stopped at their
// superstep cap while still active).
template <int C>
__global__ __launch_bounds__(kWG) void k_lane_clear(unsigned long long* __restrict__ A, int64_t n, LaneMask drop) {
  const int64_t i = gid();
  if (i >= n * C) return;
  const int c = (int)(i % C);
  if (drop.bits[c]) A[i] &= ~drop.bits[c];
}

}  // namespace

int ms_chunks(int k) { return (k + 63) / 64; }

hipError_t launch_ms_seed(int C, const int32_t* src, const int32_t* perm, int k_real, uint32_t* D,
                          unsigned long long* A, uint32_t* bits, hipStream_t s) {
  switch (C) {
    case 1: hipLaunchKernelGGL(k_ms_seed<1>, dim3(1), dim3(256), 0, s, src, perm, k_real, D, A, bits); break;
    case 2: hipLaunchKernelGGL(k_ms_seed<2>, dim3(1), dim3(256), 0, s, src, perm, k_real, D, A, bits); break;
    case 3: hipLaunchKernelGGL(k_ms_seed<3>, dim3(1), dim3(256), 0, s, src, perm, k_real, D, A, bits); break;
    default: hipLaunchKernelGGL(k_ms_seed<4>, dim3(1), dim3(256), 0, s, src, perm, k_real, D, A, bits);
  }
  return hipGetLastError();
}

namespace {
template <int C>
void ms_pull_launch(bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w, int64_t n,
                    int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles, const uint32_t* D, uint32_t* MB,
                    const unsigned long long* A, uint32_t* improved, const LaneMask& zero, hipStream_t s) {
  const size_t lds = (size_t)(tile + 2) * 8;
  if (weighted)
    hipLaunchKernelGGL((k_ms_pull<C, true>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D, MB, A, improved, zero);
  else
    hipLaunchKernelGGL((k_ms_pull<C, false>), dim3((unsigned)ntiles), dim3(64 * C), lds, s, in_off, in_src, in_w, n, m,
                       tile_v, tile, D, MB, A, improved, zero);
}
template <int C>
void ms_apply_launch(const void* off, bool off64, int64_t nwords, uint32_t* D, uint32_t* MB,
                     unsigned long long* A_next, uint32_t* improved, Counters* ctr, unsigned long long* live,
                     hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_ms_apply<C, int64_t>), dim3((unsigned)nwords), dim3(64 * C), 0, s, (const int64_t*)off,
                       nwords, D, MB, A_next, improved, ctr, live);
  else
    hipLaunchKernelGGL((k_ms_apply<C, int32_t>), dim3((unsigned)nwords), dim3(64 * C), 0, s, (const int32_t*)off,
                       nwords, D, MB, A_next, improved, ctr, live);
}
}  // namespace

hipError_t launch_ms_pull(int C, bool weighted, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                          int64_t n, int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles,
                          const uint32_t* D, uint32_t* MB, const unsigned long long* A, uint32_t* improved,
                          const LaneMask& zero, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (C) {
    case 1: ms_pull_launch<1>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, A, improved, zero, s); break;
    case 2: ms_pull_launch<2>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, A, improved, zero, s); break;
    case 3: ms_pull_launch<3>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, A, improved, zero, s); break;
    default: ms_pull_launch<4>(weighted, in_off, in_src, in_w, n, m, tile_v, tile, ntiles, D, MB, A, improved, zero, s);
  }
  return hipGetLastError();
}

hipError_t launch_ms_apply(int C, const void* off, bool off64, int64_t n, uint32_t* D, uint32_t* MB,
                           unsigned long long* A_next, uint32_t* improved, Counters* ctr, unsigned long long* live,
                           hipStream_t s) {
  const int64_t nwords = (n + 31) / 32;
  switch (C) {
    case 1: ms_apply_launch<1>(off, off64, nwords, D, MB, A_next, improved, ctr, live, s); break;
    case 2: ms_apply_launch<2>(off, off64, nwords, D, MB, A_next, improved, ctr, live, s); break;
    case 3: ms_apply_launch<3>(off, off64, nwords, D, MB, A_next, improved, ctr, live, s); break;
    default: ms_apply_launch<4>(off, off64, nwords, D, MB, A_next, improved, ctr, live, s);
  }
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

hipError_t launch_ms_output(int C, const uint32_t* D, const int32_t* perm, int64_t n, int k_real, uint32_t* out,
                            hipStream_t s) {
  const int64_t total = n * k_real;
  switch (C) {
    case 1: hipLaunchKernelGGL(k_ms_output<1>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, k_real, out); break;
    case 2: hipLaunchKernelGGL(k_ms_output<2>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, k_real, out); break;
    case 3: hipLaunchKernelGGL(k_ms_output<3>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, k_real, out); break;
    default: hipLaunchKernelGGL(k_ms_output<4>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, k_real, out);
  }
  return hipGetLastError();
}

namespace {
template <int C>
void lane_seed_cc_launch(const void* off, bool off64, const int32_t* ids, int64_t n, const int32_t* lanes, int r,
                         uint32_t* D, unsigned long long* A, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_lane_seed_cc<C, int64_t>), dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, ids, n,
                       lanes, r, D, A);
  else
    hipLaunchKernelGGL((k_lane_seed_cc<C, int32_t>), dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, ids, n,
                       lanes, r, D, A);
}
template <int C>
void lane_seed_sssp_launch(const void* off, bool off64, const int32_t* perm, const int32_t* seeds, int r, uint32_t* D,
                           unsigned long long* A, unsigned long long* stillborn, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL((k_lane_seed_sssp<C, int64_t>), dim3(grid_for(r)), dim3(kWG), 0, s, (const int64_t*)off, perm,
                       seeds, r, D, A, stillborn);
  else
    hipLaunchKernelGGL((k_lane_seed_sssp<C, int32_t>), dim3(grid_for(r)), dim3(kWG), 0, s, (const int32_t*)off, perm,
                       seeds, r, D, A, stillborn);
}
}  // namespace

hipError_t launch_lane_seed_cc(int C, const void* off, bool off64, const int32_t* ids, int64_t n,
                               const int32_t* lanes, int r, uint32_t* D, unsigned long long* A, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  switch (C) {
    case 1: lane_seed_cc_launch<1>(off, off64, ids, n, lanes, r, D, A, s); break;
    case 2: lane_seed_cc_launch<2>(off, off64, ids, n, lanes, r, D, A, s); break;
    case 3: lane_seed_cc_launch<3>(off, off64, ids, n, lanes, r, D, A, s); break;
    default: lane_seed_cc_launch<4>(off, off64, ids, n, lanes, r, D, A, s);
  }
  return hipGetLastError();
}

hipError_t launch_lane_seed_sssp(int C, const void* off, bool off64, const int32_t* perm, const int32_t* seeds, int r,
                                 uint32_t* D, unsigned long long* A, unsigned long long* stillborn, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  switch (C) {
    case 1: lane_seed_sssp_launch<1>(off, off64, perm, seeds, r, D, A, stillborn, s); break;
    case 2: lane_seed_sssp_launch<2>(off, off64, perm, seeds, r, D, A, stillborn, s); break;
    case 3: lane_seed_sssp_launch<3>(off, off64, perm, seeds, r, D, A, stillborn, s); break;
    default: lane_seed_sssp_launch<4>(off, off64, perm, seeds, r, D, A, stillborn, s);
  }
  return hipGetLastError();
}

hipError_t launch_lane_retire(int C, uint32_t* D, const int32_t* perm, int64_t n, const int32_t* lanes,
                              uint32_t* const* outs, int r, hipStream_t s) {
  if (r <= 0 || n <= 0) return hipSuccess;
  const int64_t total = n * r;
  switch (C) {
    case 1: hipLaunchKernelGGL(k_lane_retire<1>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, lanes, outs, r); break;
    case 2: hipLaunchKernelGGL(k_lane_retire<2>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, lanes, outs, r); break;
    case 3: hipLaunchKernelGGL(k_lane_retire<3>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, lanes, outs, r); break;
    default: hipLaunchKernelGGL(k_lane_retire<4>, dim3(grid_for(total)), dim3(kWG), 0, s, D, perm, n, lanes, outs, r);
  }
  return hipGetLastError();
}

hipError_t launch_lane_clear(int C, unsigned long long* A, int64_t n, const LaneMask& drop, hipStream_t s) {
  const int64_t total = n * C;
  switch (C) {
    case 1: hipLaunchKernelGGL(k_lane_clear<1>, dim3(grid_for(total)), dim3(kWG), 0, s, A, n, drop); break;
    case 2: hipLaunchKernelGGL(k_lane_clear<2>, dim3(grid_for(total)), dim3(kWG), 0, s, A, n, drop); break;
    case 3: hipLaunchKernelGGL(k_lane_clear<3>, dim3(grid_for(total)), dim3(kWG), 0, s, A, n, drop); break;
    default: hipLaunchKernelGGL(k_lane_clear<4>, dim3(grid_for(total)), dim3(kWG), 0, s, A, n, drop);
  }
  return hipGetLastError();
}

}  // namespace vc

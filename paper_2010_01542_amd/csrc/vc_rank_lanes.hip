// PageRank / PPR lanes of the request server: up to 256 rank programs on
// one graph advance together, one superstep per launch pair (pull, apply).
//
// Each lane is one program of the paper's PageRank benchmark (Section VI)
// with the sum combiner (Section III): a vertex's message is its rank over
// its out-degree, a receiver sums the messages of its in-neighbours (pull
// form, Section VI-C) and its new rank is the teleport term plus the damped
// sum.  Sums are exact: messages are unsigned fixed-point numbers with 62
// fractional bits and integer addition is associative, so a lane's ranks are
// bit-identical to the same program run alone, whatever else shares the
// superstep.  Lanes run at their own pace: a lane seeded this superstep and
// a lane at its last update share the launches.
//
// Layout is chunk-major as for the min lanes: chunk c of vertex v at
// c * n + v, a row of 64 lanes of 8-byte messages / mailboxes.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

constexpr double kFx = 4611686018427387904.0;  // 2^62
constexpr double kFxInv = 1.0 / 4611686018427387904.0;


__device__ __forceinline__ unsigned long long message(double r, int64_t deg) {
  return deg > 0 ? __double2ull_rn(r / (double)deg * kFx) : 0ull;
}

// Seeding: every vertex x starts each listed lane at rank 1/N (PageRank) or
// at 1 on the source and 0 elsewhere (PPR; sources in caller ids, ids[x] is
// x's caller id or x itself when ids is NULL), and holds the message of
// that rank.  seeds[2j] = lane, seeds[2j + 1] = source or -1.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_rl_seed(const OffT* __restrict__ off, const int32_t* __restrict__ ids,
                                                 int64_t n, const int32_t* __restrict__ seeds, int r,
                                                 unsigned long long* __restrict__ contrib) {
  const int64_t x = gid();
  if (x >= n) return;
  const int64_t deg = (int64_t)off[x + 1] - (int64_t)off[x];
  const int64_t id = ids ? (int64_t)ids[x] : x;
  const double r0 = 1.0 / (double)n;
  for (int j = 0; j < r; ++j) {
    const int l = seeds[2 * j];
    const int64_t src = seeds[2 * j + 1];
    const double rank = src >= 0 ? (id == src ? 1.0 : 0.0) : r0;
    contrib[((int64_t)(l >> 6) * n + x) * 64 + (l & 63)] = message(rank, deg);
  }
}

// Pull: per receiver v and lane, the sum of its in-neighbours' messages
// into the mailbox (stored when the tile holds all of v's in-edges, else
// added atomically).  One wavefront per chunk.
template <int C>
__global__ __launch_bounds__(64 * C) void k_rl_pull(const int64_t* __restrict__ in_off,
                                                    const int32_t* __restrict__ in_src, int64_t n, int64_t m,
                                                    const int32_t* __restrict__ tile_v, int64_t tile,
                                                    const unsigned long long* __restrict__ contrib,
                                                    unsigned long long* __restrict__ mb) {
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned char smem[];
  Tile tl;
  if (!tile_bounds(tile_v, tile, n, m, &tl)) return;
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);
  for (int x = threadIdx.x; x <= tl.cnt; x += 64 * C) s_off[x] = in_off[tl.i0 + x];
  __syncthreads();
  const int c = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const unsigned long long* Cc = contrib + (int64_t)c * n * 64 + lane;
  unsigned long long* Mc = mb + (int64_t)c * n * 64 + lane;
  int x = owner_of(s_off, tl.cnt, tl.j0);
  int64_t next = s_off[x + 1];
  unsigned long long run = 0;
  auto flush = [&](int xo, unsigned long long sum) {
    if (!sum) return;
    const int64_t v = tl.i0 + xo;
    if (s_off[xo] >= tl.j0 && s_off[xo + 1] <= tl.j1)
      Mc[v * 64] = sum;  // every in-edge of v is in this tile
    else
      atomicAdd(&Mc[v * 64], sum);
  };
  for (int64_t e0 = tl.j0; e0 < tl.j1; e0 += U) {
    int32_t u[U];
    unsigned long long val[U];
#pragma unroll
    for (int k = 0; k < U; ++k) u[k] = e0 + k < tl.j1 ? in_src[e0 + k] : 0;
#pragma unroll
    for (int k = 0; k < U; ++k) val[k] = e0 + k < tl.j1 ? Cc[(int64_t)u[k] * 64] : 0ull;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t e = e0 + k;
      if (e < tl.j1) {
        while (e >= next) {  // receiver changes (uniform over the wavefront)
          flush(x, run);
          run = 0;
          ++x;
          next = s_off[x + 1];
        }
        run += val[k];
      }
    }
  }
  flush(x, run);
}

// Apply, one thread per (chunk, vertex, lane) of the first ceff chunks:
// rank = teleport + d * sum, then either the next message or, at the lane's
// last update, the rank written to the request's output (caller's vertex
// order) and the lane cleared for its next request.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_rl_apply(const OffT* __restrict__ off, const int32_t* __restrict__ ids,
                                                  int64_t n, int ceff, const RankLane* __restrict__ lanes,
                                                  unsigned long long* __restrict__ contrib,
                                                  unsigned long long* __restrict__ mb) {
  const int64_t total = (int64_t)ceff * n * 64;
  for (int64_t i = gid(); i < total; i += grid_threads()) {
    const int lane = (int)(i & 63);
    const int64_t rowi = i >> 6;
    const int c = (int)(rowi / n);
    const int64_t v = rowi - (int64_t)c * n;
    const RankLane& P = lanes[c * 64 + lane];
    if (P.state == 0) continue;
    const int64_t id = ids ? (int64_t)ids[v] : v;
    const double tele = P.source >= 0 ? (id == P.source ? P.teleport : 0.0) : P.teleport;
    const double r = fma(P.damping, (double)mb[i] * kFxInv, tele);
    mb[i] = 0ull;
    if (P.state == 2) {
      P.out[id] = (float)r;
      contrib[i] = 0ull;
    } else {
      contrib[i] = message(r, (int64_t)off[v + 1] - (int64_t)off[v]);
    }
  }
}

template <int C>
hipError_t rl_pull_launch(const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m, const int32_t* tile_v,
                          int64_t tile, int64_t ntiles, const unsigned long long* contrib, unsigned long long* mb,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_rl_pull<C>), dim3((unsigned)ntiles), dim3(64 * C), (size_t)(tile + 2) * 8, s, in_off, in_src,
                     n, m, tile_v, tile, contrib, mb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rl_seed(const void* off, bool off64, const int32_t* ids, int64_t n, const int32_t* seeds, int r,
                          unsigned long long* contrib, hipStream_t s) {
  if (r <= 0) return hipSuccess;
  if (off64)
    hipLaunchKernelGGL(k_rl_seed<int64_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, ids, n, seeds, r,
                       contrib);
  else
    hipLaunchKernelGGL(k_rl_seed<int32_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, ids, n, seeds, r,
                       contrib);
  return hipGetLastError();
}

hipError_t launch_rl_pull(int C, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const unsigned long long* contrib,
                          unsigned long long* mb, hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  switch (C) {
    case 1: return rl_pull_launch<1>(in_off, in_src, n, m, tile_v, tile, ntiles, contrib, mb, s);
    case 2: return rl_pull_launch<2>(in_off, in_src, n, m, tile_v, tile, ntiles, contrib, mb, s);
    case 3: return rl_pull_launch<3>(in_off, in_src, n, m, tile_v, tile, ntiles, contrib, mb, s);
    case 4: return rl_pull_launch<4>(in_off, in_src, n, m, tile_v, tile, ntiles, contrib, mb, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_rl_apply(const void* off, bool off64, const int32_t* ids, int64_t n, int ceff,
                           const RankLane* lanes, unsigned long long* contrib, unsigned long long* mb, hipStream_t s) {
  if (ceff < 1 || ceff > 4) return hipErrorInvalidValue;
  const int64_t total = (int64_t)ceff * n * 64;
  if (off64)
    hipLaunchKernelGGL(k_rl_apply<int64_t>, dim3(grid_stride_for(total)), dim3(kWG), 0, s, (const int64_t*)off, ids, n,
                       ceff, lanes, contrib, mb);
  else
    hipLaunchKernelGGL(k_rl_apply<int32_t>, dim3(grid_stride_for(total)), dim3(kWG), 0, s, (const int32_t*)off, ids, n,
                       ceff, lanes, contrib, mb);
  return hipGetLastError();
}

}  // namespace vc

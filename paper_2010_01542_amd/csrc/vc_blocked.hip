// PageRank broadcast + combine by propagation blocking (a variant of the
// paper's single-broadcast pull, Section VI-C, for graphs much larger than
// the caches).
//
// The pull form gathers one 8-byte message per in-edge from anywhere in the
// message array; on a billion-edge graph most of those gathers miss the
// caches, and even those that hit cost one cache-line request per edge.
// Here the edges are laid out once by bucket (source tile, destination bin):
// a source tile's messages fit in LDS (2^14 vertices, 128 KiB), a
// destination bin's mailboxes too (2^12 vertices, 32 KiB).  A superstep is
// two streaming passes:
//   1. spread: per source tile, its messages are staged in LDS, then every
//      slot of the tile's buckets (contiguous, tile-major order) gets
//      vals[k] = message of its source: 2-byte index in, 8 bytes out;
//   2. fold: per destination bin, its runs (one per source tile) are read
//      and summed into LDS mailboxes, which are then written to the mailbox
//      array (added atomically when a bin of hubs is split over several
//      workgroups).
// Sums stay exact (uint64 fixed point), so results equal the pull form's.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

constexpr int kMaxSrcShift = 14;

// ---------------------------------------------------------------- layout build
// Source tile t holds vertices [t << shift, (t + 1) << shift); its out-edges
// are the CSR edges [te[t], te[t + 1]) with te[t] = off[t << shift], and in
// tile-major order its slots are that same range.  The build counts each
// bucket with per-workgroup LDS histograms, reserves a sub-range of each
// bucket per workgroup with one global atomic, and places the edges.

template <class OffT>
__global__ __launch_bounds__(kWG) void k_pb_tile_edges(const OffT* __restrict__ off, int64_t n, int shift,
                                                       int64_t tiles, int64_t* __restrict__ te) {
  const int64_t t = gid();
  if (t > tiles) return;
  const int64_t v = (t << shift) < n ? (t << shift) : n;
  te[t] = (int64_t)off[v];
}

// srcl_csr[e] = offset of edge e's source in its tile, by a merge-path walk.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_pb_expand(const OffT* __restrict__ off, int64_t n, int64_t m,
                                                   const int32_t* __restrict__ tile_v, int64_t tile, int shift,
                                                   uint16_t* __restrict__ srcl_csr) {
  extern __shared__ __align__(16) int64_t s_off[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);
  for (int x = threadIdx.x; x <= cnt; x += kWG) s_off[x] = (int64_t)off[i0 + x];
  __syncthreads();
  const int64_t mask = (1ll << shift) - 1;
  for (int64_t e = j0 + threadIdx.x; e < j1; e += kWG) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    srcl_csr[e] = (uint16_t)((i0 + lo) & mask);
  }
}

constexpr int kBuildWG = 1024;

// Tile of edge c0: last t with te[t] <= c0 (te[0] = 0 <= c0 < m = te[tiles]).
__device__ __forceinline__ int64_t tile_of(const int64_t* __restrict__ te, int64_t tiles, int64_t c0) {
  int64_t lo = 0, hi = tiles - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (te[mid] <= c0)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per workgroup: edges [c0, c1) of the CSR, split by source tile; per tile
// and per range of pass_bins bins, an LDS histogram of destination bins.
// PLACE = false adds the histogram into cnt (bucket counts); PLACE = true
// reserves each bucket's share at cursor and writes the slots.
template <bool PLACE>
__global__ __launch_bounds__(kBuildWG) void k_pb_build(const int64_t* __restrict__ te, int64_t tiles,
                                                       const int32_t* __restrict__ dst, int64_t m, int64_t chunk,
                                                       int64_t bins, int pass_bins,
                                                       unsigned long long* __restrict__ cnt,
                                                       const uint16_t* __restrict__ srcl_csr,
                                                       uint16_t* __restrict__ srcl, uint16_t* __restrict__ dstl) {
  extern __shared__ __align__(16) uint32_t hist[];  // pass_bins counters, then (PLACE) pass_bins offsets
  uint32_t* rel = hist + pass_bins;
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = (c0 + chunk < m) ? c0 + chunk : m;
  for (int64_t t = tile_of(te, tiles, c0); t < tiles && te[t] < c1; ++t) {
    const int64_t e0 = te[t] > c0 ? te[t] : c0;
    const int64_t e1 = te[t + 1] < c1 ? te[t + 1] : c1;
    if (e0 >= e1) continue;
    for (int64_t b_lo = 0; b_lo < bins; b_lo += pass_bins) {
      const int nb = (int)((bins - b_lo < pass_bins) ? bins - b_lo : pass_bins);
      for (int i = threadIdx.x; i < nb; i += kBuildWG) hist[i] = 0u;
      __syncthreads();
      for (int64_t e = e0 + threadIdx.x; e < e1; e += kBuildWG) {
        const int64_t b = (int64_t)(dst[e] >> kPbDstShift) - b_lo;
        if (b >= 0 && b < nb) atomicAdd(&hist[b], 1u);
      }
      __syncthreads();
      unsigned long long* C = cnt + t * bins + b_lo;
      for (int i = threadIdx.x; i < nb; i += kBuildWG) {
        const uint32_t h = hist[i];
        if (!PLACE) {
          if (h) atomicAdd(&C[i], (unsigned long long)h);
        } else {
          rel[i] = h ? (uint32_t)(atomicAdd(&C[i], (unsigned long long)h) - (unsigned long long)te[t]) : 0u;
          hist[i] = 0u;
        }
      }
      __syncthreads();
      if (PLACE) {
        // every slot reserved here lies in the tile's range [te[t], te[t + 1])
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kBuildWG) {
          const int32_t v = dst[e];
          const int64_t b = (int64_t)(v >> kPbDstShift) - b_lo;
          if (b >= 0 && b < nb) {
            const int64_t k = te[t] + (int64_t)rel[b] + (int64_t)atomicAdd(&hist[b], 1u);
            srcl[k] = srcl_csr[e];
            dstl[k] = (uint16_t)(v & ((1 << kPbDstShift) - 1));
          }
        }
        __syncthreads();
      }
    }
  }
}

// Per bin b (one thread): run prefix sums pre[b][t], slot bases base[b][t]
// and the number of fold items of the bin.
__global__ __launch_bounds__(kWG) void k_pb_tables(const int64_t* __restrict__ starts, int64_t bins, int64_t tiles,
                                                   int64_t fcap, int64_t* __restrict__ pre,
                                                   int64_t* __restrict__ base, int64_t* __restrict__ nitems) {
  const int64_t b = gid();
  if (b >= bins) return;
  int64_t* P = pre + b * (tiles + 1);
  int64_t* B = base + b * tiles;
  int64_t acc = 0;
  for (int64_t t = 0; t < tiles; ++t) {
    const int64_t q = t * bins + b;
    const int64_t s0 = starts[q], s1 = starts[q + 1];
    P[t] = acc;
    B[t] = s0 - acc;
    acc += s1 - s0;
  }
  P[tiles] = acc;
  nitems[b] = (acc + fcap - 1) / fcap;
}

// Per bin b (one thread): its fold items, positions [i fcap, (i+1) fcap).
__global__ __launch_bounds__(kWG) void k_pb_fold_items(const int64_t* __restrict__ pre, int64_t bins, int64_t tiles,
                                                       int64_t fcap, const int64_t* __restrict__ item_off,
                                                       PbFoldItem* __restrict__ items) {
  const int64_t b = gid();
  if (b >= bins) return;
  const int64_t* P = pre + b * (tiles + 1);
  const int64_t total = P[tiles];
  const int64_t first = item_off[b], count = item_off[b + 1] - item_off[b];
  int64_t r = 0;  // run holding position v: last r with P[r] <= v (v < total = P[tiles])
  for (int64_t i = 0; i < count; ++i) {
    const int64_t v0 = i * fcap;
    const int64_t v1 = (v0 + fcap < total) ? v0 + fcap : total;
    while (P[r + 1] <= v0) ++r;
    int64_t r1 = r;
    while (P[r1 + 1] <= v1 - 1) ++r1;
    items[first + i] = PbFoldItem{(int32_t)b, count == 1 ? 1 : 0, r, r1 + 1, v0, v1};
  }
}

// Pass 1: one workgroup per spread item; the tile's messages in LDS.
constexpr int kSpreadWG = 1024;

__global__ __launch_bounds__(kSpreadWG) void k_pb_spread(const PbSpreadItem* __restrict__ items, int64_t n, int shift,
                                                         const uint16_t* __restrict__ srcl,
                                                         const unsigned long long* __restrict__ msg,
                                                         unsigned long long* __restrict__ vals) {
  constexpr int U = 8;
  extern __shared__ __align__(16) unsigned long long win[];
  const PbSpreadItem it = items[blockIdx.x];
  const int64_t u0 = (int64_t)it.t << shift;
  const int64_t wl = (n - u0 < (1ll << shift)) ? n - u0 : (1ll << shift);
  for (int64_t i = threadIdx.x; i < wl; i += kSpreadWG) win[i] = msg[u0 + i];
  __syncthreads();
  for (int64_t base = it.k0 + threadIdx.x; base < it.k1; base += (int64_t)kSpreadWG * U) {
    uint16_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = base + (int64_t)u * kSpreadWG;
      x[u] = k < it.k1 ? srcl[k] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = base + (int64_t)u * kSpreadWG;
      if (k < it.k1) vals[k] = win[x[u]];
    }
  }
}

// Pass 2: one workgroup per fold item.  Runs are staged kFoldRuns at a
// time (prefix sums and slot bases in LDS); each lane takes U positions 64
// apart, finds the run of the first by binary search, steps forward for the
// rest, and adds the U messages into the LDS mailboxes.  Items are
// handed out so that each of the 8 XCDs takes a contiguous range of bins:
// runs of neighbouring bins share cache lines at their ends, which then
// meet in the same L2.
constexpr int kFoldWG = 512;
constexpr int kFoldRuns = 1024;

__global__ __launch_bounds__(kFoldWG) void k_pb_fold(const PbFoldItem* __restrict__ items, int64_t nitems,
                                                     int64_t tiles, int64_t n, const int64_t* __restrict__ pre,
                                                     const int64_t* __restrict__ base,
                                                     const unsigned long long* __restrict__ vals,
                                                     const uint16_t* __restrict__ dstl,
                                                     unsigned long long* __restrict__ mb) {
  constexpr int U = 8;
  __shared__ unsigned long long box[1 << kPbDstShift];
  __shared__ int64_t s_pre[kFoldRuns + 1];
  __shared__ int64_t s_base[kFoldRuns];
  const int64_t per = (nitems + 7) >> 3;
  const int64_t j = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (j >= nitems) return;
  const PbFoldItem it = items[j];
  for (int i = threadIdx.x; i < (1 << kPbDstShift); i += kFoldWG) box[i] = 0ull;
  const int64_t* P = pre + (int64_t)it.b * (tiles + 1);
  const int64_t* B = base + (int64_t)it.b * tiles;
  for (int64_t w0 = it.r0; w0 < it.r1; w0 += kFoldRuns) {
    const int wn = (int)((it.r1 - w0 < kFoldRuns) ? it.r1 - w0 : kFoldRuns);
    for (int i = threadIdx.x; i <= wn; i += kFoldWG) {
      s_pre[i] = P[w0 + i];  // w0 + wn <= r1 <= tiles
      if (i < wn) s_base[i] = B[w0 + i];
    }
    __syncthreads();
    const int64_t a = it.v0 > s_pre[0] ? it.v0 : s_pre[0];
    const int64_t z = it.v1 < s_pre[wn] ? it.v1 : s_pre[wn];
    // wavefront w takes positions [g0, g0 + 64 U) of every kFoldWG U, lane l
    // the positions g0 + 64 u + l: each load instruction reads 64 consecutive slots
    const int lane = threadIdx.x & 63;
    for (int64_t g0 = a + (int64_t)(threadIdx.x >> 6) * 64 * U; g0 < z; g0 += (int64_t)kFoldWG * U) {
      const int64_t e0 = g0 + lane;
      int lo = 0, hi = wn - 1;  // last run r with s_pre[r] <= e0 (or <= g0 when e0 >= z)
      const int64_t key = e0 < z ? e0 : g0;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= key)
          lo = mid;
        else
          hi = mid - 1;
      }
      int r = lo;
      int64_t k[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = e0 + (int64_t)u * 64;
        k[u] = -1;
        if (e < z) {
          while (s_pre[r + 1] <= e) ++r;  // e < z <= s_pre[wn], so r stays below wn
          k[u] = s_base[r] + e;
        }
      }
      uint16_t d[U];
      unsigned long long x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        d[u] = k[u] >= 0 ? dstl[k[u]] : 0;
        x[u] = k[u] >= 0 ? vals[k[u]] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (x[u]) atomicAdd(&box[d[u]], x[u]);
    }
    __syncthreads();
  }
  const int64_t v0 = (int64_t)it.b << kPbDstShift;
  for (int i = threadIdx.x; i < (1 << kPbDstShift) && v0 + i < n; i += kFoldWG) {
    const unsigned long long x = box[i];
    if (!x) continue;
    if (it.whole)
      mb[v0 + i] = x;  // the only item of this bin
    else
      atomicAdd(&mb[v0 + i], x);
  }
}

}  // namespace

int pb_src_shift(size_t max_lds) {
  for (int s = kMaxSrcShift; s >= 10; --s)
    if (((size_t)8 << s) <= max_lds) return s;
  return 0;
}
int64_t pb_bins(int64_t n) { return (n + (1 << kPbDstShift) - 1) >> kPbDstShift; }
int64_t pb_tiles(int64_t n, int shift) { return (n + (1ll << shift) - 1) >> shift; }

hipError_t launch_pb_tile_edges(const void* off, bool off64, int64_t n, int shift, int64_t tiles, int64_t* te,
                                hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_pb_tile_edges<int64_t>, dim3(grid_for(tiles + 1)), dim3(kWG), 0, s, (const int64_t*)off, n,
                       shift, tiles, te);
  else
    hipLaunchKernelGGL(k_pb_tile_edges<int32_t>, dim3(grid_for(tiles + 1)), dim3(kWG), 0, s, (const int32_t*)off, n,
                       shift, tiles, te);
  return hipGetLastError();
}

hipError_t launch_pb_expand(const void* off, bool off64, int64_t n, int64_t m, const int32_t* tile_v, int64_t tile,
                            int64_t ntiles, int shift, uint16_t* srcl_csr, hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile + 2) * 8;
  if (off64)
    hipLaunchKernelGGL(k_pb_expand<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int64_t*)off, n, m,
                       tile_v, tile, shift, srcl_csr);
  else
    hipLaunchKernelGGL(k_pb_expand<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int32_t*)off, n, m,
                       tile_v, tile, shift, srcl_csr);
  return hipGetLastError();
}

hipError_t launch_pb_build(bool place, const int64_t* te, int64_t tiles, const int32_t* dst, int64_t m, int64_t chunk,
                           int64_t bins, int pass_bins, unsigned long long* cnt, const uint16_t* srcl_csr,
                           uint16_t* srcl, uint16_t* dstl, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (pass_bins < 1 || chunk < 1) return hipErrorInvalidValue;
  const int64_t grid = (m + chunk - 1) / chunk;
  const size_t lds = (size_t)pass_bins * (place ? 8 : 4);
  if (place)
    hipLaunchKernelGGL(k_pb_build<true>, dim3((unsigned)grid), dim3(kBuildWG), lds, s, te, tiles, dst, m, chunk, bins,
                       pass_bins, cnt, srcl_csr, srcl, dstl);
  else
    hipLaunchKernelGGL(k_pb_build<false>, dim3((unsigned)grid), dim3(kBuildWG), lds, s, te, tiles, dst, m, chunk, bins,
                       pass_bins, cnt, srcl_csr, srcl, dstl);
  return hipGetLastError();
}

hipError_t launch_pb_tables(const int64_t* starts, int64_t bins, int64_t tiles, int64_t fcap, int64_t* pre,
                            int64_t* base, int64_t* nitems, hipStream_t s) {
  hipLaunchKernelGGL(k_pb_tables, dim3(grid_for(bins)), dim3(kWG), 0, s, starts, bins, tiles, fcap, pre, base, nitems);
  return hipGetLastError();
}

hipError_t launch_pb_fold_items(const int64_t* pre, int64_t bins, int64_t tiles, int64_t fcap, const int64_t* item_off,
                                PbFoldItem* items, hipStream_t s) {
  hipLaunchKernelGGL(k_pb_fold_items, dim3(grid_for(bins)), dim3(kWG), 0, s, pre, bins, tiles, fcap, item_off, items);
  return hipGetLastError();
}

hipError_t launch_pb_spread(const PbSpreadItem* items, int64_t nitems, int64_t n, int shift, const uint16_t* srcl,
                            const unsigned long long* msg, unsigned long long* vals, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (shift < 10 || shift > kMaxSrcShift) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pb_spread, dim3((unsigned)nitems), dim3(kSpreadWG), (size_t)8 << shift, s, items, n, shift,
                     srcl, msg, vals);
  return hipGetLastError();
}

hipError_t launch_pb_fold(const PbFoldItem* items, int64_t nitems, int64_t tiles, int64_t n, const int64_t* pre,
                          const int64_t* base, const unsigned long long* vals, const uint16_t* dstl,
                          unsigned long long* mb, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const int64_t per = (nitems + 7) >> 3;
  hipLaunchKernelGGL(k_pb_fold, dim3((unsigned)(8 * per)), dim3(kFoldWG), 0, s, items, nitems, tiles, n, pre, base,
                     vals, dstl, mb);
  return hipGetLastError();
}

}  // namespace vc

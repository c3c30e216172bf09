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

// Merge-path walk over the CSR: calls f(u, v) for every edge of tile t.
template <class OffT, class F>
__device__ __forceinline__ void for_tile_edges(const OffT* __restrict__ off, const int32_t* __restrict__ dst, int64_t n,
                                               int64_t m, const int32_t* __restrict__ tile_v, int64_t tile,
                                               int64_t* s_off, F f) {
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
  for (int64_t e = j0 + threadIdx.x; e < j1; e += kWG) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    f(i0 + lo, (int64_t)dst[e]);
  }
}

template <class OffT>
__global__ __launch_bounds__(kWG) void k_pb_count(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                  int64_t n, int64_t m, const int32_t* __restrict__ tile_v,
                                                  int64_t tile, int shift, int64_t bins,
                                                  unsigned long long* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  for_tile_edges(off, dst, n, m, tile_v, tile, reinterpret_cast<int64_t*>(smem), [&](int64_t u, int64_t v) {
    atomicAdd(&cnt[(u >> shift) * bins + (v >> kPbDstShift)], 1ull);
  });
}

template <class OffT>
__global__ __launch_bounds__(kWG) void k_pb_fill(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                 int64_t n, int64_t m, const int32_t* __restrict__ tile_v,
                                                 int64_t tile, int shift, int64_t bins,
                                                 unsigned long long* __restrict__ cursor, uint16_t* __restrict__ srcl,
                                                 uint16_t* __restrict__ dstl) {
  extern __shared__ __align__(16) unsigned char smem[];
  for_tile_edges(off, dst, n, m, tile_v, tile, reinterpret_cast<int64_t*>(smem), [&](int64_t u, int64_t v) {
    const unsigned long long k = atomicAdd(&cursor[(u >> shift) * bins + (v >> kPbDstShift)], 1ull);
    srcl[k] = (uint16_t)(u & ((1 << shift) - 1));
    dstl[k] = (uint16_t)(v & ((1 << kPbDstShift) - 1));
  });
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

hipError_t launch_pb_count(const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                           const int32_t* tile_v, int64_t tile, int64_t ntiles, int shift, unsigned long long* cnt,
                           hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile + 2) * 8;
  const int64_t bins = pb_bins(n);
  if (off64)
    hipLaunchKernelGGL(k_pb_count<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int64_t*)off, dst, n, m,
                       tile_v, tile, shift, bins, cnt);
  else
    hipLaunchKernelGGL(k_pb_count<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int32_t*)off, dst, n, m,
                       tile_v, tile, shift, bins, cnt);
  return hipGetLastError();
}

hipError_t launch_pb_fill(const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, int shift, unsigned long long* cursor,
                          uint16_t* srcl, uint16_t* dstl, hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile + 2) * 8;
  const int64_t bins = pb_bins(n);
  if (off64)
    hipLaunchKernelGGL(k_pb_fill<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int64_t*)off, dst, n, m,
                       tile_v, tile, shift, bins, cursor, srcl, dstl);
  else
    hipLaunchKernelGGL(k_pb_fill<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int32_t*)off, dst, n, m,
                       tile_v, tile, shift, bins, cursor, srcl, dstl);
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

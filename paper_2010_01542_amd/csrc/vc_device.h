// Device helpers shared by the kernel translation units of libvc.
#pragma once

#include "vc_internal.h"

namespace vc {
namespace dev {

__device__ __forceinline__ unsigned lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if ((int)lane_id() >= o) x += y;
  }
  return x;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Exclusive scan over the kWG threads of a workgroup; *total gets the sum.
// Every thread of the workgroup must call it.
template <class T>
__device__ __forceinline__ T block_excl_scan(T x, T* total) {
  __shared__ T s_w[kWG / 64];
  const T inc = wave_incl_scan(x);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[w] = inc;
  __syncthreads();
  T before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWG / 64; ++i) {
    const T v = s_w[i];
    if (i < w) before += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

template <class T>
__device__ __forceinline__ T block_sum(T x) {
  __shared__ T s_w[kWG / 64];
  x = wave_sum(x);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  T tot = 0;
#pragma unroll
  for (int i = 0; i < kWG / 64; ++i) tot += s_w[i];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ int64_t gid() { return (int64_t)blockIdx.x * kWG + threadIdx.x; }

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s < a ? kInf : s;
}

// ------------------------------------------------- PageRank messages and sums
// Sums (mailboxes) S are uint64 multiples of 2^-62 (exact, associative; ranks
// and their sums never exceed 1) or binary32 (float atomics).  Messages M
// are uint64 multiples of 2^-62 or binary32; a binary32 message summed in
// fixed point is scaled by 2^62 (exact) and rounded to an integer, so its
// sum is still exact and order-independent.
constexpr double kFixScale = 4611686018427387904.0;  // 2^62
constexpr double kFixInv = 1.0 / 4611686018427387904.0;

template <class M, class S>
__device__ __forceinline__ S msg_to_sum(M m) {
  if constexpr (sizeof(M) == 4 && sizeof(S) == 8) {
    // m = f * 2^(e - 150) with the 24-bit significand f (0 <= m <= 1):
    // m * 2^62 = f * 2^(e - 88), exact for m >= 2^-38 and truncated below
    // (an error under 2^-62 per message).  Zero and subnormal messages
    // shift out entirely.  Branch-free, so that a caller's loads are not
    // split by control flow.
    const uint32_t b = __float_as_uint(m);
    const int sh = (int)(b >> 23) - 88;
    const unsigned long long f = (unsigned long long)((b & 0x7fffffu) | 0x800000u);
    return sh >= 0 ? f << sh : f >> (-sh < 63 ? -sh : 63);
  } else {
    return (S)m;
  }
}

// The message a vertex of out-degree deg and rank r sends on each edge.
template <class M, class S>
__device__ __forceinline__ M rank_msg(double r, int64_t deg) {
  if (deg <= 0) return M(0);
  if constexpr (sizeof(M) == 8)
    return __double2ull_rn(r / (double)deg * kFixScale);
  else if constexpr (sizeof(S) == 8)
    return (float)(r / (double)deg);  // one rounding
  else
    return (float)r / (float)deg;
}

// Byte offset of the next LDS sub-array: rounded up to 16 bytes.
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// A merge-path tile of the merged (edge, item-end) sequence: workgroup
// blockIdx.x owns merged positions [t * tile, (t + 1) * tile), i.e. the
// edges j0 .. j1 - 1 of items i0 .. i0 + cnt - 1 (tile_v from the partition
// kernel).  Returns whether the tile holds any edge.
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

// Owner (local item index) of edge e: last x with s_off[x] <= e.
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

inline unsigned grid_for(int64_t count) { return (unsigned)((count + kWG - 1) / kWG); }

// Grid of a grid-stride loop over `count` items.  A dispatch counts its
// work-items in 32 bits, so one thread per item fails beyond 2^32 items;
// 2^20 workgroups stay far below that and still give every CU thousands of
// waves.
inline unsigned grid_stride_for(int64_t count) {
  const int64_t g = (count + kWG - 1) / kWG;
  return (unsigned)(g < (1 << 20) ? g : (1 << 20));
}
__device__ __forceinline__ int64_t grid_threads() { return (int64_t)gridDim.x * blockDim.x; }

}  // namespace dev
}  // namespace vc

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

// Byte offset of the next LDS sub-array: rounded up to 16 bytes.
__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

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

// Hot-first vertex relabelling (paper, Section IV: the memory accesses of a
// broadcast go to arbitrary vertices, but some vertices are accessed far more
// often than others; grouping the frequently accessed data lets cache lines
// carry mostly useful bytes).
//
// Vertices are ordered by degree class, highest first, where the class of v
// is floor(log2(outdeg(v) + indeg(v) + 1)); ties keep the input order (a
// stable partition), so the relabelling is deterministic.  With power-law
// degrees the few vertices that receive and send most messages then occupy a
// short prefix of every per-vertex array, which stays in L2.
//
// The relabelled CSR keeps every edge (parallel edges and self-loops
// included) with its weight; each row keeps its input edge order.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

constexpr int kClasses = 34;  // floor(log2(x + 1)) for x < 2^33, shifted so the hottest class is 0

__device__ __forceinline__ int degree_class(int64_t deg_sum) {
  const int lg = 63 - __clzll((unsigned long long)(deg_sum + 1));  // floor(log2(deg + 1)), 0..33
  return (kClasses - 1) - lg;                                       // hottest first
}

// hist[c * nblocks + b] = number of vertices of class c in block b (kWG vertices per block)
template <class OffT>
__global__ __launch_bounds__(kWG) void k_class_hist(const OffT* __restrict__ off,
                                                    const unsigned long long* __restrict__ indeg, int64_t n,
                                                    int64_t nblocks, int64_t* __restrict__ hist) {
  __shared__ int s_cnt[kClasses];
  for (int c = threadIdx.x; c < kClasses; c += kWG) s_cnt[c] = 0;
  __syncthreads();
  const int64_t v = gid();
  if (v < n) {
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v] + (int64_t)indeg[v];
    atomicAdd(&s_cnt[degree_class(d)], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kClasses; c += kWG) hist[(int64_t)c * nblocks + blockIdx.x] = s_cnt[c];
}

// Stable scatter: new id = (class, block) base + rank among the block's
// vertices of the same class with a smaller index.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_class_scatter(const OffT* __restrict__ off,
                                                       const unsigned long long* __restrict__ indeg, int64_t n,
                                                       int64_t nblocks, const int64_t* __restrict__ base,
                                                       int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
  __shared__ int s_wave[kWG / 64][kClasses];
  const int64_t v = gid();
  int c = -1;
  if (v < n) {
    const int64_t d = (int64_t)off[v + 1] - (int64_t)off[v] + (int64_t)indeg[v];
    c = degree_class(d);
  }
  const int w = threadIdx.x >> 6;
  const int lane = (int)lane_id();
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int my_rank = 0;
  for (int k = 0; k < kClasses; ++k) {
    const unsigned long long mask = __ballot(c == k);
    if (lane == 0) s_wave[w][k] = __popcll(mask);
    if (c == k) my_rank = __popcll(mask & below);
  }
  __syncthreads();
  if (v < n) {
    int before = 0;
    for (int ww = 0; ww < w; ++ww) before += s_wave[ww][c];
    const int64_t nv = base[(int64_t)c * nblocks + blockIdx.x] + before + my_rank;
    perm[v] = (int32_t)nv;
    inv[nv] = (int32_t)v;
  }
}

// new_deg[x] = out-degree of the old vertex inv[x] (written into P[x], scanned later)
template <class OffT>
__global__ __launch_bounds__(kWG) void k_relabel_degrees(const OffT* __restrict__ off, const int32_t* __restrict__ inv,
                                                         int64_t n, int64_t* __restrict__ P) {
  const int64_t x = gid();
  if (x < n) {
    const int64_t u = inv[x];
    P[x] = (int64_t)off[u + 1] - (int64_t)off[u];
  }
}

// Copies every edge of old row inv[x] to new row x, mapping targets through
// perm.  Merge-path tiles over the new offsets split long rows.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_relabel_edges(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                       const uint32_t* __restrict__ w, const int64_t* __restrict__ noff,
                                                       const int32_t* __restrict__ inv, const int32_t* __restrict__ perm,
                                                       int64_t n, int64_t m, const int32_t* __restrict__ tile_v,
                                                       int64_t tile, int32_t* __restrict__ ndst,
                                                       uint32_t* __restrict__ nw) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);     // new offsets, cnt + 1
  int64_t* s_old = s_off + tile + 2;                      // old row start - new row start, cnt
  for (int x = threadIdx.x; x <= cnt; x += kWG) s_off[x] = noff[i0 + x];
  for (int x = threadIdx.x; x < cnt; x += kWG) s_old[x] = (int64_t)off[inv[i0 + x]] - noff[i0 + x];
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
    const int64_t oe = e + s_old[lo];
    ndst[e] = perm[dst[oe]];
    if (w) nw[e] = w[oe];
  }
}

// out[u] = vals[perm[u]] (4-byte values)
__global__ __launch_bounds__(kWG) void k_unpermute(const uint32_t* __restrict__ vals, const int32_t* __restrict__ perm,
                                                   int64_t n, int64_t stride, uint32_t* __restrict__ out) {
  const int64_t u = gid();
  if (u < n) out[u] = vals[(int64_t)perm[u] * stride];
}

template <class OffT>
__global__ __launch_bounds__(kWG) void k_union_member(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                      const uint32_t* __restrict__ w, int64_t n, int64_t m,
                                                      int64_t vbase, int64_t ebase, int weight_mode,
                                                      int64_t* __restrict__ u_off, int32_t* __restrict__ u_dst,
                                                      uint32_t* __restrict__ u_w) {
  const int64_t stride = (int64_t)gridDim.x * kWG;
  for (int64_t v = gid(); v < n; v += stride) u_off[vbase + v] = ebase + (int64_t)off[v];
  for (int64_t e = gid(); e < m; e += stride) {
    u_dst[ebase + e] = (int32_t)(vbase + dst[e]);
    u_w[ebase + e] = weight_mode == 1 ? w[e] : (weight_mode == 2 ? 1u : 0u);
  }
}

__global__ __launch_bounds__(kWG) void k_union_init(int64_t n, int64_t vbase, int mode, int64_t source,
                                                    uint32_t* __restrict__ init) {
  const int64_t v = gid();
  if (v < n) init[vbase + v] = mode == 0 ? (uint32_t)v : (v == source ? 0u : 0xFFFFFFFFu);
}

__global__ __launch_bounds__(kWG) void k_permute(const uint32_t* __restrict__ vals, const int32_t* __restrict__ perm,
                                                 int64_t n, uint32_t* __restrict__ out) {
  const int64_t u = gid();
  if (u < n) out[perm[u]] = vals[u];
}

}  // namespace

hipError_t launch_union_member(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n, int64_t m,
                               int64_t vbase, int64_t ebase, int weight_mode, int64_t* u_off, int32_t* u_dst,
                               uint32_t* u_w, hipStream_t s) {
  const int64_t work = n > m ? n : m;
  const int64_t blocks = (work + kWG - 1) / kWG;
  const unsigned g = (unsigned)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  if (off64)
    hipLaunchKernelGGL(k_union_member<int64_t>, dim3(g), dim3(kWG), 0, s, (const int64_t*)off, dst, w, n, m, vbase,
                       ebase, weight_mode, u_off, u_dst, u_w);
  else
    hipLaunchKernelGGL(k_union_member<int32_t>, dim3(g), dim3(kWG), 0, s, (const int32_t*)off, dst, w, n, m, vbase,
                       ebase, weight_mode, u_off, u_dst, u_w);
  return hipGetLastError();
}

hipError_t launch_union_init(int64_t n, int64_t vbase, int mode, int64_t source, uint32_t* init, hipStream_t s) {
  hipLaunchKernelGGL(k_union_init, dim3(grid_for(n)), dim3(kWG), 0, s, n, vbase, mode, source, init);
  return hipGetLastError();
}

hipError_t launch_permute(const uint32_t* vals, const int32_t* perm, int64_t n, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_permute, dim3(grid_for(n)), dim3(kWG), 0, s, vals, perm, n, out);
  return hipGetLastError();
}

int relabel_classes() { return kClasses; }

hipError_t launch_relabel_perm(const void* off, bool off64, const unsigned long long* indeg, int64_t n,
                               int64_t* hist_scratch, int64_t* scan_blocks, int32_t* perm, int32_t* inv,
                               hipStream_t s) {
  const int64_t nblocks = (n + kWG - 1) / kWG;
  if (off64)
    hipLaunchKernelGGL(k_class_hist<int64_t>, dim3((unsigned)nblocks), dim3(kWG), 0, s, (const int64_t*)off, indeg, n,
                       nblocks, hist_scratch);
  else
    hipLaunchKernelGGL(k_class_hist<int32_t>, dim3((unsigned)nblocks), dim3(kWG), 0, s, (const int32_t*)off, indeg, n,
                       nblocks, hist_scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_exclusive_scan(hist_scratch, (int64_t)kClasses * nblocks, scan_blocks, s);
  if (e != hipSuccess) return e;
  if (off64)
    hipLaunchKernelGGL(k_class_scatter<int64_t>, dim3((unsigned)nblocks), dim3(kWG), 0, s, (const int64_t*)off, indeg,
                       n, nblocks, hist_scratch, perm, inv);
  else
    hipLaunchKernelGGL(k_class_scatter<int32_t>, dim3((unsigned)nblocks), dim3(kWG), 0, s, (const int32_t*)off, indeg,
                       n, nblocks, hist_scratch, perm, inv);
  return hipGetLastError();
}

hipError_t launch_relabel_degrees(const void* off, bool off64, const int32_t* inv, int64_t n, int64_t* P,
                                  hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_relabel_degrees<int64_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, inv, n, P);
  else
    hipLaunchKernelGGL(k_relabel_degrees<int32_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, inv, n, P);
  return hipGetLastError();
}

hipError_t launch_relabel_edges(const void* off, bool off64, const int32_t* dst, const uint32_t* w,
                                const int64_t* noff, const int32_t* inv, const int32_t* perm, int64_t n, int64_t m,
                                const int32_t* tile_v, int64_t tile, int64_t ntiles, int32_t* ndst, uint32_t* nw,
                                hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile + 2) * 8 + (size_t)(tile + 1) * 8;
  if (off64)
    hipLaunchKernelGGL(k_relabel_edges<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int64_t*)off, dst, w,
                       noff, inv, perm, n, m, tile_v, tile, ndst, nw);
  else
    hipLaunchKernelGGL(k_relabel_edges<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int32_t*)off, dst, w,
                       noff, inv, perm, n, m, tile_v, tile, ndst, nw);
  return hipGetLastError();
}

hipError_t launch_unpermute(const uint32_t* vals, int64_t stride, const int32_t* perm, int64_t n, uint32_t* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute, dim3(grid_for(n)), dim3(kWG), 0, s, vals, perm, n, stride, out);
  return hipGetLastError();
}

}  // namespace vc

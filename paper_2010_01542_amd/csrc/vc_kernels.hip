// HIP kernels of the vertex-centric superstep for CDNA4 (gfx950).
//
// One superstep = broadcast along CSR out-edges + combine into per-vertex
// mailboxes (paper, Sections I and III), followed by the vertex update.
//
// Layout (paper, Section IV: keep the fields touched per message together and
// apart from everything else):
//   PageRank  contrib[N] f32 (the message each vertex sends: rank / outdeg)
//             mb[N]      f32 (sum mailbox, neutral 0)
//   CC/SSSP   vm[N]      (value, mailbox) u32 pairs: the per-target check,
//                        the combine and the update all touch one 8-byte slot
//             bitmap     one bit per vertex: "value improved this superstep"
//
// Work distribution (paper, Section V): either one thread per active vertex,
// or merge-path tiles that give every workgroup the same number of items of
// the merged (edge, vertex-end) sequence, so hubs are split across
// workgroups and runs of edge-less vertices cost one item each.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

// ------------------------------------------------------------------ generic

__global__ __launch_bounds__(kWG) void k_fill_u32(uint32_t* __restrict__ p, int64_t count, uint32_t value) {
  for (int64_t i = gid(); i < count; i += grid_threads()) p[i] = value;
}

__global__ void k_zero_counters(Counters* c) {
  if (threadIdx.x == 0) {
    c->active = 0;
    c->listed = 0;
    c->edges = 0;
    c->flags = 0;
  }
}

// CSR checks: off[0] = 0, off[n] = m, non-decreasing, targets in range.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_validate(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                  int64_t n, int64_t m, Counters* ctr) {
  const int64_t i = gid();
  unsigned long long bad = 0;
  if (i == 0) {
    if ((int64_t)off[0] != 0) bad |= 1;
    if ((int64_t)off[n] != m) bad |= 2;
  }
  if (i < n && (int64_t)off[i + 1] < (int64_t)off[i]) bad |= 4;
  for (int64_t e = i; e < m; e += (int64_t)gridDim.x * kWG) {
    const int32_t d = dst[e];
    if (d < 0 || (int64_t)d >= n) bad |= 8;
  }
  if (bad) atomicOr(&ctr->flags, bad);
}

// Symmetry check of a graph declared symmetric: the multiset of its edges
// (u, v, w) must equal that of its reversed edges (v, u, w).  Each edge adds
// h(u, v, w) - h(v, u, w) to a wrapping 64-bit sum, for two independent
// hashes; both sums are zero for a symmetric graph, and an asymmetric one
// leaves both at zero only by a hash collision.  The mixing step is the
// 64-bit finaliser of MurmurHash3 (A. Appleby).  One wavefront per 64
// consecutive vertices; its lanes read the offsets coalesced and then stride
// over each vertex's edges.
__device__ __forceinline__ unsigned long long fmix64(unsigned long long k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ void sym_terms(unsigned long long u, unsigned long long v, unsigned long long w,
                                          unsigned long long* a, unsigned long long* b) {
  const unsigned long long f = (u << 32) | v, r = (v << 32) | u;
  const unsigned long long sw = w * 0x9e3779b97f4a7c15ull;
  *a += fmix64(f ^ sw) - fmix64(r ^ sw);
  *b += fmix64(fmix64(f + 0x632be59bd9b4e019ull) ^ w) - fmix64(fmix64(r + 0x632be59bd9b4e019ull) ^ w);
}

template <class OffT>
__global__ __launch_bounds__(kWG) void k_sym_hash(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                  const uint32_t* __restrict__ w, int64_t n,
                                                  unsigned long long* __restrict__ acc) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t nwaves = grid_threads() >> 6;
  unsigned long long a = 0, b = 0;
  for (int64_t v0 = (gid() >> 6) * 64; v0 < n; v0 += nwaves * 64) {
    const int64_t mv = v0 + lane;
    const long long me0 = mv < n ? (long long)off[mv] : 0, me1 = mv < n ? (long long)off[mv + 1] : 0;
    const int cnt = n - v0 < 64 ? (int)(n - v0) : 64;
    for (int i = 0; i < cnt; ++i) {
      const long long e0 = __shfl(me0, i, 64), e1 = __shfl(me1, i, 64);
      for (long long e = e0 + lane; e < e1; e += 64)
        sym_terms((unsigned long long)(v0 + i), (unsigned long long)(uint32_t)dst[e], w ? w[e] : 1u, &a, &b);
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0 && (a | b)) {
    atomicAdd(&acc[0], a);
    atomicAdd(&acc[1], b);
  }
}

// tile_v[t] = #{x in [0, items) : P[x+1] + x + 1 <= k}, k = min(t * tile, total):
// the number of vertex-ends that precede merged position k when edge e of
// item x sits at position e + x and the end of item x at P[x+1] + x.
template <class PT>
__device__ __forceinline__ int32_t mp_tile_start(const PT* __restrict__ P, int64_t items, int64_t total, int64_t tile,
                                                 int64_t t) {
  const int64_t k = t * tile < total ? t * tile : total;
  int64_t lo = 0, hi = items;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)P[mid + 1] + mid + 1 <= k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (int32_t)lo;
}

template <class PT>
__global__ __launch_bounds__(kWG) void k_mp_partition(const PT* __restrict__ P, int64_t items, int64_t total,
                                                      int64_t tile, int64_t ntiles, int32_t* __restrict__ tile_v) {
  const int64_t t = gid();
  if (t > ntiles) return;
  tile_v[t] = mp_tile_start(P, items, total, tile, t);
}

// The partition of a device-driven loop's broadcast list, sized from the
// loop state (grid-stride over at most max_tiles + 1 tile starts).
__global__ __launch_bounds__(kWG) void k_loop_partition(const int64_t* __restrict__ P, int64_t tile,
                                                        int64_t max_tiles, int32_t* __restrict__ tile_v,
                                                        const LoopState* __restrict__ loop) {
  if (loop->done || loop->mode != VC_SCHED_EDGE) return;
  const int64_t items = loop->listed, total = items + loop->edges;
  int64_t ntiles = (total + tile - 1) / tile;
  if (ntiles > max_tiles) ntiles = max_tiles;  // cannot happen for a valid loop state; keeps writes in bounds
  for (int64_t t = gid(); t <= ntiles; t += grid_threads()) tile_v[t] = mp_tile_start(P, items, total, tile, t);
}

// ------------------------------------------------------------------ PageRank
// Three forms of the sum combiner (message type M, mailbox type S):
//  * fixed point (default, M = S = uint64 multiples of 2^-62): integer
//    addition is exact and associative, so a mailbox holds the exact sum of
//    its messages in any arrival order; the vertex update runs in binary64
//    and only the final result is rounded to binary32;
//  * binary32 messages, fixed-point sums (M = float, S = uint64): each
//    message rounded once to binary32, then summed exactly as above (half
//    the message bytes, still order-independent);
//  * binary32 (M = S = float): float messages combined with hardware float
//    atomics (rounding at every combination, in arrival order).

template <class S>
__device__ __forceinline__ void sum_combine(S* __restrict__ mb, int32_t d, S x);
template <>
__device__ __forceinline__ void sum_combine<float>(float* __restrict__ mb, int32_t d, float x) {
  unsafeAtomicAdd(&mb[d], x);
}
template <>
__device__ __forceinline__ void sum_combine<unsigned long long>(unsigned long long* __restrict__ mb, int32_t d,
                                                                unsigned long long x) {
  atomicAdd(&mb[d], x);
}

template <class OffT, class M, class S>
__global__ __launch_bounds__(kWG) void k_pr_init(const OffT* __restrict__ off, int64_t n, double r0, int64_t source,
                                                 M* __restrict__ contrib, S* __restrict__ mb,
                                                 float* __restrict__ out_if_t0) {
  const int64_t v = gid();
  if (v >= n) return;
  const double r = source >= 0 ? (v == source ? 1.0 : 0.0) : r0;
  if (out_if_t0) {
    out_if_t0[v] = (float)r;
    return;
  }
  const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
  contrib[v] = rank_msg<M, S>(r, deg);
  mb[v] = S(0);
}

// Hub targets (paper, Section III: combinations contend at the recipient's
// mailbox, most at high in-degree vertices).  A push workgroup combines the
// messages addressed to targets 0 .. nhub-1 in an LDS table (after the
// default hot-first relabelling these are the highest-degree vertices) and
// flushes every touched entry with one global combination at its end;
// nhub = 0 sends every message to its global mailbox.  The table is
// kHubBytes of LDS; min tables start at the neutral value, sum tables at 0.
template <class S>
__device__ __forceinline__ void hub_init(S* __restrict__ s_hub, int nhub, S neutral) {
  for (int x = threadIdx.x; x < nhub; x += kWG) s_hub[x] = neutral;
}

template <class S>
__device__ __forceinline__ void hub_flush_sum(const S* __restrict__ s_hub, int nhub, S* __restrict__ mb) {
  for (int x = threadIdx.x; x < nhub; x += kWG) {
    const S c = s_hub[x];
    if (c != S(0)) sum_combine<S>(mb, x, c);
  }
}

// Vertex-per-thread broadcast: thread v sends contrib[v] along its out-edges.
template <class OffT, class M, class S>
__global__ __launch_bounds__(kWG) void k_pr_scatter_vertex(const OffT* __restrict__ off,
                                                           const int32_t* __restrict__ dst, int64_t n,
                                                           const M* __restrict__ contrib, S* __restrict__ mb,
                                                           int nhub) {
  extern __shared__ __align__(16) unsigned char smem[];
  S* s_hub = reinterpret_cast<S*>(smem);
  if (nhub) {  // uniform over the grid
    hub_init<S>(s_hub, nhub, S(0));
    __syncthreads();
  }
  const int64_t v = gid();
  const S c = v < n ? msg_to_sum<M, S>(contrib[v]) : S(0);
  if (c != S(0)) {  // adding zero changes no sum (PPR vertices the walk has not reached)
    const int64_t e1 = (int64_t)off[v + 1];
    for (int64_t e = (int64_t)off[v]; e < e1; ++e) {
      const int32_t d = dst[e];
      if (d < nhub)
        atomicAdd(&s_hub[d], c);
      else
        sum_combine<S>(mb, d, c);
    }
  }
  if (nhub) {
    __syncthreads();
    hub_flush_sum<S>(s_hub, nhub, mb);
  }
}

// Merge-path broadcast: workgroup t owns merged positions [t*tile, (t+1)*tile).
template <class OffT, class M, class S>
__global__ __launch_bounds__(kWG) void k_pr_scatter_mp(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                       int64_t n, int64_t m, const int32_t* __restrict__ tile_v,
                                                       int64_t tile, const M* __restrict__ contrib,
                                                       S* __restrict__ mb, int nhub) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;  // only vertex-ends in this tile (uniform over the workgroup)
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);  // vertices i0..ilast own the tile's edges
  S* s_val = reinterpret_cast<S*>(smem);                                         // tile + 1
  OffT* s_off = reinterpret_cast<OffT*>(smem + align16((tile + 1) * sizeof(S)));  // tile + 2
  S* s_hub = reinterpret_cast<S*>(smem + align16((tile + 1) * sizeof(S)) + align16((tile + 2) * sizeof(OffT)));
  for (int x = threadIdx.x; x <= cnt; x += kWG) s_off[x] = off[i0 + x];
  for (int x = threadIdx.x; x < cnt; x += kWG) s_val[x] = msg_to_sum<M, S>(contrib[i0 + x]);
  hub_init<S>(s_hub, nhub, S(0));
  __syncthreads();
  for (int64_t e = j0 + threadIdx.x; e < j1; e += kWG) {
    int lo = 0, hi = cnt - 1;  // owner = last x with s_off[x] <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((int64_t)s_off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    const S c = s_val[lo];
    const int32_t d = dst[e];
    if (c != S(0)) {
      if (d < nhub)
        atomicAdd(&s_hub[d], c);
      else
        sum_combine<S>(mb, d, c);
    }
  }
  if (nhub) {
    __syncthreads();
    hub_flush_sum<S>(s_hub, nhub, mb);
  }
}

// rank = teleport + d * (sum of messages); reset the mailbox; next message.
// With the blocked form's bin kinds, a bin without in-edges has sum zero
// (its mailboxes are not read) and only split bins' mailboxes are reset
// (the fold stores every mailbox of a one-item bin).
// keep_empty: the messages of vertices in bins without in-edges are already
// in contrib and stay as they are (such a vertex's rank is the teleport
// term at every update, so its message is the same from the first update
// on): the update skips those bins (a workgroup's vertices share one bin).
// Four consecutive vertices per thread (one bin, since bins are aligned to
// 4096 vertices): mailboxes and messages move as 16-byte vectors, a quarter
// of the load and store instructions for the texture addresser (the
// offsets are read one by one, since a borrowed offset array need not be
// 16-byte aligned; so are the final ranks when the caller's buffer is not).
// The last n % 4 vertices go one per thread.
template <class S>
struct Vec4;
template <>
struct Vec4<unsigned long long> {
  __device__ __forceinline__ static void load(const unsigned long long* p, unsigned long long* x) {
    const ulonglong2 a = reinterpret_cast<const ulonglong2*>(p)[0], b = reinterpret_cast<const ulonglong2*>(p)[1];
    x[0] = a.x; x[1] = a.y; x[2] = b.x; x[3] = b.y;
  }
  __device__ __forceinline__ static void store(unsigned long long* p, const unsigned long long* x) {
    reinterpret_cast<ulonglong2*>(p)[0] = make_ulonglong2(x[0], x[1]);
    reinterpret_cast<ulonglong2*>(p)[1] = make_ulonglong2(x[2], x[3]);
  }
};
template <>
struct Vec4<float> {
  __device__ __forceinline__ static void load(const float* p, float* x) {
    const float4 a = reinterpret_cast<const float4*>(p)[0];
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
  }
  __device__ __forceinline__ static void store(float* p, const float* x) {
    reinterpret_cast<float4*>(p)[0] = make_float4(x[0], x[1], x[2], x[3]);
  }
};

template <class OffT, class M, class S>
__global__ __launch_bounds__(kWG) void k_pr_apply4(const OffT* __restrict__ off, int64_t n, double teleport,
                                                   double damping, int64_t source, S* __restrict__ mb,
                                                   M* __restrict__ contrib, float* __restrict__ out, int last,
                                                   const uint8_t* __restrict__ kinds, int keep_empty) {
  const int64_t v0 = gid() * 4;
  if (v0 >= n) return;
  if (v0 + 4 > n) {  // the tail, one vertex at a time
    for (int64_t v = v0; v < n; ++v) {
      const int kind = kinds ? kinds[v >> kPbDstShift] : kBinSplit;
      if (keep_empty && kind == kBinEmpty) continue;
      const S x = kind != kBinEmpty ? mb[v] : S(0);
      const double tele = source >= 0 ? (v == source ? teleport : 0.0) : teleport;
      double r;
      if constexpr (sizeof(S) == 8)
        r = fma(damping, (double)x * kFixInv, tele);
      else
        r = (double)fmaf((float)damping, x, (float)tele);
      if (last) {
        out[v] = (float)r;
        continue;
      }
      if (kind == kBinSplit) mb[v] = S(0);
      contrib[v] = rank_msg<M, S>(r, (int64_t)off[v + 1] - (int64_t)off[v]);
    }
    return;
  }
  const int kind = kinds ? kinds[v0 >> kPbDstShift] : kBinSplit;
  if (keep_empty && kind == kBinEmpty) return;
  S x[4] = {S(0), S(0), S(0), S(0)};
  if (kind != kBinEmpty) Vec4<S>::load(mb + v0, x);
  double r[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double tele = source >= 0 ? (v0 + j == source ? teleport : 0.0) : teleport;
    if constexpr (sizeof(S) == 8)
      r[j] = fma(damping, (double)x[j] * kFixInv, tele);
    else
      r[j] = (double)fmaf((float)damping, x[j], (float)tele);
  }
  if (last) {
    if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {  // uniform: the caller's buffer may be 4-byte aligned only
      reinterpret_cast<float4*>(out + v0)[0] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[v0 + j] = (float)r[j];
    }
    return;
  }
  if (kind == kBinSplit) {
    const S z[4] = {S(0), S(0), S(0), S(0)};
    Vec4<S>::store(mb + v0, z);
  }
  int64_t o[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) o[j] = (int64_t)off[v0 + j];
  M msg[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) msg[j] = rank_msg<M, S>(r[j], o[j + 1] - o[j]);
  Vec4<M>::store(contrib + v0, msg);
}

// ------------------------------------------------------------------ CC / SSSP

__global__ __launch_bounds__(kWG) void k_min_init(int kind, int64_t n, int64_t source, const int32_t* __restrict__ ids,
                                                  uint2* __restrict__ vm) {
  const int64_t v = gid();
  if (v >= n) return;
  const uint32_t val = kind == kCC ? (uint32_t)(ids ? (int64_t)ids[v] : v) : (v == source ? 0u : kInf);
  vm[v] = make_uint2(val, kInf);
}

template <class OffT>
__global__ void k_min_seed_source(const OffT* __restrict__ off, int64_t source, int32_t* __restrict__ fq,
                                  int64_t* __restrict__ P, uint32_t* __restrict__ active) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    fq[0] = (int32_t)source;
    P[0] = 0;
    P[1] = (int64_t)off[source + 1] - (int64_t)off[source];
    active[source >> 5] |= 1u << (source & 31);
  }
}

template <int KIND>
__device__ __forceinline__ uint32_t message(uint32_t val, const uint32_t* __restrict__ w, int64_t pos) {
  if (KIND == kCC) return val;
  if (KIND == kSsspUnit) return sat_add(val, 1u);
  return sat_add(val, w[pos]);
}

// Min combine into target d.  Messages that cannot lower d's value are
// dropped; the mailbox is read first and the atomic skipped when it cannot
// win (the skip of a no-op combination, paper Section III, Figure 1).  The
// message that first lowers an untouched mailbox marks d as improved.
template <bool TBA>
__device__ __forceinline__ void relax(uint2* __restrict__ vm, uint32_t* __restrict__ bitmap, int32_t d,
                                      uint32_t msg) {
  const uint2 cur = vm[d];
  if (msg < cur.x && (!TBA || msg < cur.y)) {
    const uint32_t old = atomicMin(&reinterpret_cast<uint32_t*>(vm)[2 * (int64_t)d + 1], msg);
    if (old == kInf) atomicOr(&bitmap[d >> 5], 1u << (d & 31));
  }
}

// A hub entry's minimum goes through the same filter and atomic as a
// single message would.
template <bool TBA>
__device__ __forceinline__ void hub_flush_min(const uint32_t* __restrict__ s_hub, int nhub, uint2* __restrict__ vm,
                                              uint32_t* __restrict__ bitmap) {
  for (int x = threadIdx.x; x < nhub; x += kWG) {
    const uint32_t msg = s_hub[x];
    if (msg != kInf) relax<TBA>(vm, bitmap, x, msg);
  }
}

template <class OffT, int KIND, bool LIST, bool TBA>
__global__ __launch_bounds__(kWG) void k_min_scatter_vertex(const OffT* __restrict__ off,
                                                            const int32_t* __restrict__ dst,
                                                            const uint32_t* __restrict__ w, int64_t items,
                                                            const int32_t* __restrict__ fq, uint2* __restrict__ vm,
                                                            uint32_t* __restrict__ bitmap, int nhub) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* s_hub = reinterpret_cast<uint32_t*>(smem);
  if (nhub) {  // uniform over the grid
    hub_init<uint32_t>(s_hub, nhub, kInf);
    __syncthreads();
  }
  const int64_t x = gid();
  if (x < items) {
    const int64_t v = LIST ? (int64_t)fq[x] : x;
    const uint32_t val = vm[v].x;
    const int64_t e1 = (int64_t)off[v + 1];
    for (int64_t e = (int64_t)off[v]; e < e1; ++e) {
      const int32_t d = dst[e];
      const uint32_t msg = message<KIND>(val, w, e);
      if (d < nhub)
        atomicMin(&s_hub[d], msg);
      else
        relax<TBA>(vm, bitmap, d, msg);
    }
  }
  if (nhub) {
    __syncthreads();
    hub_flush_min<TBA>(s_hub, nhub, vm, bitmap);
  }
}

// Merge-path broadcast for the min programs.  Dense mode: items are all
// vertices and P is the CSR offsets.  List mode: items are the broadcast
// list fq and P its degree prefix; item x's edges start at off[fq[x]].
template <class PT, class OffT, int KIND, bool LIST, bool TBA>
__device__ __forceinline__ void min_scatter_mp_tile(int64_t t, unsigned char* smem, const OffT* __restrict__ off,
                                                    const int32_t* __restrict__ dst,
                                                    const uint32_t* __restrict__ w, int64_t items, int64_t total,
                                                    const PT* __restrict__ P, const int32_t* __restrict__ fq,
                                                    const int32_t* __restrict__ tile_v, int64_t tile,
                                                    uint2* __restrict__ vm, uint32_t* __restrict__ bitmap, int nhub) {
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < total) ? k0 + tile : total;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < items ? i1 : items - 1;
  const int cnt = (int)(ilast - i0 + 1);
  int64_t* s_p = reinterpret_cast<int64_t*>(smem);  // tile + 2 entries
  int64_t* s_base = s_p + tile + 2;                 // tile + 1 entries (list mode; 8-byte aligned)
  uint32_t* s_val = reinterpret_cast<uint32_t*>(LIST ? s_base + tile + 1 : s_base);  // tile + 1 entries
  uint32_t* s_hub = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(s_val) + align16((tile + 1) * 4));
  for (int x = threadIdx.x; x <= cnt; x += kWG) s_p[x] = (int64_t)P[i0 + x];
  for (int x = threadIdx.x; x < cnt; x += kWG) {
    const int64_t v = LIST ? (int64_t)fq[i0 + x] : i0 + x;
    if (LIST) s_base[x] = (int64_t)off[v] - (int64_t)P[i0 + x];
    s_val[x] = vm[v].x;
  }
  hub_init<uint32_t>(s_hub, nhub, kInf);
  __syncthreads();
  for (int64_t j = j0 + threadIdx.x; j < j1; j += kWG) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_p[mid] <= j)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t pos = LIST ? j + s_base[lo] : j;
    const int32_t d = dst[pos];
    const uint32_t msg = message<KIND>(s_val[lo], w, pos);
    if (d < nhub)
      atomicMin(&s_hub[d], msg);
    else
      relax<TBA>(vm, bitmap, d, msg);
  }
  if (nhub) {
    __syncthreads();
    hub_flush_min<TBA>(s_hub, nhub, vm, bitmap);
  }
}

template <class PT, class OffT, int KIND, bool LIST, bool TBA>
__global__ __launch_bounds__(kWG) void k_min_scatter_mp(const OffT* __restrict__ off,
                                                        const int32_t* __restrict__ dst,
                                                        const uint32_t* __restrict__ w, int64_t items, int64_t total,
                                                        const PT* __restrict__ P, const int32_t* __restrict__ fq,
                                                        const int32_t* __restrict__ tile_v, int64_t tile,
                                                        uint2* __restrict__ vm, uint32_t* __restrict__ bitmap,
                                                        int nhub) {
  extern __shared__ __align__(16) unsigned char smem[];
  min_scatter_mp_tile<PT, OffT, KIND, LIST, TBA>(blockIdx.x, smem, off, dst, w, items, total, P, fq, tile_v, tile, vm,
                                                 bitmap, nhub);
}

// List-mode merge-path broadcast of a device-driven loop: the list length and
// message count come from the loop state, and a fixed grid takes the tiles
// round robin (the tile count is known only on the device).
template <class OffT, int KIND, bool TBA>
__global__ __launch_bounds__(kWG) void k_loop_scatter_mp(const OffT* __restrict__ off,
                                                         const int32_t* __restrict__ dst,
                                                         const uint32_t* __restrict__ w,
                                                         const int64_t* __restrict__ P,
                                                         const int32_t* __restrict__ fq,
                                                         const int32_t* __restrict__ tile_v, int64_t tile,
                                                         int64_t max_tiles, uint2* __restrict__ vm,
                                                         uint32_t* __restrict__ bitmap, int nhub,
                                                         const LoopState* __restrict__ loop) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (loop->done || loop->mode != VC_SCHED_EDGE) return;  // uniform
  const int64_t items = loop->listed, total = items + loop->edges;
  int64_t ntiles = (total + tile - 1) / tile;
  if (ntiles > max_tiles) ntiles = max_tiles;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    min_scatter_mp_tile<int64_t, OffT, KIND, true, TBA>(t, smem, off, dst, w, items, total, P, fq, tile_v, tile, vm,
                                                        bitmap, nhub);
    __syncthreads();  // the next tile restages the LDS
  }
}

// Vertex update + frontier compaction.  Every improved vertex adopts its
// mailbox (value = mailbox, mailbox = neutral); those with out-edges are
// appended, in id order within the workgroup, to the broadcast list with
// their degree (for the next merge-path prefix).  A workgroup covers kWG
// bitmap words; each wavefront takes its 64 words (2,048 vertices) in 32
// rounds of 64 consecutive vertices, one per lane, so vertex values and
// offsets are read and written coalesced; a round's listed vertices are
// one ballot, whose popcounts place them in the list.  `bitmap` (this
// superstep's improvements) is kept: it is the next superstep's active set
// for the pull form.  `stale` (the previous active set) is cleared so it can
// collect the next improvements.  With `seed` set the values are already in
// place (the initial senders of a seeded run) and only the list and
// counters are built.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_min_compact(const OffT* __restrict__ off, int64_t n, uint2* __restrict__ vm,
                                                     const uint32_t* __restrict__ bitmap, uint32_t* __restrict__ stale,
                                                     int64_t nwords, int32_t* __restrict__ fq,
                                                     int64_t* __restrict__ P, Counters* __restrict__ ctr, int seed,
                                                     const LoopState* loop) {
  if (loop && loop->done) return;  // device-driven loop already quiescent
  const int lane = (int)(threadIdx.x & 63);
  const int64_t wbase = (int64_t)blockIdx.x * kWG + (int64_t)(threadIdx.x & ~63u);  // first word of the wavefront
  const int64_t wi = wbase + lane;
  uint32_t myword = 0;
  if (wi < nwords) {
    myword = bitmap[wi];
    if (stale[wi]) stale[wi] = 0;
  }
  uint32_t active = 0, wave_listed = 0;
  unsigned long long edges = 0, mymask = 0;  // lane i keeps round i's listed mask
  for (int i = 0; i < 32; ++i) {
    // vertex wbase*32 + 64 i + lane: word 2 i + lane / 32 of the wavefront, bit lane % 32
    const uint32_t w = __shfl(myword, 2 * i + (lane >> 5), 64);
    bool listed = false;
    if ((w >> (lane & 31)) & 1u) {
      const int64_t v = wbase * 32 + (int64_t)i * 64 + lane;
      if (!seed) {
        const uint2 p = vm[v];
        vm[v] = make_uint2(p.y, kInf);
      }
      const int64_t deg = (int64_t)off[v + 1] - (int64_t)off[v];
      ++active;
      edges += (unsigned long long)deg;
      listed = deg > 0;
    }
    const unsigned long long mk = __ballot(listed);
    if (lane == i) mymask = mk;
    wave_listed += (uint32_t)__popcll(mk);
  }
  uint32_t tot_listed;
  const uint32_t before = block_excl_scan<uint32_t>(lane == 0 ? wave_listed : 0u, &tot_listed);
  const uint32_t tot_active = block_sum<uint32_t>(active);
  const unsigned long long tot_edges = block_sum<unsigned long long>(edges);
  __shared__ unsigned long long s_base;
  if (threadIdx.x == 0) {
    s_base = tot_listed ? atomicAdd(&ctr->listed, (unsigned long long)tot_listed) : 0ull;
    if (tot_active) atomicAdd(&ctr->active, (unsigned long long)tot_active);
    if (tot_edges) atomicAdd(&ctr->edges, tot_edges);
  }
  __syncthreads();
  if (!wave_listed) return;  // uniform over the wavefront; no barrier follows
  int64_t at = (int64_t)s_base + (int64_t)__shfl(before, 0, 64);
  for (int i = 0; i < 32; ++i) {
    const unsigned long long mk = __shfl(mymask, i, 64);
    if ((mk >> lane) & 1ull) {
      const int64_t v = wbase * 32 + (int64_t)i * 64 + lane;
      const int64_t pos = at + __popcll(mk & ((1ull << lane) - 1ull));
      fq[pos] = (int32_t)v;
      P[pos] = (int64_t)off[v + 1] - (int64_t)off[v];
    }
    at += __popcll(mk);
  }
}

// Seeded start: value = init, mailbox neutral; every vertex with a finite
// initial value broadcasts at superstep 0 (bit set).  One thread per word.
__global__ __launch_bounds__(kWG) void k_min_init_from(const uint32_t* __restrict__ init, int64_t n, int64_t nwords,
                                                       uint2* __restrict__ vm, uint32_t* __restrict__ bitmap) {
  const int64_t wi = gid();
  if (wi >= nwords) return;
  uint32_t word = 0;
  for (int b = 0; b < 32; ++b) {
    const int64_t v = wi * 32 + b;
    if (v >= n) break;
    const uint32_t x = init[v];
    vm[v] = make_uint2(x, kInf);
    if (x != kInf) word |= 1u << b;
  }
  bitmap[wi] = word;
}

__global__ __launch_bounds__(kWG) void k_min_output(int64_t n, const uint2* __restrict__ vm,
                                                    uint32_t* __restrict__ out) {
  const int64_t v = gid();
  if (v < n) out[v] = vm[v].x;
}

// ------------------------------------------------------------------ scan
// Reduce-then-scan over blocks of kScanItems int64 values.
constexpr int kScanPer = 8;
constexpr int64_t kScanItems = (int64_t)kWG * kScanPer;

// loop (may be NULL): in a device-driven loop the count is the broadcast
// list's length and the kernels run only for an edge-balanced push; a fixed
// grid then takes the blocks round robin.
__device__ __forceinline__ bool scan_count(const LoopState* loop, int64_t* count) {
  if (!loop) return true;
  if (loop->done || loop->mode != VC_SCHED_EDGE) return false;
  *count = loop->listed;
  return true;
}

__global__ __launch_bounds__(kWG) void k_scan_reduce(const int64_t* __restrict__ P, int64_t count,
                                                     int64_t* __restrict__ blocks, const LoopState* loop) {
  if (!scan_count(loop, &count)) return;
  const int64_t nb = (count + kScanItems - 1) / kScanItems;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int64_t base = b * kScanItems;
    long long acc = 0;
    for (int k = 0; k < kScanPer; ++k) {
      const int64_t i = base + (int64_t)k * kWG + threadIdx.x;
      if (i < count) acc += P[i];
    }
    acc = block_sum<long long>(acc);  // ends with a barrier, so the next block may reuse its LDS
    if (threadIdx.x == 0) blocks[b] = acc;
  }
}

// One workgroup scans the block sums in place and writes P[count] = total.
__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ blocks, int64_t nblocks,
                                                   int64_t* __restrict__ P, int64_t count, const LoopState* loop) {
  __shared__ long long s_w[1024 / 64];
  __shared__ long long s_carry;
  if (loop) {
    if (!scan_count(loop, &count)) return;
    nblocks = (count + kScanItems - 1) / kScanItems;
  }
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nblocks; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const long long x = i < nblocks ? blocks[i] : 0;
    const long long inc = wave_incl_scan<long long>(x);
    if (lane_id() == 63) s_w[threadIdx.x >> 6] = inc;
    __syncthreads();
    long long before = s_carry, tot = 0;
    for (int k = 0; k < 1024 / 64; ++k) {
      if (k < (int)(threadIdx.x >> 6)) before += s_w[k];
      tot += s_w[k];
    }
    if (i < nblocks) blocks[i] = before + inc - x;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) P[count] = s_carry;
}

__global__ __launch_bounds__(kWG) void k_scan_down(int64_t* __restrict__ P, int64_t count,
                                                   const int64_t* __restrict__ blocks, const LoopState* loop) {
  if (!scan_count(loop, &count)) return;
  const int64_t nb = (count + kScanItems - 1) / kScanItems;
  for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int64_t base = b * kScanItems + (int64_t)threadIdx.x * kScanPer;
    long long v[kScanPer];
    long long sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = (base + k < count) ? P[base + k] : 0;
      sum += v[k];
    }
    long long tot;
    long long run = block_excl_scan<long long>(sum, &tot) + blocks[b];  // ends with a barrier
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (base + k < count) P[base + k] = run;
      run += v[k];
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

size_t pr_mp_lds_bytes(int64_t tile, bool off64) {
  return align16((size_t)(tile + 1) * 8) + align16((size_t)(tile + 2) * (off64 ? 8 : 4)) + kHubBytes;
}

size_t min_mp_lds_bytes(int64_t tile, bool list) {
  return (size_t)(tile + 2) * 8 + (list ? (size_t)(tile + 1) * 8 : 0) + align16((size_t)(tile + 1) * 4) + kHubBytes;
}

int hub_slots(int64_t n, size_t entry_bytes, bool hub) {
  if (!hub) return 0;
  const int64_t cap = (int64_t)(kHubBytes / entry_bytes);
  return (int)(n < cap ? n : cap);
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_stride_for(count)), dim3(kWG), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_zero_counters(Counters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, ctr);
  return hipGetLastError();
}

hipError_t launch_validate(const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m, Counters* ctr,
                           hipStream_t s) {
  const int64_t blocks = (n + kWG) / kWG;
  const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
  if (off64)
    hipLaunchKernelGGL(k_validate<int64_t>, dim3(g), dim3(kWG), 0, s, (const int64_t*)off, dst, n, m, ctr);
  else
    hipLaunchKernelGGL(k_validate<int32_t>, dim3(g), dim3(kWG), 0, s, (const int32_t*)off, dst, n, m, ctr);
  return hipGetLastError();
}

hipError_t launch_sym_hash(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n,
                           unsigned long long* acc, hipStream_t s) {
  const unsigned g = grid_stride_for((n + 63) / 64 * 64);
  if (off64)
    hipLaunchKernelGGL(k_sym_hash<int64_t>, dim3(g), dim3(kWG), 0, s, (const int64_t*)off, dst, w, n, acc);
  else
    hipLaunchKernelGGL(k_sym_hash<int32_t>, dim3(g), dim3(kWG), 0, s, (const int32_t*)off, dst, w, n, acc);
  return hipGetLastError();
}

hipError_t launch_mp_partition(const void* P, bool p64, int64_t items, int64_t total, int64_t tile, int64_t ntiles,
                               int32_t* tile_v, hipStream_t s) {
  const unsigned g = grid_for(ntiles + 1);
  if (p64)
    hipLaunchKernelGGL(k_mp_partition<int64_t>, dim3(g), dim3(kWG), 0, s, (const int64_t*)P, items, total, tile,
                       ntiles, tile_v);
  else
    hipLaunchKernelGGL(k_mp_partition<int32_t>, dim3(g), dim3(kWG), 0, s, (const int32_t*)P, items, total, tile,
                       ntiles, tile_v);
  return hipGetLastError();
}

hipError_t launch_loop_partition(const int64_t* P, int64_t tile, int64_t max_tiles, int32_t* tile_v,
                                 const LoopState* loop, hipStream_t s) {
  const int64_t want = max_tiles + 1;
  const unsigned g = grid_for(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_loop_partition, dim3(g), dim3(kWG), 0, s, P, tile, max_tiles, tile_v, loop);
  return hipGetLastError();
}

namespace {
template <class M, class S>
hipError_t pr_launch_all(int what, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                         const int32_t* tile_v, int64_t tile, int64_t ntiles, double a, double b, int64_t source,
                         void* contrib, void* mb, float* out, bool last, hipStream_t s,
                         const uint8_t* kinds = nullptr, bool hub = false, bool keep_empty = false) {
  M* c = static_cast<M*>(contrib);
  S* mbx = static_cast<S*>(mb);
  const int nhub = hub_slots(n, sizeof(S), hub);
  switch (what) {
    case 0:  // init; a = r0
      if (off64)
        hipLaunchKernelGGL((k_pr_init<int64_t, M, S>), dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, n, a,
                           source, c, mbx, out);
      else
        hipLaunchKernelGGL((k_pr_init<int32_t, M, S>), dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, n, a,
                           source, c, mbx, out);
      break;
    case 1: {  // vertex-per-thread broadcast
      const size_t lds = (size_t)nhub * sizeof(S);
      if (off64)
        hipLaunchKernelGGL((k_pr_scatter_vertex<int64_t, M, S>), dim3(grid_for(n)), dim3(kWG), lds, s,
                           (const int64_t*)off, dst, n, c, mbx, nhub);
      else
        hipLaunchKernelGGL((k_pr_scatter_vertex<int32_t, M, S>), dim3(grid_for(n)), dim3(kWG), lds, s,
                           (const int32_t*)off, dst, n, c, mbx, nhub);
      break;
    }
    case 2: {  // merge-path broadcast
      const size_t lds = align16((size_t)(tile + 1) * sizeof(S)) + align16((size_t)(tile + 2) * (off64 ? 8 : 4)) +
                         (size_t)nhub * sizeof(S);
      if (off64)
        hipLaunchKernelGGL((k_pr_scatter_mp<int64_t, M, S>), dim3((unsigned)ntiles), dim3(kWG), lds, s,
                           (const int64_t*)off, dst, n, m, tile_v, tile, c, mbx, nhub);
      else
        hipLaunchKernelGGL((k_pr_scatter_mp<int32_t, M, S>), dim3((unsigned)ntiles), dim3(kWG), lds, s,
                           (const int32_t*)off, dst, n, m, tile_v, tile, c, mbx, nhub);
      break;
    }
    default:  // apply; a = teleport, b = damping
      if (off64)
        hipLaunchKernelGGL((k_pr_apply4<int64_t, M, S>), dim3(grid_for((n + 3) / 4)), dim3(kWG), 0, s,
                           (const int64_t*)off, n, a, b, source, mbx, c, out, (int)last, kinds, (int)keep_empty);
      else
        hipLaunchKernelGGL((k_pr_apply4<int32_t, M, S>), dim3(grid_for((n + 3) / 4)), dim3(kWG), 0, s,
                           (const int32_t*)off, n, a, b, source, mbx, c, out, (int)last, kinds, (int)keep_empty);
  }
  return hipGetLastError();
}

inline hipError_t pr_launch(int mode, int what, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                            const int32_t* tile_v, int64_t tile, int64_t ntiles, double a, double b, int64_t source,
                            void* contrib, void* mb, float* out, bool last, hipStream_t s,
                            const uint8_t* kinds = nullptr, bool hub = false, bool keep_empty = false) {
  switch (mode) {
    case kRankFixed:
      return pr_launch_all<unsigned long long, unsigned long long>(what, off, off64, dst, n, m, tile_v, tile, ntiles,
                                                                   a, b, source, contrib, mb, out, last, s, kinds,
                                                                   hub, keep_empty);
    case kRankF32Msg:
      return pr_launch_all<float, unsigned long long>(what, off, off64, dst, n, m, tile_v, tile, ntiles, a, b, source,
                                                      contrib, mb, out, last, s, kinds, hub, keep_empty);
    case kRankF32:
      return pr_launch_all<float, float>(what, off, off64, dst, n, m, tile_v, tile, ntiles, a, b, source, contrib, mb,
                                         out, last, s, kinds, hub, keep_empty);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_pr_init(int mode, const void* off, bool off64, int64_t n, double r0, int64_t source, void* contrib,
                          void* mb, float* out_if_t0, hipStream_t s) {
  return pr_launch(mode, 0, off, off64, nullptr, n, 0, nullptr, 0, 0, r0, 0, source, contrib, mb, out_if_t0, false, s);
}

hipError_t launch_pr_scatter_vertex(int mode, const void* off, bool off64, const int32_t* dst, int64_t n,
                                    const void* contrib, void* mb, bool hub, hipStream_t s) {
  return pr_launch(mode, 1, off, off64, dst, n, 0, nullptr, 0, 0, 0, 0, -1, const_cast<void*>(contrib), mb, nullptr,
                   false, s, nullptr, hub);
}

hipError_t launch_pr_scatter_mp(int mode, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                                const int32_t* tile_v, int64_t tile, int64_t ntiles, const void* contrib, void* mb,
                                bool hub, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  return pr_launch(mode, 2, off, off64, dst, n, m, tile_v, tile, ntiles, 0, 0, -1, const_cast<void*>(contrib), mb,
                   nullptr, false, s, nullptr, hub);
}

hipError_t launch_pr_apply(int mode, const void* off, bool off64, int64_t n, double teleport, double damping,
                           int64_t source, void* mb, void* contrib, float* out, bool last, hipStream_t s,
                           const uint8_t* kinds, bool keep_empty) {
  return pr_launch(mode, 3, off, off64, nullptr, n, 0, nullptr, 0, 0, teleport, damping, source, contrib, mb, out,
                   last, s, kinds, false, keep_empty && kinds && !last);
}

hipError_t launch_min_init(int kind, int64_t n, int64_t source, const int32_t* ids, uint2* vm, hipStream_t s) {
  hipLaunchKernelGGL(k_min_init, dim3(grid_for(n)), dim3(kWG), 0, s, kind, n, source, ids, vm);
  return hipGetLastError();
}

hipError_t launch_min_seed_source(const void* off, bool off64, int64_t source, int32_t* fq, int64_t* P,
                                  uint32_t* active, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_min_seed_source<int64_t>, dim3(1), dim3(64), 0, s, (const int64_t*)off, source, fq, P,
                       active);
  else
    hipLaunchKernelGGL(k_min_seed_source<int32_t>, dim3(1), dim3(64), 0, s, (const int32_t*)off, source, fq, P,
                       active);
  return hipGetLastError();
}

namespace {
template <class OffT, int KIND, bool LIST, bool TBA>
void vertex_launch(const void* off, const int32_t* dst, const uint32_t* w, int64_t items, const int32_t* fq,
                   uint2* vm, uint32_t* bitmap, int nhub, hipStream_t s) {
  hipLaunchKernelGGL((k_min_scatter_vertex<OffT, KIND, LIST, TBA>), dim3(grid_for(items)), dim3(kWG),
                     (size_t)nhub * 4, s, (const OffT*)off, dst, w, items, fq, vm, bitmap, nhub);
}

template <class OffT, int KIND, bool LIST, bool TBA>
void mp_launch(const void* off, const int32_t* dst, const uint32_t* w, int64_t items, int64_t total,
               const int64_t* P, const int32_t* fq, const int32_t* tile_v, int64_t tile, int64_t ntiles, uint2* vm,
               uint32_t* bitmap, int nhub, hipStream_t s) {
  const size_t lds = min_mp_lds_bytes(tile, LIST) - kHubBytes + (size_t)nhub * 4;
  if (LIST)
    hipLaunchKernelGGL((k_min_scatter_mp<int64_t, OffT, KIND, LIST, TBA>), dim3((unsigned)ntiles), dim3(kWG), lds,
                       s, (const OffT*)off, dst, w, items, total, P, fq, tile_v, tile, vm, bitmap, nhub);
  else  // dense: the prefix is the CSR offsets themselves
    hipLaunchKernelGGL((k_min_scatter_mp<OffT, OffT, KIND, LIST, TBA>), dim3((unsigned)ntiles), dim3(kWG), lds, s,
                       (const OffT*)off, dst, w, items, total, (const OffT*)off, fq, tile_v, tile, vm, bitmap, nhub);
}

template <class OffT, int KIND>
void vertex_dispatch(bool list, bool tba, const void* off, const int32_t* dst, const uint32_t* w, int64_t items,
                     const int32_t* fq, uint2* vm, uint32_t* bitmap, int nhub, hipStream_t s) {
  if (list) {
    if (tba)
      vertex_launch<OffT, KIND, true, true>(off, dst, w, items, fq, vm, bitmap, nhub, s);
    else
      vertex_launch<OffT, KIND, true, false>(off, dst, w, items, fq, vm, bitmap, nhub, s);
  } else {
    if (tba)
      vertex_launch<OffT, KIND, false, true>(off, dst, w, items, fq, vm, bitmap, nhub, s);
    else
      vertex_launch<OffT, KIND, false, false>(off, dst, w, items, fq, vm, bitmap, nhub, s);
  }
}

template <class OffT, int KIND>
void mp_dispatch(bool list, bool tba, const void* off, const int32_t* dst, const uint32_t* w, int64_t items,
                 int64_t total, const int64_t* P, const int32_t* fq, const int32_t* tile_v, int64_t tile,
                 int64_t ntiles, uint2* vm, uint32_t* bitmap, int nhub, hipStream_t s) {
  if (list) {
    if (tba)
      mp_launch<OffT, KIND, true, true>(off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub, s);
    else
      mp_launch<OffT, KIND, true, false>(off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub, s);
  } else {
    if (tba)
      mp_launch<OffT, KIND, false, true>(off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub, s);
    else
      mp_launch<OffT, KIND, false, false>(off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub,
                                          s);
  }
}
}  // namespace

hipError_t launch_min_scatter_vertex(int kind, bool list, bool tba, const void* off, bool off64, const int32_t* dst,
                                     const uint32_t* w, int64_t n, int64_t items, const int32_t* fq, uint2* vm,
                                     uint32_t* bitmap, bool hub, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const int nhub = hub_slots(n, 4, hub);
  if (off64) {
    if (kind == kCC) vertex_dispatch<int64_t, kCC>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
    else if (kind == kSsspUnit)
      vertex_dispatch<int64_t, kSsspUnit>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
    else vertex_dispatch<int64_t, kSsspWeighted>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
  } else {
    if (kind == kCC) vertex_dispatch<int32_t, kCC>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
    else if (kind == kSsspUnit)
      vertex_dispatch<int32_t, kSsspUnit>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
    else vertex_dispatch<int32_t, kSsspWeighted>(list, tba, off, dst, w, items, fq, vm, bitmap, nhub, s);
  }
  return hipGetLastError();
}

hipError_t launch_min_scatter_mp(int kind, bool list, bool tba, const void* off, bool off64, const int32_t* dst,
                                 const uint32_t* w, int64_t n, int64_t items, int64_t total, const int64_t* P,
                                 const int32_t* fq, const int32_t* tile_v, int64_t tile, int64_t ntiles, uint2* vm,
                                 uint32_t* bitmap, bool hub, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const int nhub = hub_slots(n, 4, hub);
  if (off64) {
    if (kind == kCC)
      mp_dispatch<int64_t, kCC>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub,
                                s);
    else if (kind == kSsspUnit)
      mp_dispatch<int64_t, kSsspUnit>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap,
                                      nhub, s);
    else
      mp_dispatch<int64_t, kSsspWeighted>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm,
                                          bitmap, nhub, s);
  } else {
    if (kind == kCC)
      mp_dispatch<int32_t, kCC>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap, nhub,
                                s);
    else if (kind == kSsspUnit)
      mp_dispatch<int32_t, kSsspUnit>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm, bitmap,
                                      nhub, s);
    else
      mp_dispatch<int32_t, kSsspWeighted>(list, tba, off, dst, w, items, total, P, fq, tile_v, tile, ntiles, vm,
                                          bitmap, nhub, s);
  }
  return hipGetLastError();
}

namespace {
template <class OffT, int KIND>
void loop_mp_launch(bool tba, const void* off, const int32_t* dst, const uint32_t* w, const int64_t* P,
                    const int32_t* fq, const int32_t* tile_v, int64_t tile, int64_t max_tiles, uint2* vm,
                    uint32_t* bitmap, int nhub, const LoopState* loop, hipStream_t s) {
  const size_t lds = min_mp_lds_bytes(tile, true) - kHubBytes + (size_t)nhub * 4;
  const unsigned g = (unsigned)(max_tiles < 4096 ? (max_tiles > 0 ? max_tiles : 1) : 4096);
  if (tba)
    hipLaunchKernelGGL((k_loop_scatter_mp<OffT, KIND, true>), dim3(g), dim3(kWG), lds, s, (const OffT*)off, dst, w, P,
                       fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop);
  else
    hipLaunchKernelGGL((k_loop_scatter_mp<OffT, KIND, false>), dim3(g), dim3(kWG), lds, s, (const OffT*)off, dst, w,
                       P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop);
}
}  // namespace

hipError_t launch_loop_scatter_mp(int kind, bool tba, const void* off, bool off64, const int32_t* dst,
                                  const uint32_t* w, int64_t n, const int64_t* P, const int32_t* fq,
                                  const int32_t* tile_v, int64_t tile, int64_t max_tiles, uint2* vm, uint32_t* bitmap,
                                  bool hub, const LoopState* loop, hipStream_t s) {
  const int nhub = hub_slots(n, 4, hub);
  if (off64) {
    if (kind == kCC)
      loop_mp_launch<int64_t, kCC>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop, s);
    else if (kind == kSsspUnit)
      loop_mp_launch<int64_t, kSsspUnit>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop, s);
    else
      loop_mp_launch<int64_t, kSsspWeighted>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop,
                                             s);
  } else {
    if (kind == kCC)
      loop_mp_launch<int32_t, kCC>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop, s);
    else if (kind == kSsspUnit)
      loop_mp_launch<int32_t, kSsspUnit>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop, s);
    else
      loop_mp_launch<int32_t, kSsspWeighted>(tba, off, dst, w, P, fq, tile_v, tile, max_tiles, vm, bitmap, nhub, loop,
                                             s);
  }
  return hipGetLastError();
}

hipError_t launch_min_compact(const void* off, bool off64, int64_t n, uint2* vm, const uint32_t* bitmap,
                              uint32_t* stale, int32_t* fq, int64_t* P, Counters* ctr, bool seed,
                              const LoopState* loop, hipStream_t s) {
  const int64_t nwords = (n + 31) / 32;
  if (off64)
    hipLaunchKernelGGL(k_min_compact<int64_t>, dim3(grid_for(nwords)), dim3(kWG), 0, s, (const int64_t*)off, n, vm,
                       bitmap, stale, nwords, fq, P, ctr, (int)seed, loop);
  else
    hipLaunchKernelGGL(k_min_compact<int32_t>, dim3(grid_for(nwords)), dim3(kWG), 0, s, (const int32_t*)off, n, vm,
                       bitmap, stale, nwords, fq, P, ctr, (int)seed, loop);
  return hipGetLastError();
}

// End of a device-driven superstep: record |F|, E of the next superstep and
// the form it takes (dense_mode from dense_edges messages on, else the
// edge-balanced push), decide termination, reset the counters.
__global__ void k_loop_step(Counters* __restrict__ ctr, LoopState* __restrict__ loop, long long* __restrict__ steps,
                            int64_t max_recorded, long long dense_edges, int dense_mode) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || loop->done) return;
  const long long s = loop->step + 1;
  const long long f = (long long)ctr->active, l = (long long)ctr->listed, e = (long long)ctr->edges;
  const long long mode = (f == 0 || e == 0) ? 0 : (e >= dense_edges ? dense_mode : VC_SCHED_EDGE);
  if (s < max_recorded) {
    steps[3 * s] = f;
    steps[3 * s + 1] = e;
    steps[3 * s + 2] = mode;
  }
  loop->step = s;
  loop->listed = l;
  loop->edges = e;
  loop->mode = mode;
  ctr->active = 0;
  ctr->listed = 0;
  ctr->edges = 0;
  if (mode == 0) {
    loop->done = 1;
  } else if (s >= loop->cap) {
    loop->done = 1;
    loop->capped = 1;
  }
}

hipError_t launch_loop_step(Counters* ctr, LoopState* loop, long long* steps, int64_t max_recorded,
                            long long dense_edges, int dense_mode, hipStream_t s) {
  hipLaunchKernelGGL(k_loop_step, dim3(1), dim3(64), 0, s, ctr, loop, steps, max_recorded, dense_edges, dense_mode);
  return hipGetLastError();
}

hipError_t launch_min_init_from(const uint32_t* init, int64_t n, uint2* vm, uint32_t* bitmap, hipStream_t s) {
  const int64_t nwords = (n + 31) / 32;
  hipLaunchKernelGGL(k_min_init_from, dim3(grid_for(nwords)), dim3(kWG), 0, s, init, n, nwords, vm, bitmap);
  return hipGetLastError();
}

hipError_t launch_min_output(int64_t n, const uint2* vm, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_min_output, dim3(grid_for(n)), dim3(kWG), 0, s, n, vm, out);
  return hipGetLastError();
}

int64_t scan_scratch_entries(int64_t count) { return (count + kScanItems - 1) / kScanItems + 1; }

hipError_t launch_exclusive_scan(int64_t* P, int64_t count, int64_t* blocks, hipStream_t s) {
  const int64_t nb = (count + kScanItems - 1) / kScanItems;
  const LoopState* none = nullptr;
  if (nb > 0) hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kWG), 0, s, P, count, blocks, none);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, blocks, nb, P, count, none);
  if (nb > 0) hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kWG), 0, s, P, count, blocks, none);
  return hipGetLastError();
}

hipError_t launch_loop_scan(int64_t* P, int64_t max_count, int64_t* blocks, const LoopState* loop, hipStream_t s) {
  const int64_t nb_max = (max_count + kScanItems - 1) / kScanItems;
  const unsigned g = (unsigned)(nb_max < 1024 ? (nb_max > 0 ? nb_max : 1) : 1024);
  hipLaunchKernelGGL(k_scan_reduce, dim3(g), dim3(kWG), 0, s, P, max_count, blocks, loop);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, blocks, nb_max, P, max_count, loop);
  hipLaunchKernelGGL(k_scan_down, dim3(g), dim3(kWG), 0, s, P, max_count, blocks, loop);
  return hipGetLastError();
}

}  // namespace vc

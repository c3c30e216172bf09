// One superstep of message passing with a combiner that has no native
// atomic: the paper's hybrid combiner (Section III, Figure 1), redesigned
// for a GPU without locks.
//
// The paper keeps, per mailbox, a message and a "has a message" flag: the
// first message is stored as is (so no neutral value is needed) and later
// ones are merged with compare-and-swap; a lock orders the first store
// against the flag, and the flag must never become visible before its
// message.  A spin lock inside a wavefront can deadlock (the lanes of a wave
// do not progress independently), so here the flag is a three-state word:
// EMPTY -> WRITING (claimed by one compare-and-swap) -> FULL (a release store
// after the message is written).  Delivery runs in rounds that are uniform
// over the wavefront; in each round every pending lane makes one attempt and
// never waits: the claiming lane writes the message and publishes FULL in
// that attempt, and a lane that sees WRITING tries again next round.  A lane
// that sees FULL (acquire load, so the first message is visible) merges with
// one compare-and-swap per round on the 8-byte message, skipping the swap
// when the merge changes nothing (the no-op test of Figure 1).
#include "vc_device.h"
#include "vc_graph.h"

namespace vc {
namespace {

using namespace dev;

constexpr uint32_t kEmpty = 0, kFull = 1, kWriting = 2;

__device__ __forceinline__ double as_f64(unsigned long long x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ unsigned long long f64_bits(double d) { return (unsigned long long)__double_as_longlong(d); }

__device__ __forceinline__ unsigned long long merge(int op, unsigned long long stored, unsigned long long msg) {
  switch (op) {
    case VC_COMBINE_SUM_U64: return stored + msg;
    case VC_COMBINE_PROD_U64: return stored * msg;
    case VC_COMBINE_MAX_F64: return as_f64(msg) > as_f64(stored) ? msg : stored;
    case VC_COMBINE_MINARG: {
      const float a = __uint_as_float((uint32_t)stored), b = __uint_as_float((uint32_t)msg);
      const uint32_t ia = (uint32_t)(stored >> 32), ib = (uint32_t)(msg >> 32);
      return (b < a || (b == a && ib < ia)) ? msg : stored;
    }
    default: return f64_bits(as_f64(stored) + as_f64(msg));
  }
}

// One attempt to deliver msg; true when it is merged (or stored first).
// Never waits: a lane that finds the mailbox claimed by another writer
// returns false and tries again on the next round.
__device__ __forceinline__ bool try_combine(int op, unsigned long long* box, uint32_t* flag, unsigned long long msg) {
  const uint32_t f = __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (f == kEmpty) {
    uint32_t expect = kEmpty;
    if (!__hip_atomic_compare_exchange_strong(flag, &expect, kWriting, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT))
      return false;
    __hip_atomic_store(box, msg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(flag, kFull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  if (f == kFull) {
    unsigned long long old = __hip_atomic_load(box, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long nv = merge(op, old, msg);
    if (nv == old) return true;  // the merge changes nothing: no swap
    return __hip_atomic_compare_exchange_strong(box, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
  }
  return false;  // WRITING: the claiming lane publishes within its own attempt
}

// Merge-path tiles over the CSR (edge-balanced): the tile's senders stage
// their message and active flag in LDS, then each thread takes edges in turn.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_combine(int op, const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                 int64_t n, int64_t m, const int32_t* __restrict__ tile_v, int64_t tile,
                                                 const int32_t* __restrict__ inv,
                                                 const unsigned long long* __restrict__ msg,
                                                 const uint8_t* __restrict__ active, unsigned long long* mailbox,
                                                 uint32_t* flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);                                   // tile + 2
  unsigned long long* s_msg = reinterpret_cast<unsigned long long*>(smem + align16((size_t)(tile + 2) * 8));
  uint8_t* s_act = reinterpret_cast<uint8_t*>(smem + align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8));
  for (int x = threadIdx.x; x <= cnt; x += kWG) {
    s_off[x] = (int64_t)off[i0 + x];
    if (x < cnt) {
      const int64_t v = inv ? (int64_t)inv[i0 + x] : i0 + x;
      s_msg[x] = msg[v];
      s_act[x] = active ? active[v] : 1;
    }
  }
  __syncthreads();
  // Rounds of one attempt per pending lane, repeated while any lane of the
  // wavefront is pending: the loops are uniform over the wavefront, so no
  // lane leaves a loop on its own and a claimed mailbox is always published
  // in the round that claimed it.  (With a per-lane retry loop the compiler
  // may place the claiming lane's stores after the loop, where they wait for
  // lanes that are themselves waiting for the stores.)
  for (int64_t b0 = j0; b0 < j1; b0 += kWG) {
    const int64_t e = b0 + threadIdx.x;
    bool pending = false;
    unsigned long long m = 0;
    int64_t u = 0;
    if (e < j1) {
      int lo = 0, hi = cnt - 1;  // owner: last x with s_off[x] <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= e)
          lo = mid;
        else
          hi = mid - 1;
      }
      if (s_act[lo]) {
        const int32_t y = dst[e];
        u = inv ? (int64_t)inv[y] : y;
        m = s_msg[lo];
        pending = true;
      }
    }
    while (__ballot(pending)) {
      if (pending) pending = !try_combine(op, &mailbox[u], &flag[u], m);
    }
  }
}

// The same protocol on a workgroup's LDS slots (workgroup scope).
__device__ __forceinline__ bool try_combine_lds(int op, unsigned long long* box, uint32_t* flag,
                                                unsigned long long msg) {
  const uint32_t f = __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (f == kEmpty) {
    uint32_t expect = kEmpty;
    if (!__hip_atomic_compare_exchange_strong(flag, &expect, kWriting, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP))
      return false;
    __hip_atomic_store(box, msg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_store(flag, kFull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    return true;
  }
  if (f == kFull) {
    unsigned long long old = __hip_atomic_load(box, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const unsigned long long nv = merge(op, old, msg);
    if (nv == old) return true;
    return __hip_atomic_compare_exchange_strong(box, &old, nv, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return false;
}

constexpr int kPullChunk = 8;  // in-edges folded in registers per thread and round

// Pull form (paper, Section VI-C): merge-path tiles over the transpose.  A
// thread folds a run of kPullChunk in-edges in registers, one partial per
// receiver it meets; partials meet in the receiver's LDS slot (flag +
// message, the protocol above at workgroup scope); then every receiver the
// tile touched is written: directly when all its in-edges lie in the tile,
// else merged into global memory with the protocol at device scope.
__global__ __launch_bounds__(kWG) void k_combine_pull(int op, const int64_t* __restrict__ in_off,
                                                      const int32_t* __restrict__ in_src, int64_t n, int64_t m,
                                                      const int32_t* __restrict__ tile_v, int64_t tile,
                                                      const int32_t* __restrict__ inv,
                                                      const unsigned long long* __restrict__ msg,
                                                      const uint8_t* __restrict__ active,
                                                      unsigned long long* mailbox, uint32_t* flag) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);                                             // tile + 2
  unsigned long long* s_box = reinterpret_cast<unsigned long long*>(smem + align16((size_t)(tile + 2) * 8));  // tile + 1
  uint32_t* s_flag = reinterpret_cast<uint32_t*>(smem + align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8));
  for (int x = threadIdx.x; x <= cnt; x += kWG) {
    s_off[x] = in_off[i0 + x];
    if (x < cnt) s_flag[x] = kEmpty;
  }
  __syncthreads();
  for (int64_t b0 = j0; b0 < j1; b0 += (int64_t)kWG * kPullChunk) {
    const int64_t c0 = b0 + (int64_t)threadIdx.x * kPullChunk;
    const int64_t c1 = c0 + kPullChunk < j1 ? c0 + kPullChunk : j1;
    // gather the run's messages first (independent loads), then fold
    unsigned long long val[kPullChunk];
    bool on[kPullChunk];
#pragma unroll
    for (int k = 0; k < kPullChunk; ++k) {
      on[k] = false;
      val[k] = 0;
      if (c0 + k < c1) {
        const int32_t x = in_src[c0 + k];
        const int64_t v = inv ? (int64_t)inv[x] : x;
        on[k] = active ? active[v] != 0 : true;
        if (on[k]) val[k] = msg[v];
      }
    }
    int r = 0;  // receiver of edge c0: last r with s_off[r] <= c0
    bool pending = false;
    unsigned long long acc = 0;
    int racc = 0;
    if (c0 < c1) {
      int lo = 0, hi = cnt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= c0)
          lo = mid;
        else
          hi = mid - 1;
      }
      r = lo;
    }
    // fold run by run; a finished run's partial goes to LDS in uniform rounds
#pragma unroll
    for (int k = 0; k < kPullChunk; ++k) {
      const int64_t e = c0 + k;
      const bool valid = e < c1;
      bool flush = false;
      unsigned long long out = 0;
      int rout = 0;
      if (valid) {
        while (e >= s_off[r + 1]) ++r;
        if (pending && r != racc) {  // the run of receiver racc ended
          flush = true;
          out = acc;
          rout = racc;
          pending = false;
        }
        if (on[k]) {
          acc = pending ? merge(op, acc, val[k]) : val[k];
          racc = r;
          pending = true;
        }
      }
      while (__ballot(flush)) {
        if (flush) flush = !try_combine_lds(op, &s_box[rout], &s_flag[rout], out);
      }
    }
    bool last = pending;
    while (__ballot(last)) {
      if (last) last = !try_combine_lds(op, &s_box[racc], &s_flag[racc], acc);
    }
  }
  __syncthreads();
  for (int xb = 0; xb < cnt; xb += kWG) {
    const int x = xb + threadIdx.x;
    bool pending = false;
    int64_t u = 0;
    unsigned long long val = 0;
    if (x < cnt && s_flag[x] == kFull) {
      const int64_t y = i0 + x;
      u = inv ? (int64_t)inv[y] : y;
      val = s_box[x];
      if (s_off[x] >= j0 && s_off[x + 1] <= j1) {  // every in-edge of the receiver is in this tile
        mailbox[u] = val;
        flag[u] = kFull;
      } else {
        pending = true;
      }
    }
    while (__ballot(pending)) {
      if (pending) pending = !try_combine(op, &mailbox[u], &flag[u], val);
    }
  }
}

// ctr->edges += out-edges of the active senders.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_active_edges(const OffT* __restrict__ off, int64_t n,
                                                      const int32_t* __restrict__ inv,
                                                      const uint8_t* __restrict__ active, Counters* __restrict__ ctr) {
  const int64_t x = gid();
  unsigned long long d = 0;
  if (x < n && active[inv ? (int64_t)inv[x] : x]) d = (unsigned long long)((int64_t)off[x + 1] - (int64_t)off[x]);
  d = block_sum<unsigned long long>(d);
  if (threadIdx.x == 0 && d) atomicAdd(&ctr->edges, d);
}

}  // namespace

hipError_t launch_active_edges(const void* off, bool off64, int64_t n, const int32_t* inv, const uint8_t* active,
                               Counters* ctr, hipStream_t s) {
  if (off64)
    hipLaunchKernelGGL(k_active_edges<int64_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int64_t*)off, n, inv, active,
                       ctr);
  else
    hipLaunchKernelGGL(k_active_edges<int32_t>, dim3(grid_for(n)), dim3(kWG), 0, s, (const int32_t*)off, n, inv, active,
                       ctr);
  return hipGetLastError();
}

size_t combine_pull_lds_bytes(int64_t tile) {
  return align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8) + (size_t)(tile + 1) * 4;
}

hipError_t launch_combine_pull(int op, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                               const int32_t* tile_v, int64_t tile, int64_t ntiles, const int32_t* inv,
                               const unsigned long long* msg, const uint8_t* active, unsigned long long* mailbox,
                               uint32_t* flag, hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_pull, dim3((unsigned)ntiles), dim3(kWG), combine_pull_lds_bytes(tile), s, op, in_off,
                     in_src, n, m, tile_v, tile, inv, msg, active, mailbox, flag);
  return hipGetLastError();
}

size_t combine_lds_bytes(int64_t tile) {
  return align16((size_t)(tile + 2) * 8) + align16((size_t)(tile + 1) * 8) + (size_t)(tile + 1);
}

hipError_t launch_combine(int op, const void* off, bool off64, const int32_t* dst, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const int32_t* inv,
                          const unsigned long long* msg, const uint8_t* active, unsigned long long* mailbox,
                          uint32_t* flag, hipStream_t s) {
  if (ntiles <= 0 || m <= 0) return hipSuccess;
  const size_t lds = combine_lds_bytes(tile);
  if (off64)
    hipLaunchKernelGGL(k_combine<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, op, (const int64_t*)off, dst, n,
                       m, tile_v, tile, inv, msg, active, mailbox, flag);
  else
    hipLaunchKernelGGL(k_combine<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, op, (const int32_t*)off, dst, n,
                       m, tile_v, tile, inv, msg, active, mailbox, flag);
  return hipGetLastError();
}

}  // namespace vc

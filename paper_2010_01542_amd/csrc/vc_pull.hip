// Pull (receiver-side) form of the superstep and the transpose it reads.
//
// In the pull form every vertex writes one outbox message (its contribution
// or its value) and receivers iterate over their in-edges, fetch the outbox
// messages of the in-neighbours that broadcast, and combine them (paper,
// Section VI-C: the "single-broadcast" versions used for PageRank and CC;
// Section IV: the per-neighbour flag + message read).  Because the combine
// happens in registers and LDS of the workgroup that owns the receiver, no
// per-message global atomic is issued; only receivers whose in-edges span two
// merge-path tiles are combined across workgroups (at most two per tile).
//
// Work distribution: merge-path tiles over the merged (in-edge, vertex-end)
// sequence of the CSC, so every workgroup gets the same number of items.  In
// a tile each thread walks a contiguous run of in-edges, keeps a running
// combination while the receiver stays the same, and flushes it to the LDS
// slot of that receiver when the receiver changes.
#include "vc_device.h"

namespace vc {
namespace {

using namespace dev;

// --------------------------------------------------------------- transpose

__global__ __launch_bounds__(kWG) void k_widen(const int32_t* __restrict__ a, int64_t count, int64_t* __restrict__ b) {
  const int64_t i = gid();
  if (i < count) b[i] = a[i];
}

// in-degree histogram: cnt[d] += 1 for every edge (cnt has n + 1 zeroed entries)
__global__ __launch_bounds__(kWG) void k_csc_count(const int32_t* __restrict__ dst, int64_t m,
                                                   unsigned long long* __restrict__ cnt) {
  for (int64_t e = gid(); e < m; e += (int64_t)gridDim.x * kWG) atomicAdd(&cnt[dst[e]], 1ull);
}

// In-degree histogram without per-edge global atomics (a counting sort of
// the targets by bin): targets are grouped into bins of 2^shift vertices,
// (1) every chunk of edges counts its targets per bin in LDS, (2) a column
// scan over the chunks gives each chunk its place inside every bin, (3) each
// chunk writes its targets' offsets inside their bins (2 bytes each) to
// those places, so the offsets end up grouped by bin, (4) each piece of at
// most `piece` grouped offsets counts them per vertex in LDS and writes the
// counts: stored where the bin is one piece, added where it spans several.
constexpr int kIdWG = 1024;

__global__ __launch_bounds__(kIdWG) void k_id_hist(const int32_t* __restrict__ dst, int64_t m, int64_t chunk,
                                                   int nb, int shift, uint32_t* __restrict__ hist) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* h = reinterpret_cast<uint32_t*>(smem);
  for (int b = threadIdx.x; b < nb; b += kIdWG) h[b] = 0;
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * chunk;
  const int64_t e1 = e0 + chunk < m ? e0 + chunk : m;
  int64_t e = e0 + threadIdx.x;
  for (; e + 3 * kIdWG < e1; e += 4 * kIdWG) {  // four loads in flight before the LDS adds
    const int32_t a = dst[e], b = dst[e + kIdWG], c = dst[e + 2 * kIdWG], d = dst[e + 3 * kIdWG];
    atomicAdd(&h[a >> shift], 1u);
    atomicAdd(&h[b >> shift], 1u);
    atomicAdd(&h[c >> shift], 1u);
    atomicAdd(&h[d >> shift], 1u);
  }
  for (; e < e1; e += kIdWG) atomicAdd(&h[dst[e] >> shift], 1u);
  __syncthreads();
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += kIdWG) row[b] = h[b];
}

// Per bin b (one thread): hist[w][b] becomes the number of b's targets in
// chunks before w, tot[b] the bin's size.
__global__ __launch_bounds__(kWG) void k_id_colscan(uint32_t* __restrict__ hist, int64_t chunks, int nb,
                                                    int64_t* __restrict__ tot) {
  const int64_t b = gid();
  if (b >= nb) return;
  uint32_t run = 0;
  int64_t w = 0;
  for (; w + 8 <= chunks; w += 8) {
    uint32_t x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = hist[(w + i) * nb + b];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      hist[(w + i) * nb + b] = run;
      run += x[i];
    }
  }
  for (; w < chunks; ++w) {
    const uint32_t x = hist[w * nb + b];
    hist[w * nb + b] = run;
    run += x;
  }
  tot[b] = run;
}

// Writes every target's offset inside its bin at its chunk's next place in
// the bin; positions are below m < 2^32.
__global__ __launch_bounds__(kIdWG) void k_id_scatter(const int32_t* __restrict__ dst, int64_t m, int64_t chunk,
                                                      int nb, int shift, const uint32_t* __restrict__ hist,
                                                      const int64_t* __restrict__ bin_start,
                                                      uint16_t* __restrict__ grouped) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* cur = reinterpret_cast<uint32_t*>(smem);
  const uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  for (int b = threadIdx.x; b < nb; b += kIdWG) cur[b] = (uint32_t)bin_start[b] + row[b];
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * chunk;
  const int64_t e1 = e0 + chunk < m ? e0 + chunk : m;
  const int32_t mask = (1 << shift) - 1;
  int64_t e = e0 + threadIdx.x;
  for (; e + 3 * kIdWG < e1; e += 4 * kIdWG) {
    const int32_t a = dst[e], b = dst[e + kIdWG], c = dst[e + 2 * kIdWG], d = dst[e + 3 * kIdWG];
    grouped[atomicAdd(&cur[a >> shift], 1u)] = (uint16_t)(a & mask);
    grouped[atomicAdd(&cur[b >> shift], 1u)] = (uint16_t)(b & mask);
    grouped[atomicAdd(&cur[c >> shift], 1u)] = (uint16_t)(c & mask);
    grouped[atomicAdd(&cur[d >> shift], 1u)] = (uint16_t)(d & mask);
  }
  for (; e < e1; e += kIdWG) {
    const int32_t a = dst[e];
    grouped[atomicAdd(&cur[a >> shift], 1u)] = (uint16_t)(a & mask);
  }
}

// pieces[b] = number of pieces of bin b (bin_start holds nb + 1 entries).
__global__ __launch_bounds__(kWG) void k_id_pieces(const int64_t* __restrict__ bin_start, int nb, int64_t piece,
                                                   int64_t* __restrict__ pieces) {
  const int64_t b = gid();
  if (b < nb) pieces[b] = (bin_start[b + 1] - bin_start[b] + piece - 1) / piece;
}

// One workgroup per piece (grid: an upper bound of the piece count; the rest
// return at once).  cnt: n + 1 entries, zero on entry.
__global__ __launch_bounds__(kIdWG) void k_id_count(const uint16_t* __restrict__ grouped,
                                                    const int64_t* __restrict__ bin_start,
                                                    const int64_t* __restrict__ piece_pre, int nb, int shift,
                                                    int64_t piece, int64_t n, unsigned long long* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* c = reinterpret_cast<uint32_t*>(smem);
  const int64_t w = blockIdx.x;
  if (w >= piece_pre[nb]) return;  // uniform over the workgroup
  int lo = 0, hi = nb - 1;         // bin: last b with piece_pre[b] <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (piece_pre[mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int b = lo;
  const int width = 1 << shift;
  for (int x = threadIdx.x; x < width; x += kIdWG) c[x] = 0;
  __syncthreads();
  const int64_t s0 = bin_start[b] + (w - piece_pre[b]) * piece;
  const int64_t s1 = s0 + piece < bin_start[b + 1] ? s0 + piece : bin_start[b + 1];
  int64_t i = s0 + threadIdx.x;
  for (; i + 3 * kIdWG < s1; i += 4 * kIdWG) {
    const uint16_t a = grouped[i], bb = grouped[i + kIdWG], cc = grouped[i + 2 * kIdWG], d = grouped[i + 3 * kIdWG];
    atomicAdd(&c[a], 1u);
    atomicAdd(&c[bb], 1u);
    atomicAdd(&c[cc], 1u);
    atomicAdd(&c[d], 1u);
  }
  for (; i < s1; i += kIdWG) atomicAdd(&c[grouped[i]], 1u);
  __syncthreads();
  const bool whole = piece_pre[b + 1] - piece_pre[b] == 1;
  const int64_t v0 = (int64_t)b << shift;
  const int64_t vend = v0 + width < n ? v0 + width : n;
  for (int64_t v = v0 + threadIdx.x; v < vend; v += kIdWG) {
    const uint32_t x = c[v - v0];
    if (whole)
      cnt[v] = x;
    else if (x)
      atomicAdd(&cnt[v], (unsigned long long)x);
  }
}

// Places every edge u->v at cursor[v]++ in the CSC.  Workgroups own merge-path
// tiles of the CSR so hubs are split; the source of an edge is found by a
// binary search over the tile's offsets staged in LDS.
template <class OffT>
__global__ __launch_bounds__(kWG) void k_csc_fill(const OffT* __restrict__ off, const int32_t* __restrict__ dst,
                                                  const uint32_t* __restrict__ w, int64_t n, int64_t m,
                                                  const int32_t* __restrict__ tile_v, int64_t tile,
                                                  unsigned long long* __restrict__ cursor,
                                                  int32_t* __restrict__ in_src, uint32_t* __restrict__ in_w) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t t = blockIdx.x;
  const int64_t k0 = t * tile;
  const int64_t k1 = (k0 + tile < n + m) ? k0 + tile : n + m;
  const int64_t i0 = tile_v[t], i1 = tile_v[t + 1];
  const int64_t j0 = k0 - i0, j1 = k1 - i1;
  if (j1 <= j0) return;
  const int64_t ilast = i1 < n ? i1 : n - 1;
  const int cnt = (int)(ilast - i0 + 1);
  int64_t* s_off = reinterpret_cast<int64_t*>(smem);
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
    const int32_t v = dst[e];
    const unsigned long long p = atomicAdd(&cursor[v], 1ull);
    in_src[p] = (int32_t)(i0 + lo);
    if (w) in_w[p] = w[e];
  }
}


// --------------------------------------------------------------- PageRank pull

template <class V>
__device__ __forceinline__ void lds_add(V* p, V x);
template <>
__device__ __forceinline__ void lds_add<float>(float* p, float x) {
  atomicAdd(p, x);
}
template <>
__device__ __forceinline__ void lds_add<unsigned long long>(unsigned long long* p, unsigned long long x) {
  atomicAdd(p, x);
}
template <class V>
__device__ __forceinline__ void global_add(V* p, V x);
template <>
__device__ __forceinline__ void global_add<float>(float* p, float x) {
  unsafeAtomicAdd(p, x);
}
template <>
__device__ __forceinline__ void global_add<unsigned long long>(unsigned long long* p, unsigned long long x) {
  atomicAdd(p, x);
}

// mb[v] = sum of contrib[u] over in-edges u->v.  mb must be zero on entry for
// receivers whose in-edges cross a tile boundary (the update step leaves
// every mailbox at zero).  Tiles hold kWG * VT items, so a thread's run is at
// most VT in-edges: all of its source ids are loaded first, then all of its
// gathers are issued back to back, and only then combined.
template <class M, class V, int VT>
__global__ __launch_bounds__(kWG) void k_pr_pull(const int64_t* __restrict__ in_off, const int32_t* __restrict__ in_src,
                                                 int64_t n, int64_t m, const int32_t* __restrict__ tile_v,
                                                 const M* __restrict__ contrib, V* __restrict__ mb) {
  constexpr int64_t tile = (int64_t)kWG * VT;
  extern __shared__ __align__(16) unsigned char smem[];
  Tile tl;
  if (!tile_bounds(tile_v, tile, n, m, &tl)) return;
  V* s_acc = reinterpret_cast<V*>(smem);                                              // tile + 1
  int64_t* s_off = reinterpret_cast<int64_t*>(smem + align16((tile + 1) * sizeof(V)));  // tile + 2
  for (int x = threadIdx.x; x <= tl.cnt; x += kWG) s_off[x] = in_off[tl.i0 + x];
  for (int x = threadIdx.x; x < tl.cnt; x += kWG) s_acc[x] = V(0);
  const int64_t ne = tl.j1 - tl.j0;
  const int per = (int)((ne + kWG - 1) / kWG);  // <= VT
  const int64_t e0 = tl.j0 + (int64_t)threadIdx.x * per;
  const int run_len = e0 < tl.j1 ? (int)((tl.j1 - e0) < per ? (tl.j1 - e0) : per) : 0;
  int32_t src[VT];
#pragma unroll
  for (int k = 0; k < VT; ++k) src[k] = k < run_len ? __builtin_nontemporal_load(&in_src[e0 + k]) : 0;
  V c[VT];
#pragma unroll
  for (int k = 0; k < VT; ++k) c[k] = k < run_len ? msg_to_sum<M, V>(contrib[src[k]]) : V(0);
  __syncthreads();
  if (run_len > 0) {
    int x = owner_of(s_off, tl.cnt, e0);
    int64_t next = s_off[x + 1];
    V run = V(0);
#pragma unroll
    for (int k = 0; k < VT; ++k) {
      if (k < run_len) {
        while (e0 + k >= next) {  // receiver changes: flush the running sum
          if (run != V(0)) lds_add<V>(&s_acc[x], run);
          run = V(0);
          ++x;
          next = s_off[x + 1];
        }
        run += c[k];
      }
    }
    if (run != V(0)) lds_add<V>(&s_acc[x], run);
  }
  __syncthreads();
  for (int x = threadIdx.x; x < tl.cnt; x += kWG) {
    const V a = s_acc[x];
    if (a == V(0)) continue;
    const int64_t v = tl.i0 + x;
    if (s_off[x] >= tl.j0 && s_off[x + 1] <= tl.j1)
      mb[v] = a;  // every in-edge of v is in this tile
    else
      global_add<V>(&mb[v], a);
  }
}

// --------------------------------------------------------------- CC / SSSP pull

template <int KIND>
__device__ __forceinline__ uint32_t pull_message(uint32_t val, const uint32_t* __restrict__ in_w, int64_t e) {
  if (KIND == kCC) return val;
  if (KIND == kSsspUnit) return sat_add(val, 1u);
  return sat_add(val, in_w[e]);
}

__device__ __forceinline__ bool bit_set(const uint32_t* __restrict__ bits, int64_t u) {
  return (bits[u >> 5] >> (u & 31)) & 1u;
}

// For every receiver v: best = min over in-edges u->v with u active of
// value(u) (+ w).  When best lowers value(v), the mailbox of v takes it and
// v is marked in `improved` (the same outcome as the push form, so the
// compaction step is shared).  `active` = NULL means every vertex broadcast.
// As in the PageRank pull, a thread first loads its run of VT in-edges, then
// the activity words of their sources, then the values of the active ones.
template <int KIND, bool CHECK, int VT>
__global__ __launch_bounds__(kWG) void k_min_pull(const int64_t* __restrict__ in_off,
                                                  const int32_t* __restrict__ in_src,
                                                  const uint32_t* __restrict__ in_w, int64_t n, int64_t m,
                                                  const int32_t* __restrict__ tile_v, uint2* __restrict__ vm,
                                                  const uint32_t* __restrict__ active,
                                                  uint32_t* __restrict__ improved, const LoopState* loop) {
  constexpr int64_t tile = (int64_t)kWG * VT;
  extern __shared__ __align__(16) unsigned char smem[];
  if (loop && (loop->done || loop->mode != VC_SCHED_PULL)) return;  // quiescent, or another form this superstep
  Tile tl;
  if (!tile_bounds(tile_v, tile, n, m, &tl)) return;
  uint32_t* s_min = reinterpret_cast<uint32_t*>(smem);                          // tile + 1
  int64_t* s_off = reinterpret_cast<int64_t*>(smem + align16((tile + 1) * 4));  // tile + 2
  for (int x = threadIdx.x; x <= tl.cnt; x += kWG) s_off[x] = in_off[tl.i0 + x];
  for (int x = threadIdx.x; x < tl.cnt; x += kWG) s_min[x] = kInf;
  const uint32_t* val = reinterpret_cast<const uint32_t*>(vm);  // value of u at val[2u]
  const int64_t ne = tl.j1 - tl.j0;
  const int per = (int)((ne + kWG - 1) / kWG);
  const int64_t e0 = tl.j0 + (int64_t)threadIdx.x * per;
  const int run_len = e0 < tl.j1 ? (int)((tl.j1 - e0) < per ? (tl.j1 - e0) : per) : 0;
  int32_t src[VT];
#pragma unroll
  for (int k = 0; k < VT; ++k) src[k] = k < run_len ? __builtin_nontemporal_load(&in_src[e0 + k]) : 0;
  bool act[VT];
#pragma unroll
  for (int k = 0; k < VT; ++k) act[k] = k < run_len && (!CHECK || bit_set(active, src[k]));
  uint32_t msg[VT];
#pragma unroll
  for (int k = 0; k < VT; ++k) {
    msg[k] = kInf;
    if (act[k]) {
      const uint32_t wv = KIND == kSsspWeighted ? __builtin_nontemporal_load(&in_w[e0 + k]) : 1u;
      const uint32_t x = val[2 * (int64_t)src[k]];
      msg[k] = KIND == kCC ? x : sat_add(x, wv);
    }
  }
  __syncthreads();
  if (run_len > 0) {
    int x = owner_of(s_off, tl.cnt, e0);
    int64_t next = s_off[x + 1];
    uint32_t run = kInf;
#pragma unroll
    for (int k = 0; k < VT; ++k) {
      if (k < run_len) {
        while (e0 + k >= next) {
          if (run != kInf) atomicMin(&s_min[x], run);
          run = kInf;
          ++x;
          next = s_off[x + 1];
        }
        run = msg[k] < run ? msg[k] : run;
      }
    }
    if (run != kInf) atomicMin(&s_min[x], run);
  }
  __syncthreads();
  // per receiver: complete ones are owned by this tile; boundary ones are
  // combined with an atomic min.  Improvement bits are OR-ed per word from a
  // wave ballot (lanes hold consecutive receivers).
  for (int base = 0; base < tl.cnt; base += kWG) {
    const int x = base + (int)threadIdx.x;
    const int64_t v = tl.i0 + x;
    bool imp = false;
    if (x < tl.cnt) {
      const uint32_t best = s_min[x];
      if (best != kInf) {
        const uint2 cur = vm[v];
        if (best < cur.x) {
          if (s_off[x] >= tl.j0 && s_off[x + 1] <= tl.j1) {
            vm[v].y = best;
            imp = true;
          } else if (best < cur.y) {
            const uint32_t old = atomicMin(&reinterpret_cast<uint32_t*>(vm)[2 * v + 1], best);
            imp = old == kInf;
          }
        }
      }
    }
    const unsigned long long mask = __ballot(imp);
    const int lane = (int)lane_id();
    const bool leader = lane == 0 || (v & 31) == 0;
    if (leader && mask) {
      const int room = (int)(32 - (v & 31));
      const int len = room < 64 - lane ? room : 64 - lane;
      const unsigned long long seg = len >= 64 ? ~0ull : ((1ull << len) - 1ull);
      const uint32_t bits = (uint32_t)(((mask >> lane) & seg) << (v & 31));
      if (bits) atomicOr(&improved[v >> 5], bits);
    }
  }
}

}  // namespace

// --------------------------------------------------------------- launchers

size_t pull_lds_bytes(int64_t tile) { return align16((size_t)(tile + 1) * 8) + (size_t)(tile + 2) * 8; }

// The pull kernels use tiles of kWG * VT items with VT in {4, 8, 16}.
int64_t pull_tile(int64_t requested) {
  if (requested <= (int64_t)kWG * 4) return (int64_t)kWG * 4;
  if (requested <= (int64_t)kWG * 8) return (int64_t)kWG * 8;
  return (int64_t)kWG * 16;
}

hipError_t launch_widen_offsets(const int32_t* a, int64_t count, int64_t* b, hipStream_t s) {
  hipLaunchKernelGGL(k_widen, dim3(grid_for(count)), dim3(kWG), 0, s, a, count, b);
  return hipGetLastError();
}

hipError_t launch_csc_count(const int32_t* dst, int64_t m, unsigned long long* cnt, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t blocks = (m + kWG - 1) / kWG;
  hipLaunchKernelGGL(k_csc_count, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kWG), 0, s, dst, m, cnt);
  return hipGetLastError();
}

bool id_binned(int64_t n, int64_t m, size_t max_lds, IdPlan* plan) {
  if (m < kIdMinEdges || m >= (1ll << 32)) return false;
  const int shift = kIdBinShift;
  const int64_t nb = (n + (1ll << shift) - 1) >> shift;
  if (nb > kIdMaxBins || ((size_t)4 << shift) > max_lds || (size_t)nb * 4 > max_lds) return false;
  plan->shift = shift;
  plan->nb = (int)nb;
  plan->chunk = std::max<int64_t>(kIdMinChunk, (m + kIdMaxChunks - 1) / kIdMaxChunks);
  plan->chunks = (m + plan->chunk - 1) / plan->chunk;
  plan->piece = kIdPiece;
  plan->max_pieces = plan->nb + (m + plan->piece - 1) / plan->piece;
  return true;
}

hipError_t launch_id_binned(const IdPlan& p, const int32_t* dst, int64_t n, int64_t m, uint32_t* hist,
                            int64_t* bin_start, int64_t* piece_pre, int64_t* scan_blocks, uint16_t* grouped,
                            unsigned long long* cnt, hipStream_t s) {
  const size_t lds_bins = (size_t)p.nb * 4;
  hipLaunchKernelGGL(k_id_hist, dim3((unsigned)p.chunks), dim3(kIdWG), lds_bins, s, dst, m, p.chunk, p.nb, p.shift,
                     hist);
  hipLaunchKernelGGL(k_id_colscan, dim3(grid_for(p.nb)), dim3(kWG), 0, s, hist, p.chunks, p.nb, bin_start);
  hipError_t e = launch_exclusive_scan(bin_start, p.nb, scan_blocks, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_id_scatter, dim3((unsigned)p.chunks), dim3(kIdWG), lds_bins, s, dst, m, p.chunk, p.nb,
                     p.shift, hist, bin_start, grouped);
  hipLaunchKernelGGL(k_id_pieces, dim3(grid_for(p.nb)), dim3(kWG), 0, s, bin_start, p.nb, p.piece, piece_pre);
  e = launch_exclusive_scan(piece_pre, p.nb, scan_blocks, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_id_count, dim3((unsigned)p.max_pieces), dim3(kIdWG), (size_t)4 << p.shift, s, grouped,
                     bin_start, piece_pre, p.nb, p.shift, p.piece, n, cnt);
  return hipGetLastError();
}

hipError_t launch_csc_fill(const void* off, bool off64, const int32_t* dst, const uint32_t* w, int64_t n, int64_t m,
                           const int32_t* tile_v, int64_t tile, int64_t ntiles, unsigned long long* cursor,
                           int32_t* in_src, uint32_t* in_w, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const size_t lds = (size_t)(tile + 2) * 8;
  if (off64)
    hipLaunchKernelGGL(k_csc_fill<int64_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int64_t*)off, dst, w, n,
                       m, tile_v, tile, cursor, in_src, in_w);
  else
    hipLaunchKernelGGL(k_csc_fill<int32_t>, dim3((unsigned)ntiles), dim3(kWG), lds, s, (const int32_t*)off, dst, w, n,
                       m, tile_v, tile, cursor, in_src, in_w);
  return hipGetLastError();
}

namespace {
template <class M, class V, int VT>
void pr_pull_launch(const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m, const int32_t* tile_v,
                    int64_t ntiles, const void* contrib, void* mb, hipStream_t s) {
  const int64_t tile = (int64_t)kWG * VT;
  const size_t lds = align16((size_t)(tile + 1) * sizeof(V)) + (size_t)(tile + 2) * 8;
  hipLaunchKernelGGL((k_pr_pull<M, V, VT>), dim3((unsigned)ntiles), dim3(kWG), lds, s, in_off, in_src, n, m, tile_v,
                     (const M*)contrib, (V*)mb);
}
template <class M, class V>
void pr_pull_vt(int64_t tile, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                const int32_t* tile_v, int64_t ntiles, const void* contrib, void* mb, hipStream_t s) {
  if (tile == kWG * 4)
    pr_pull_launch<M, V, 4>(in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s);
  else if (tile == kWG * 8)
    pr_pull_launch<M, V, 8>(in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s);
  else
    pr_pull_launch<M, V, 16>(in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s);
}
template <int KIND, int VT>
void min_pull_launch(bool check, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w, int64_t n,
                     int64_t m, const int32_t* tile_v, int64_t ntiles, uint2* vm, const uint32_t* active,
                     uint32_t* improved, const LoopState* loop, hipStream_t s) {
  const int64_t tile = (int64_t)kWG * VT;
  const size_t lds = align16((size_t)(tile + 1) * 4) + (size_t)(tile + 2) * 8;
  if (check)
    hipLaunchKernelGGL((k_min_pull<KIND, true, VT>), dim3((unsigned)ntiles), dim3(kWG), lds, s, in_off, in_src, in_w,
                       n, m, tile_v, vm, active, improved, loop);
  else
    hipLaunchKernelGGL((k_min_pull<KIND, false, VT>), dim3((unsigned)ntiles), dim3(kWG), lds, s, in_off, in_src,
                       in_w, n, m, tile_v, vm, active, improved, loop);
}
template <int KIND>
void min_pull_vt(int64_t tile, bool check, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w,
                 int64_t n, int64_t m, const int32_t* tile_v, int64_t ntiles, uint2* vm, const uint32_t* active,
                 uint32_t* improved, const LoopState* loop, hipStream_t s) {
  if (tile == kWG * 4)
    min_pull_launch<KIND, 4>(check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop, s);
  else if (tile == kWG * 8)
    min_pull_launch<KIND, 8>(check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop, s);
  else
    min_pull_launch<KIND, 16>(check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop, s);
}
}  // namespace

hipError_t launch_pr_pull(int mode, const int64_t* in_off, const int32_t* in_src, int64_t n, int64_t m,
                          const int32_t* tile_v, int64_t tile, int64_t ntiles, const void* contrib, void* mb,
                          hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tile != pull_tile(tile)) return hipErrorInvalidValue;
  using U64 = unsigned long long;
  switch (mode) {
    case kRankFixed: pr_pull_vt<U64, U64>(tile, in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s); break;
    case kRankF32Msg: pr_pull_vt<float, U64>(tile, in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s); break;
    case kRankF32: pr_pull_vt<float, float>(tile, in_off, in_src, n, m, tile_v, ntiles, contrib, mb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_min_pull(int kind, const int64_t* in_off, const int32_t* in_src, const uint32_t* in_w, int64_t n,
                           int64_t m, const int32_t* tile_v, int64_t tile, int64_t ntiles, uint2* vm,
                           const uint32_t* active, uint32_t* improved, const LoopState* loop, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (tile != pull_tile(tile)) return hipErrorInvalidValue;
  const bool check = active != nullptr;
  if (kind == kCC)
    min_pull_vt<kCC>(tile, check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop, s);
  else if (kind == kSsspUnit)
    min_pull_vt<kSsspUnit>(tile, check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop, s);
  else
    min_pull_vt<kSsspWeighted>(tile, check, in_off, in_src, in_w, n, m, tile_v, ntiles, vm, active, improved, loop,
                               s);
  return hipGetLastError();
}

}  // namespace vc

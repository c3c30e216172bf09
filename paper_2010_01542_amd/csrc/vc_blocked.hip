// PageRank broadcast + combine by propagation blocking (a variant of the
// paper's single-broadcast pull, Section VI-C, for graphs much larger than
// the caches).
//
// The pull form gathers one 8-byte message per in-edge from anywhere in the
// message array; on a billion-edge graph most of those gathers miss the
// caches, and even those that hit cost one cache-line request per edge.
// Here the edges are laid out once by bucket (source tile, destination bin):
// a source tile's messages fit in LDS (2^14 vertices: 64 KiB of binary32 or
// 128 KiB of uint64 messages), a destination bin's mailboxes too (2^12
// vertices, 32 KiB).  A superstep is two streaming passes:
//   1. spread: per source tile, its messages are staged in LDS, then every
//      slot of the tile's buckets (contiguous, tile-major order) gets
//      vals[k] = message of its source: 2-byte index in, 4 or 8 bytes out;
//   2. fold: per destination bin, its runs (one per source tile that has
//      edges into it) are read and summed into LDS mailboxes, which are then
//      written to the mailbox array (added atomically when a bin of hubs is
//      split over several workgroups).
// Sums stay exact (uint64 fixed point), so results equal the pull form's.
// Messages are uint64 fixed point or binary32 (half the slot bytes).  The
// same two passes serve the dense supersteps of the min programs (CC,
// SSSP): the spread writes each slot's message (unreached for a source
// outside the frontier), the fold takes minima in LDS and applies the pull
// form's mailbox and improvement rule.
#include <type_traits>

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

// *out = max(*out, largest of the m weights).  A grid of a few workgroups
// per CU streams the weights in 16-byte loads (after a head of up to three
// words that brings the pointer to 16-byte alignment), reduces in each
// wavefront and then in LDS, and issues one atomic per workgroup.
__global__ __launch_bounds__(kWG) void k_pb_wmax(const uint32_t* __restrict__ w, int64_t m, uint32_t* __restrict__ out) {
  __shared__ uint32_t s_w[kWG / 64];
  const int64_t lead = (int64_t)(((16 - ((uintptr_t)w & 15)) & 15) >> 2);  // words before a 16-byte boundary
  const int64_t head = lead < m ? lead : m;
  uint32_t x = 0;
  if (gid() < head) x = w[gid()];
  const uint4* w4 = reinterpret_cast<const uint4*>(w + head);
  const int64_t m4 = (m - head) >> 2;
  for (int64_t i = gid(); i < m4; i += grid_threads()) {
    const uint4 q = w4[i];
    const uint32_t a = q.x > q.y ? q.x : q.y, b = q.z > q.w ? q.z : q.w;
    const uint32_t c = a > b ? a : b;
    x = c > x ? c : x;
  }
  for (int64_t e = head + (m4 << 2) + gid(); e < m; e += grid_threads()) x = w[e] > x ? w[e] : x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kWG / 64; ++i) r = s_w[i] > r ? s_w[i] : r;
    if (r) atomicMax(out, r);
  }
}

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
// reserves each bucket's share at cursor and writes the slots (and the
// edge weights in slot order when w is given, as bytes when wbytes is 1).
template <bool PLACE>
__global__ __launch_bounds__(kBuildWG) void k_pb_build(const int64_t* __restrict__ te, int64_t tiles,
                                                       const int32_t* __restrict__ dst, int64_t m, int64_t chunk,
                                                       int64_t bins, int pass_bins,
                                                       unsigned long long* __restrict__ cnt,
                                                       const uint16_t* __restrict__ srcl_csr,
                                                       uint16_t* __restrict__ srcl, uint16_t* __restrict__ dstl,
                                                       const uint32_t* __restrict__ w, void* __restrict__ wslot,
                                                       int wbytes) {
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
            if (w) {
              if (wbytes == 1)
                static_cast<uint8_t*>(wslot)[k] = (uint8_t)w[e];
              else
                static_cast<uint32_t*>(wslot)[k] = w[e];
            }
          }
        }
        __syncthreads();
      }
    }
  }
}

// Two-level placement.  Placing each edge straight into its bucket writes
// a few bytes at a time into runs of about 16 edges spread over thousands
// of open lines per workgroup (8x the bytes placed reach HBM).  Instead:
// level 1 sorts each tile's edges into groups of kPbGroupBins bins, whose
// slot ranges (tile-major, bins in order) are contiguous, writing each
// edge's target, source offset and weight at a free position of its group
// (runs of thousands of edges per workgroup); level 2 takes each group in
// pieces of up to kPbPiece edges and places them into their buckets.
constexpr int kPbGroupShift = 7;
constexpr int kPbGroupBins = 1 << kPbGroupShift;
constexpr int64_t kPbPiece = 8192;

// gcur[t * groups + g] = first slot of bucket (t, g * kPbGroupBins).
__global__ __launch_bounds__(kWG) void k_pb_group_starts(const int64_t* __restrict__ starts, int64_t tiles,
                                                         int64_t bins, int64_t groups,
                                                         unsigned long long* __restrict__ gcur,
                                                         int64_t* __restrict__ pieces) {
  const int64_t i = gid();
  if (i >= tiles * groups) return;
  const int64_t t = i / groups, g = i - t * groups;
  const int64_t b1 = (g + 1) * kPbGroupBins < bins ? (g + 1) * kPbGroupBins : bins;
  const int64_t s0 = starts[t * bins + g * kPbGroupBins], s1 = starts[t * bins + b1];
  gcur[i] = (unsigned long long)s0;
  pieces[i] = (s1 - s0 + kPbPiece - 1) / kPbPiece;
}

// Level 1: per workgroup, CSR edges [c0, c1) split by tile; LDS histogram
// of groups, one global atomic per (tile, group) to reserve, then each
// edge's record at its group position.
__global__ __launch_bounds__(kBuildWG) void k_pb_group(const int64_t* __restrict__ te, int64_t tiles,
                                                       const int32_t* __restrict__ dst, int64_t m, int64_t chunk,
                                                       int64_t groups, unsigned long long* __restrict__ gcur,
                                                       const uint16_t* __restrict__ srcl_csr,
                                                       const uint32_t* __restrict__ w, int wbytes,
                                                       int32_t* __restrict__ tdst, uint16_t* __restrict__ tsrcl,
                                                       void* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned long long* base = reinterpret_cast<unsigned long long*>(smem);  // groups
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + groups);             // groups
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = (c0 + chunk < m) ? c0 + chunk : m;
  for (int64_t t = tile_of(te, tiles, c0); t < tiles && te[t] < c1; ++t) {
    const int64_t e0 = te[t] > c0 ? te[t] : c0;
    const int64_t e1 = te[t + 1] < c1 ? te[t + 1] : c1;
    if (e0 >= e1) continue;
    for (int64_t i = threadIdx.x; i < groups; i += kBuildWG) hist[i] = 0u;
    __syncthreads();
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBuildWG)
      atomicAdd(&hist[dst[e] >> (kPbDstShift + kPbGroupShift)], 1u);
    __syncthreads();
    for (int64_t i = threadIdx.x; i < groups; i += kBuildWG) {
      const uint32_t h = hist[i];
      base[i] = h ? atomicAdd(&gcur[t * groups + i], (unsigned long long)h) : 0ull;
      hist[i] = 0u;
    }
    __syncthreads();
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kBuildWG) {
      const int32_t v = dst[e];
      const int g = v >> (kPbDstShift + kPbGroupShift);
      const int64_t k = (int64_t)base[g] + (int64_t)atomicAdd(&hist[g], 1u);
      tdst[k] = v;
      tsrcl[k] = srcl_csr[e];
      if (w) {
        if (wbytes == 1)
          static_cast<uint8_t*>(tw)[k] = (uint8_t)w[e];
        else
          static_cast<uint32_t*>(tw)[k] = w[e];
      }
    }
    __syncthreads();
  }
}

// Level 2: workgroup j takes piece j (poff: exclusive scan of the pieces
// per (tile, group), tiles * groups + 1 entries) and places its edges in
// their buckets.  The piece is sorted by bin in LDS (histogram, scan,
// scatter into LDS), then written out in slot order, so consecutive lanes
// write consecutive slots.  A piece that is its group's only one owns the
// group's whole slot range (bucket starts from `starts`); otherwise each
// bucket's share is reserved with one global atomic on its cursor in cnt.
__global__ __launch_bounds__(kBuildWG) void k_pb_place(const int64_t* __restrict__ poff, int64_t segs,
                                                       int64_t groups, int64_t bins,
                                                       const int64_t* __restrict__ starts,
                                                       unsigned long long* __restrict__ cnt,
                                                       const int32_t* __restrict__ tdst,
                                                       const uint16_t* __restrict__ tsrcl, const void* __restrict__ tw,
                                                       int wbytes, bool weighted, uint16_t* __restrict__ srcl,
                                                       uint16_t* __restrict__ dstl, void* __restrict__ wslot) {
  __shared__ unsigned long long base[kPbGroupBins];  // first slot of each bin's share
  __shared__ uint32_t hist[kPbGroupBins], lpos[kPbGroupBins + 1];
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* s_srcl = reinterpret_cast<uint16_t*>(smem);  // kPbPiece each, in bin order
  uint16_t* s_dstl = s_srcl + kPbPiece;
  unsigned char* s_w = reinterpret_cast<unsigned char*>(s_dstl + kPbPiece);  // kPbPiece * wbytes
  const int64_t j = blockIdx.x;
  int64_t lo = 0, hi = segs - 1;  // last segment with poff <= j
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (poff[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t sg = lo, t = sg / groups, g = sg - t * groups;
  const int64_t b0 = g * kPbGroupBins, b1 = b0 + kPbGroupBins < bins ? b0 + kPbGroupBins : bins;
  const int64_t s1 = starts[t * bins + b1];
  const int64_t a = starts[t * bins + b0] + (j - poff[sg]) * kPbPiece;
  const int64_t z = a + kPbPiece < s1 ? a + kPbPiece : s1;
  const int cnt_here = (int)(z - a);
  for (int i = threadIdx.x; i < kPbGroupBins; i += kBuildWG) hist[i] = 0u;
  __syncthreads();
  for (int64_t k = a + threadIdx.x; k < z; k += kBuildWG) atomicAdd(&hist[(tdst[k] >> kPbDstShift) - b0], 1u);
  __syncthreads();
  const bool alone = poff[sg + 1] - poff[sg] == 1;  // the group's only piece: its buckets are all ours
  if (threadIdx.x == 0) {  // exclusive scan of the piece's bin counts (128 entries)
    uint32_t acc = 0;
    for (int i = 0; i < kPbGroupBins; ++i) {
      lpos[i] = acc;
      acc += hist[i];
    }
    lpos[kPbGroupBins] = acc;
  }
  for (int i = threadIdx.x; i < kPbGroupBins; i += kBuildWG) {
    const uint32_t h = hist[i];
    if (alone)
      base[i] = b0 + i < bins ? (unsigned long long)starts[t * bins + b0 + i] : 0ull;
    else
      base[i] = h ? atomicAdd(&cnt[t * bins + b0 + i], (unsigned long long)h) : 0ull;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPbGroupBins; i += kBuildWG) hist[i] = lpos[i];  // LDS cursors
  __syncthreads();
  for (int64_t k = a + threadIdx.x; k < z; k += kBuildWG) {
    const int32_t v = tdst[k];
    const int i = (v >> kPbDstShift) - (int)b0;
    const uint32_t p = atomicAdd(&hist[i], 1u);
    s_srcl[p] = tsrcl[k];
    s_dstl[p] = (uint16_t)(v & ((1 << kPbDstShift) - 1));
    if (weighted) {
      if (wbytes == 1)
        s_w[p] = static_cast<const uint8_t*>(tw)[k];
      else
        reinterpret_cast<uint32_t*>(s_w)[p] = static_cast<const uint32_t*>(tw)[k];
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < cnt_here; p += kBuildWG) {
    int b = 0;  // bin of sorted position p: last b with lpos[b] <= p
    for (int step = kPbGroupBins / 2; step > 0; step >>= 1)
      if (lpos[b + step] <= (uint32_t)p) b += step;
    const int64_t q = (int64_t)base[b] + (int64_t)(p - (int)lpos[b]);
    srcl[q] = s_srcl[p];
    dstl[q] = s_dstl[p];
    if (weighted) {
      if (wbytes == 1)
        static_cast<uint8_t*>(wslot)[q] = s_w[p];
      else
        static_cast<uint32_t*>(wslot)[q] = reinterpret_cast<const uint32_t*>(s_w)[p];
    }
  }
}

// Run tables, one thread per bin b; runs are the non-empty buckets (t, b)
// in tile order.  Count pass: number of runs, edges of the bin (btotal)
// and fold items of up to fcap positions.  Fill pass: for run i of bin b
// (index run_off[b] + i), rpre = its first position in the concatenation
// of the bin's runs and rbase = its first slot minus rpre.
template <bool FILL>
__global__ __launch_bounds__(kWG) void k_pb_tables(const int64_t* __restrict__ starts, int64_t bins, int64_t tiles,
                                                   int64_t fcap, int64_t* __restrict__ nruns,
                                                   int64_t* __restrict__ btotal, int64_t* __restrict__ nitems,
                                                   const int64_t* __restrict__ run_off, int64_t* __restrict__ rpre,
                                                   int64_t* __restrict__ rbase) {
  const int64_t b = gid();
  if (b >= bins) return;
  int64_t acc = 0, runs = 0;
  const int64_t r0 = FILL ? run_off[b] : 0;
  for (int64_t t = 0; t < tiles; ++t) {
    const int64_t q = t * bins + b;
    const int64_t s0 = starts[q], len = starts[q + 1] - s0;
    if (len == 0) continue;
    if (FILL) {
      rpre[r0 + runs] = acc;
      rbase[r0 + runs] = s0 - acc;
    }
    acc += len;
    ++runs;
  }
  if (!FILL) {
    nruns[b] = runs;
    btotal[b] = acc;
    nitems[b] = (acc + fcap - 1) / fcap;
  }
}

// Per bin b (one thread): its fold items, count = ceil(total / fcap) equal
// shares of the bin's positions, cut at multiples of 64 (a share is at least
// 2,048 positions when a bin has several).
__global__ __launch_bounds__(kWG) void k_pb_fold_items(const int64_t* __restrict__ btotal, int64_t bins,
                                                       const int64_t* __restrict__ item_off,
                                                       PbFoldItem* __restrict__ items) {
  const int64_t b = gid();
  if (b >= bins) return;
  const int64_t total = btotal[b];
  const int64_t first = item_off[b], count = item_off[b + 1] - item_off[b];
  auto cut = [&](int64_t i) {
    if (i == count) return total;
    return (total / count * i + (total % count) * i / count) & ~(int64_t)63;
  };
  for (int64_t i = 0; i < count; ++i) items[first + i] = PbFoldItem{(int32_t)b, count == 1 ? 1 : 0, cut(i), cut(i + 1)};
}

// Per bin b: chunks of 64 positions, ceil(total / 64) of them.
__global__ __launch_bounds__(kWG) void k_pb_chunk_counts(const int64_t* __restrict__ btotal, int64_t bins,
                                                         int64_t* __restrict__ nchunks) {
  const int64_t b = gid();
  if (b < bins) nchunks[b] = (btotal[b] + 63) >> 6;
}

// One thread per chunk: chunk c of bin b (positions 64 c .. 64 c + 63 of
// the bin's concatenation of runs) gets the run holding position 64 c and a
// mask of the run starts inside it (bit i: a run starts at 64 c + i,
// i >= 1).  The fold then finds any position's run with one masked
// popcount.  Bin and run are found by binary search (chunk_off: exclusive
// scan of the bins' chunk counts, nchunks in all).
__global__ __launch_bounds__(kWG) void k_pb_chunks(const int64_t* __restrict__ run_off,
                                                   const int64_t* __restrict__ rpre,
                                                   const int64_t* __restrict__ chunk_off, int64_t bins,
                                                   int64_t nchunks, PbChunk* __restrict__ chunks) {
  for (int64_t g = gid(); g < nchunks; g += grid_threads()) {
    int64_t lo = 0, hi = bins - 1;  // the bin: last b with chunk_off[b] <= g (a bin with chunks)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (chunk_off[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t b = lo;
    const int64_t base = (g - chunk_off[b]) * 64;
    const int64_t* P = rpre + run_off[b];
    const int64_t nr = run_off[b + 1] - run_off[b];
    lo = 0;
    hi = nr - 1;  // the run: last r with P[r] <= base (P[0] = 0, runs non-empty)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (P[mid] <= base)
        lo = mid;
      else
        hi = mid - 1;
    }
    unsigned long long starts = 0;
    for (int64_t t = lo + 1; t < nr && P[t] <= base + 63; ++t) starts |= 1ull << (P[t] - base);
    chunks[g] = PbChunk{(int32_t)lo, 0, starts};
  }
}

// Pass 1: one workgroup per spread item; the tile's messages in LDS.
constexpr int kSpreadWG = 1024;
constexpr int kStageU = 4;  // a min window's loads per thread in flight while staging

template <class M>
__global__ __launch_bounds__(kSpreadWG) void k_pb_spread(const PbSpreadItem* __restrict__ items, int64_t n, int shift,
                                                         const uint16_t* __restrict__ srcl, const M* __restrict__ msg,
                                                         M* __restrict__ vals) {
  extern __shared__ __align__(16) unsigned char smem[];
  M* win = reinterpret_cast<M*>(smem);
  const PbSpreadItem it = items[blockIdx.x];
  const int64_t u0 = (int64_t)it.t << shift;
  const int64_t wl = (n - u0 < (1ll << shift)) ? n - u0 : (1ll << shift);
  for (int64_t i = threadIdx.x; i < wl; i += kSpreadWG) win[i] = msg[u0 + i];
  __syncthreads();
  // slots [a, z) (multiples of 4) four per lane: one 8-byte load of source
  // offsets and one store of four messages; the at most 3 + 3 slots
  // outside go one per thread.  (One slot per lane made the 2-byte loads
  // cost the texture addresser as much per byte-moved as 8-byte ones: it
  // was busy about 80 % of the pass.)
  const int64_t au = (it.k0 + 3) & ~(int64_t)3, zd = it.k1 & ~(int64_t)3;
  const int64_t a = au < it.k1 ? au : it.k1, z = zd > a ? zd : a;  // head [k0, a), body [a, z), tail [z, k1)
  if (threadIdx.x < 4) {
    const int64_t k = it.k0 + threadIdx.x;
    if (k < a) vals[k] = win[srcl[k]];
  } else if (threadIdx.x < 8) {
    const int64_t k = z + (threadIdx.x - 4);
    if (k < it.k1) vals[k] = win[srcl[k]];
  }
  if (z <= a) return;
  const int64_t g0 = a >> 2, g1 = z >> 2;
  constexpr int U4 = 2;
  for (int64_t base = g0 + threadIdx.x; base < g1; base += (int64_t)kSpreadWG * U4) {
    uint2 x[U4];
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int64_t g = base + (int64_t)u * kSpreadWG;
      x[u] = reinterpret_cast<const uint2*>(srcl)[g < g1 ? g : g1 - 1];
    }
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int64_t g = base + (int64_t)u * kSpreadWG;
      if (g < g1) {
        const M m0 = win[x[u].x & 0xFFFFu], m1 = win[x[u].x >> 16], m2 = win[x[u].y & 0xFFFFu], m3 = win[x[u].y >> 16];
        if constexpr (sizeof(M) == 4) {
          reinterpret_cast<float4*>(vals)[g] = make_float4(m0, m1, m2, m3);
        } else {
          ulonglong2* o = reinterpret_cast<ulonglong2*>(vals) + 2 * g;
          o[0] = make_ulonglong2(m0, m1);
          o[1] = make_ulonglong2(m2, m3);
        }
      }
    }
  }
}

// wmin[i] = value of vertex u0 + i, or kInf when ACT and its frontier bit
// is clear, for i < wl (wl > 0).  Clamped loads, so they issue together.
template <bool ACT>
__device__ __forceinline__ void stage_min_window(uint32_t* wmin, const uint2* __restrict__ vm,
                                                 const uint32_t* __restrict__ active, int64_t u0, int64_t wl) {
  for (int64_t i0 = threadIdx.x; i0 < wl; i0 += (int64_t)kSpreadWG * kStageU) {
    uint32_t v[kStageU], on[kStageU];
#pragma unroll
    for (int s = 0; s < kStageU; ++s) {
      const int64_t i = i0 + (int64_t)s * kSpreadWG;
      const int64_t u = u0 + (i < wl ? i : wl - 1);
      v[s] = vm[u].x;
      on[s] = ACT ? (active[u >> 5] >> (u & 31)) & 1u : 1u;
    }
#pragma unroll
    for (int s = 0; s < kStageU; ++s) {
      const int64_t i = i0 + (int64_t)s * kSpreadWG;
      if (i < wl) wmin[i] = on[s] ? v[s] : kInf;
    }
  }
}

// Pass 1 of a min program (CC, SSSP): the tile's values in LDS, a source
// that is not in the frontier (bit clear in `active`; NULL: every vertex)
// reading as unreached, then vals[k] = the message on slot k: the value
// (CC) or the value plus the edge's weight (SSSP, saturating; unweighted:
// plus 1), unreached (kInf) for an inactive source.  Slot weights are bytes
// (WT = uint8_t) when every weight of the graph fits one.  Slot messages are
// MT: uint32_t, or uint16_t when the caller knows every message of the
// superstep is below 0xFFFF, which then stands for unreached.
template <class MT>
__device__ __forceinline__ MT slot_msg(uint32_t m) {
  if constexpr (sizeof(MT) == 2)
    return (MT)(m < 0xFFFFu ? m : 0xFFFFu);
  else
    return m;
}

template <int KIND, class WT, class MT>
__global__ __launch_bounds__(kSpreadWG) void k_pb_spread_min(const PbSpreadItem* __restrict__ items, int64_t n,
                                                             int shift, const uint16_t* __restrict__ srcl,
                                                             const WT* __restrict__ wslot,
                                                             const uint2* __restrict__ vm,
                                                             const uint32_t* __restrict__ active,
                                                             MT* __restrict__ vals,
                                                             const LoopState* __restrict__ loop) {
  extern __shared__ __align__(16) uint32_t wmin[];
  if (loop && (loop->done || loop->mode != VC_SCHED_BLOCKED)) return;  // uniform: another form runs this superstep
  const PbSpreadItem it = items[blockIdx.x];
  const int64_t u0 = (int64_t)it.t << shift;
  const int64_t wl = (n - u0 < (1ll << shift)) ? n - u0 : (1ll << shift);
  if (active)
    stage_min_window<true>(wmin, vm, active, u0, wl);
  else
    stage_min_window<false>(wmin, vm, active, u0, wl);
  __syncthreads();
  auto msg_of = [&](uint32_t src, uint32_t w) -> MT {
    const uint32_t val = wmin[src];
    return slot_msg<MT>(KIND == kCC ? val : sat_add(val, w));  // kInf stays unreached
  };
  // slots [a, z) (multiples of 4) four per lane: one load of source offsets,
  // one of weights and one store of four messages; the at most 3 + 3 slots
  // outside go one per thread
  const int64_t au = (it.k0 + 3) & ~(int64_t)3, zd = it.k1 & ~(int64_t)3;
  const int64_t a = au < it.k1 ? au : it.k1, z = zd > a ? zd : a;  // head [k0, a), body [a, z), tail [z, k1)
  if (threadIdx.x < 8) {
    const int64_t k = threadIdx.x < 4 ? it.k0 + threadIdx.x : z + (threadIdx.x - 4);
    if (threadIdx.x < 4 ? k < a : k < it.k1)
      vals[k] = msg_of(srcl[k], KIND == kSsspWeighted ? (uint32_t)wslot[k] : 1u);
  }
  if (z <= a) return;
  const int64_t g0 = a >> 2, g1 = z >> 2;
  constexpr int U4 = 2;
  using W4 = typename std::conditional<sizeof(WT) == 1, uint32_t, uint4>::type;
  for (int64_t base = g0 + threadIdx.x; base < g1; base += (int64_t)kSpreadWG * U4) {
    uint2 x[U4];
    W4 wq[U4];
#pragma unroll
    for (int u = 0; u < U4; ++u) {  // unconditional (clamped) loads: all issue before the first wait
      const int64_t g = base + (int64_t)u * kSpreadWG;
      const int64_t gc = g < g1 ? g : g1 - 1;
      x[u] = reinterpret_cast<const uint2*>(srcl)[gc];
      if (KIND == kSsspWeighted) wq[u] = reinterpret_cast<const W4*>(wslot)[gc];
    }
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const int64_t g = base + (int64_t)u * kSpreadWG;
      if (g < g1) {
        uint32_t w0 = 1u, w1 = 1u, w2 = 1u, w3 = 1u;
        if constexpr (KIND == kSsspWeighted) {
          if constexpr (sizeof(WT) == 1) {
            w0 = wq[u] & 0xFFu;
            w1 = (wq[u] >> 8) & 0xFFu;
            w2 = (wq[u] >> 16) & 0xFFu;
            w3 = wq[u] >> 24;
          } else {
            w0 = wq[u].x;
            w1 = wq[u].y;
            w2 = wq[u].z;
            w3 = wq[u].w;
          }
        }
        const MT m0 = msg_of(x[u].x & 0xFFFFu, w0), m1 = msg_of(x[u].x >> 16, w1);
        const MT m2 = msg_of(x[u].y & 0xFFFFu, w2), m3 = msg_of(x[u].y >> 16, w3);
        if constexpr (sizeof(MT) == 2)
          reinterpret_cast<uint2*>(vals)[g] = make_uint2((uint32_t)m0 | ((uint32_t)m1 << 16),
                                                         (uint32_t)m2 | ((uint32_t)m3 << 16));
        else
          reinterpret_cast<uint4*>(vals)[g] = make_uint4(m0, m1, m2, m3);
      }
    }
  }
}

// Pass 2: one workgroup per fold item.  The item's chunk descriptors (one
// per 64 positions: first run, run starts inside) are staged in LDS once;
// its runs' slot bases in windows of kFoldRuns runs.  Per window,
// wavefronts take the chunks overlapping the window's positions round
// robin, U at a time, lane l the position 64 c + l, so every load
// instruction reads 64 consecutive positions; a lane's run is its chunk's
// first run plus the run starts at or below its position (one masked
// popcount) and its slot that run's base plus the position.  Item j runs on
// workgroup j, so the hardware's round-robin dispatch deals consecutive
// items to different XCDs: bins come hottest first, and handing each XCD a
// contiguous eighth of the items instead left the XCDs with 0.7-17.5 % of
// the positions each (scale 24), the fold as slow as the busiest XCD.
constexpr int kFoldWG = 1024;
constexpr int kFoldRuns = 1024;
constexpr int kFoldChunks = (int)(kPbMaxItemPositions / 64 + 1);  // an item's chunks, from a multiple of 64
static_assert((1 << kPbDstShift) % kFoldWG == 0, "the min fold's flush runs every lane in every round");

// The combiners of the fold.  Sum (PageRank): exact fixed-point mailboxes,
// all stored for a bin that is one item, added otherwise.  Min (CC, SSSP): as the
// pull form, a receiver whose best message lowers its value takes it into
// its mailbox (stored for a bin that is one item, an atomic min otherwise)
// and its improvement bit is set.
template <class M>
struct FoldSum {
  using Val = M;
  using Box = unsigned long long;
  unsigned long long* mb;
  static constexpr Box kEmpty = 0ull;
  __device__ __forceinline__ static void add(Box* box, uint16_t d, Val v) {
    const unsigned long long x = msg_to_sum<M, unsigned long long>(v);
    if (x) atomicAdd(&box[d], x);
  }
  __device__ __forceinline__ void flush(const PbFoldItem& it, const Box* box, int64_t n) const {
    const int64_t v0 = (int64_t)it.b << kPbDstShift;
    for (int i = threadIdx.x; i < (1 << kPbDstShift) && v0 + i < n; i += kFoldWG) {
      const unsigned long long x = box[i];
      if (it.whole)
        mb[v0 + i] = x;  // the only item of this bin: every mailbox stored, so none needs a reset
      else if (x)
        atomicAdd(&mb[v0 + i], x);
    }
  }
};

template <class V>
struct FoldMinT {
  using Val = V;  // slot messages: uint32_t, or uint16_t with 0xFFFF for unreached
  using Box = uint32_t;
  uint2* vm;
  uint32_t* improved;
  static constexpr Box kEmpty = kInf;
  __device__ __forceinline__ static void add(Box* box, uint16_t d, Val v) {
    if (v != Val(~Val(0))) atomicMin(&box[d], (uint32_t)v);
  }
  __device__ __forceinline__ void flush(const PbFoldItem& it, const Box* box, int64_t n) const {
    constexpr int R = (1 << kPbDstShift) / kFoldWG;  // rounds; every lane runs every round
    const int64_t v0 = (int64_t)it.b << kPbDstShift;  // a multiple of 64: lanes 0..31 and 32..63 fill one word each
    const int lane = threadIdx.x & 63;
    uint32_t best[R];
    uint2 cur[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {  // all rounds' loads first, clamped to vertex n - 1 (v0 < n), so they issue together
      const int64_t v = v0 + threadIdx.x + r * kFoldWG;
      best[r] = box[threadIdx.x + r * kFoldWG];
      cur[r] = vm[v < n ? v : n - 1];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t v = v0 + threadIdx.x + r * kFoldWG;
      bool imp = false;
      if (v < n && best[r] != kInf && best[r] < cur[r].x) {
        if (it.whole) {
          vm[v].y = best[r];
          imp = true;
        } else if (best[r] < cur[r].y) {
          const uint32_t old = atomicMin(&reinterpret_cast<uint32_t*>(vm)[2 * v + 1], best[r]);
          imp = old == kInf;  // the first improver of v sets its bit
        }
      }
      const unsigned long long mask = __ballot(imp);
      if (lane == 0 && (uint32_t)mask) atomicOr(&improved[v >> 5], (uint32_t)mask);
      if (lane == 32 && (uint32_t)(mask >> 32)) atomicOr(&improved[v >> 5], (uint32_t)(mask >> 32));
    }
  }
};
using FoldMin = FoldMinT<uint32_t>;
using FoldMin16 = FoldMinT<uint16_t>;

template <class Op>
__global__ __launch_bounds__(kFoldWG) void k_pb_fold(const PbFoldItem* __restrict__ items, int64_t nitems,
                                                     const int64_t* __restrict__ run_off,
                                                     const int64_t* __restrict__ rpre,
                                                     const int64_t* __restrict__ btotal,
                                                     const int64_t* __restrict__ chunk_off,
                                                     const PbChunk* __restrict__ chunks,
                                                     const int64_t* __restrict__ rbase, int64_t n,
                                                     const typename Op::Val* __restrict__ vals,
                                                     const uint16_t* __restrict__ dstl, Op op,
                                                     const LoopState* __restrict__ loop) {
  using M = typename Op::Val;
  using Box = typename Op::Box;
  constexpr int U = 8;
  constexpr int W = kFoldWG / 64;  // wavefronts
  __shared__ Box box[1 << kPbDstShift];
  __shared__ int64_t s_base[kFoldRuns];
  __shared__ PbChunk s_chunk[kFoldChunks];
  if (loop && (loop->done || loop->mode != VC_SCHED_BLOCKED)) return;  // uniform: another form runs this superstep
  const int64_t j = blockIdx.x;
  if (j >= nitems) return;
  const PbFoldItem it = items[j];
  const int64_t R0 = run_off[it.b], nr = run_off[it.b + 1] - R0, total = btotal[it.b];
  const int64_t cfirst = it.v0 >> 6, c_end = (it.v1 + 63) >> 6;  // it.v0 is a multiple of 64
  const int nch = (int)(c_end - cfirst);                           // <= kFoldChunks
  for (int i = threadIdx.x; i < (1 << kPbDstShift); i += kFoldWG) box[i] = Op::kEmpty;
  for (int i = threadIdx.x; i < nch; i += kFoldWG) s_chunk[i] = chunks[chunk_off[it.b] + cfirst + i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // bits 0..lane
  const int64_t r_first = s_chunk[0].rb;
  const int64_t r_last = s_chunk[nch - 1].rb + __popcll(s_chunk[nch - 1].starts);  // run of the item's last chunk's end
  for (int64_t w0 = r_first; w0 <= r_last; w0 += kFoldRuns) {
    const int wn = (int)((r_last + 1 - w0 < kFoldRuns) ? r_last + 1 - w0 : kFoldRuns);
    for (int i = threadIdx.x; i < wn; i += kFoldWG) s_base[i] = rbase[R0 + w0 + i];
    __syncthreads();
    // positions of the window's runs, within the item
    const int64_t pa = rpre[R0 + w0], pz = w0 + wn < nr ? rpre[R0 + w0 + wn] : total;
    const int64_t a = pa > it.v0 ? pa : it.v0, z = pz < it.v1 ? pz : it.v1;
    for (int64_t c = (a >> 6) + wave; c <= ((z - 1) >> 6); c += (int64_t)W * U) {
      int64_t k[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t cc = c + (int64_t)u * W;
        k[u] = -1;
        const int64_t q = cc * 64 + lane;
        if (cc <= ((z - 1) >> 6) && q >= a && q < z) {
          const PbChunk ch = s_chunk[cc - cfirst];
          k[u] = s_base[ch.rb + __popcll(ch.starts & upto) - w0] + q;  // the run lies in this window: q in [a, z)
        }
      }
      uint16_t dl[U];
      M raw[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // all loads first, then the conversions and adds
        dl[u] = k[u] >= 0 ? dstl[k[u]] : 0;
        raw[u] = k[u] >= 0 ? vals[k[u]] : M(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k[u] >= 0) Op::add(box, dl[u], raw[u]);
    }
    __syncthreads();
  }
  op.flush(it, box, n);
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

hipError_t launch_pb_wmax(const uint32_t* w, int64_t m, uint32_t* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int64_t g = (m / 4 + kWG - 1) / kWG;  // one 16-byte load per thread at most, 2,048 workgroups at most
  hipLaunchKernelGGL(k_pb_wmax, dim3((unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048)), dim3(kWG), 0, s, w, m, out);
  return hipGetLastError();
}

hipError_t launch_pb_build(bool place, const int64_t* te, int64_t tiles, const int32_t* dst, int64_t m, int64_t chunk,
                           int64_t bins, int pass_bins, unsigned long long* cnt, const uint16_t* srcl_csr,
                           uint16_t* srcl, uint16_t* dstl, const uint32_t* w, void* wslot, int wbytes,
                           hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (pass_bins < 1 || chunk < 1) return hipErrorInvalidValue;
  const int64_t grid = (m + chunk - 1) / chunk;
  const size_t lds = (size_t)pass_bins * (place ? 8 : 4);
  if (place)
    hipLaunchKernelGGL(k_pb_build<true>, dim3((unsigned)grid), dim3(kBuildWG), lds, s, te, tiles, dst, m, chunk, bins,
                       pass_bins, cnt, srcl_csr, srcl, dstl, w, wslot, wbytes);
  else
    hipLaunchKernelGGL(k_pb_build<false>, dim3((unsigned)grid), dim3(kBuildWG), lds, s, te, tiles, dst, m, chunk, bins,
                       pass_bins, cnt, srcl_csr, srcl, dstl, nullptr, nullptr, 4);
  return hipGetLastError();
}

int64_t pb_groups(int64_t bins) { return (bins + kPbGroupBins - 1) / kPbGroupBins; }
size_t pb_place_lds(bool weighted, int wbytes) {
  return (size_t)kPbPiece * (4 + (weighted ? (size_t)wbytes : 0)) + 2048;  // + the static part
}

hipError_t launch_pb_group_starts(const int64_t* starts, int64_t tiles, int64_t bins, unsigned long long* gcur,
                                  int64_t* pieces, hipStream_t s) {
  const int64_t groups = pb_groups(bins);
  if (tiles * groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_group_starts, dim3(grid_for(tiles * groups)), dim3(kWG), 0, s, starts, tiles, bins, groups,
                     gcur, pieces);
  return hipGetLastError();
}

hipError_t launch_pb_group(const int64_t* te, int64_t tiles, const int32_t* dst, int64_t m, int64_t chunk,
                           int64_t bins, unsigned long long* gcur, const uint16_t* srcl_csr, const uint32_t* w,
                           int wbytes, int32_t* tdst, uint16_t* tsrcl, void* tw, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (chunk < 1) return hipErrorInvalidValue;
  const int64_t groups = pb_groups(bins);
  const int64_t grid = (m + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_pb_group, dim3((unsigned)grid), dim3(kBuildWG), (size_t)groups * 12, s, te, tiles, dst, m,
                     chunk, groups, gcur, srcl_csr, w, wbytes, tdst, tsrcl, tw);
  return hipGetLastError();
}

hipError_t launch_pb_place(const int64_t* poff, int64_t tiles, int64_t bins, int64_t npieces, const int64_t* starts,
                           unsigned long long* cnt, const int32_t* tdst, const uint16_t* tsrcl, const void* tw,
                           int wbytes, bool weighted, uint16_t* srcl, uint16_t* dstl, void* wslot, hipStream_t s) {
  if (npieces <= 0) return hipSuccess;
  const int64_t groups = pb_groups(bins);
  const size_t lds = pb_place_lds(weighted, wbytes) - 2048;
  hipLaunchKernelGGL(k_pb_place, dim3((unsigned)npieces), dim3(kBuildWG), lds, s, poff, tiles * groups, groups, bins,
                     starts, cnt, tdst, tsrcl, tw, wbytes, weighted, srcl, dstl, wslot);
  return hipGetLastError();
}

hipError_t launch_pb_tables(bool fill, const int64_t* starts, int64_t bins, int64_t tiles, int64_t fcap,
                            int64_t* nruns, int64_t* btotal, int64_t* nitems, const int64_t* run_off, int64_t* rpre,
                            int64_t* rbase, hipStream_t s) {
  if (fill)
    hipLaunchKernelGGL(k_pb_tables<true>, dim3(grid_for(bins)), dim3(kWG), 0, s, starts, bins, tiles, fcap, nruns,
                       btotal, nitems, run_off, rpre, rbase);
  else
    hipLaunchKernelGGL(k_pb_tables<false>, dim3(grid_for(bins)), dim3(kWG), 0, s, starts, bins, tiles, fcap, nruns,
                       btotal, nitems, run_off, rpre, rbase);
  return hipGetLastError();
}

hipError_t launch_pb_fold_items(const int64_t* btotal, int64_t bins, const int64_t* item_off, PbFoldItem* items,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_pb_fold_items, dim3(grid_for(bins)), dim3(kWG), 0, s, btotal, bins, item_off, items);
  return hipGetLastError();
}

hipError_t launch_pb_chunk_counts(const int64_t* btotal, int64_t bins, int64_t* nchunks, hipStream_t s) {
  hipLaunchKernelGGL(k_pb_chunk_counts, dim3(grid_for(bins)), dim3(kWG), 0, s, btotal, bins, nchunks);
  return hipGetLastError();
}

hipError_t launch_pb_chunks(const int64_t* run_off, const int64_t* rpre, const int64_t* chunk_off, int64_t bins,
                            int64_t nchunks, PbChunk* chunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pb_chunks, dim3(grid_stride_for(nchunks)), dim3(kWG), 0, s, run_off, rpre, chunk_off, bins,
                     nchunks, chunks);
  return hipGetLastError();
}

hipError_t launch_pb_spread(bool f32msg, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                            const uint16_t* srcl, const void* msg, void* vals, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (shift < 10 || shift > kMaxSrcShift) return hipErrorInvalidValue;
  if (f32msg)
    hipLaunchKernelGGL(k_pb_spread<float>, dim3((unsigned)nitems), dim3(kSpreadWG), (size_t)4 << shift, s, items, n,
                       shift, srcl, (const float*)msg, (float*)vals);
  else
    hipLaunchKernelGGL(k_pb_spread<unsigned long long>, dim3((unsigned)nitems), dim3(kSpreadWG), (size_t)8 << shift,
                       s, items, n, shift, srcl, (const unsigned long long*)msg, (unsigned long long*)vals);
  return hipGetLastError();
}

hipError_t launch_pb_fold(bool f32msg, const PbFoldItem* items, int64_t nitems, const int64_t* run_off,
                          const int64_t* rpre, const int64_t* btotal, const int64_t* chunk_off, const PbChunk* chunks,
                          const int64_t* rbase, int64_t n, const void* vals, const uint16_t* dstl,
                          unsigned long long* mb, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (f32msg)
    hipLaunchKernelGGL(k_pb_fold<FoldSum<float>>, dim3((unsigned)nitems), dim3(kFoldWG), 0, s, items, nitems,
                       run_off, rpre, btotal, chunk_off, chunks, rbase, n, (const float*)vals, dstl,
                       FoldSum<float>{mb}, nullptr);
  else
    hipLaunchKernelGGL(k_pb_fold<FoldSum<unsigned long long>>, dim3((unsigned)nitems), dim3(kFoldWG), 0, s, items,
                       nitems, run_off, rpre, btotal, chunk_off, chunks, rbase, n,
                       (const unsigned long long*)vals, dstl, FoldSum<unsigned long long>{mb}, nullptr);
  return hipGetLastError();
}

namespace {
template <class WT, class MT>
hipError_t spread_min_launch(int kind, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                             const uint16_t* srcl, const WT* wslot, const uint2* vm, const uint32_t* active,
                             MT* vals, const LoopState* loop, hipStream_t s) {
  const size_t lds = (size_t)4 << shift;
  switch (kind) {
    case kCC:
      hipLaunchKernelGGL((k_pb_spread_min<kCC, WT, MT>), dim3((unsigned)nitems), dim3(kSpreadWG), lds, s, items, n,
                         shift, srcl, wslot, vm, active, vals, loop);
      break;
    case kSsspUnit:
      hipLaunchKernelGGL((k_pb_spread_min<kSsspUnit, WT, MT>), dim3((unsigned)nitems), dim3(kSpreadWG), lds, s, items,
                         n, shift, srcl, wslot, vm, active, vals, loop);
      break;
    case kSsspWeighted:
      hipLaunchKernelGGL((k_pb_spread_min<kSsspWeighted, WT, MT>), dim3((unsigned)nitems), dim3(kSpreadWG), lds, s,
                         items, n, shift, srcl, wslot, vm, active, vals, loop);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class WT>
hipError_t spread_min_width(bool narrow, int kind, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                            const uint16_t* srcl, const WT* wslot, const uint2* vm, const uint32_t* active,
                            void* vals, const LoopState* loop, hipStream_t s) {
  if (narrow)
    return spread_min_launch(kind, items, nitems, n, shift, srcl, wslot, vm, active, static_cast<uint16_t*>(vals),
                             loop, s);
  return spread_min_launch(kind, items, nitems, n, shift, srcl, wslot, vm, active, static_cast<uint32_t*>(vals), loop,
                           s);
}
}  // namespace

hipError_t launch_pb_spread_min(int kind, const PbSpreadItem* items, int64_t nitems, int64_t n, int shift,
                                const uint16_t* srcl, const void* wslot, int wbytes, const uint2* vm,
                                const uint32_t* active, void* vals, bool narrow, const LoopState* loop,
                                hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (shift < 10 || shift > kMaxSrcShift) return hipErrorInvalidValue;
  if (kind == kSsspWeighted && !wslot) return hipErrorInvalidValue;
  if (narrow && kind == kCC) return hipErrorInvalidValue;  // labels are vertex ids
  if (wbytes == 1)
    return spread_min_width(narrow, kind, items, nitems, n, shift, srcl, static_cast<const uint8_t*>(wslot), vm,
                            active, vals, loop, s);
  return spread_min_width(narrow, kind, items, nitems, n, shift, srcl, static_cast<const uint32_t*>(wslot), vm, active,
                          vals, loop, s);
}

hipError_t launch_pb_fold_min(const PbFoldItem* items, int64_t nitems, const int64_t* run_off,
                              const int64_t* rpre, const int64_t* btotal, const int64_t* chunk_off,
                              const PbChunk* chunks, const int64_t* rbase, int64_t n, const void* vals, bool narrow,
                              const uint16_t* dstl, uint2* vm, uint32_t* improved, const LoopState* loop,
                              hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (narrow)
    hipLaunchKernelGGL(k_pb_fold<FoldMin16>, dim3((unsigned)nitems), dim3(kFoldWG), 0, s, items, nitems, run_off,
                       rpre, btotal, chunk_off, chunks, rbase, n, static_cast<const uint16_t*>(vals), dstl,
                       FoldMin16{vm, improved}, loop);
  else
    hipLaunchKernelGGL(k_pb_fold<FoldMin>, dim3((unsigned)nitems), dim3(kFoldWG), 0, s, items, nitems, run_off,
                       rpre, btotal, chunk_off, chunks, rbase, n, static_cast<const uint32_t*>(vals), dstl,
                       FoldMin{vm, improved}, loop);
  return hipGetLastError();
}

}  // namespace vc

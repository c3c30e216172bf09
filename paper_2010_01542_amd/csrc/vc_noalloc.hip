// vc_run_noalloc: vc_run for callers that cannot allocate device memory.
//
// The run's workspace (values and mailboxes, frontier bitmaps, broadcast
// list, degree prefix, scan scratch, partitions of the superstep's list,
// counters; PageRank messages and sums) lives in one fixed device array of
// this library instead of the graph's own buffers.  Each GPU the library runs
// on holds its own copy of the array, at its own address, until the process
// ends; that address is looked up once per device and passed to the kernels
// like any other buffer.  Every call on a GPU shares that GPU's array and
// leaves its contents behind; the run initialises every piece it reads, so a
// call never depends on what an earlier one left.  Calls that overlap on one
// GPU (two host threads, or two streams in flight at once) race on it.
#include <mutex>

#include "vc_graph.h"

// File scope, so that its address can be looked up by symbol.  Host code
// names it only in the lookup below: on the host it is a stand-in, not a
// device address.
static __device__ __align__(256) unsigned char scratch[VC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device, once looked up

// Address of the current device's copy of `scratch`; looked up on the first
// call made with that device current.
vc_status scratch_of(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return vc::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return vc::fail(VC_ERR_HIP, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[dev];
  return VC_OK;
}

}  // namespace

extern "C" vc_status vc_run_noalloc(vc_graph g, vc_program program, const vc_params* params, void* out,
                                    hipStream_t stream, vc_stats* stats) {
  if (!g) return vc::fail(VC_ERR_INVALID_ARG, "null graph");
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return vc::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return vc::fail(VC_ERR_UNSUPPORTED, "device ordinal beyond the library's table");
  unsigned char* base = nullptr;
  const vc_status st = scratch_of(dev, &base);
  if (st != VC_OK) return st;
  vc::Arena arena;
  arena.base = base;
  arena.bytes = VC_NOALLOC_SCRATCH_BYTES;
  return vc::run_entry(g, program, params, out, stream, stats, &arena);
}

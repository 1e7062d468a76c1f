// dg_sssp_noalloc: Bellman-Ford single-source shortest paths (as dg_sssp)
// for callers that cannot allocate memory during the call.  Every device
// buffer the sweeps need beyond the caller's graph and output lives in one
// fixed array of this library, `scratch`, whose device address is looked up
// once per device; the call makes no device or pinned-host allocation, no
// event, and no allocating library call.
//
// Scratch layout for a graph of n vertices and K compact-region slots (each
// part 256-byte aligned): the distance array [n+K] (two in synchronous mode),
// the per-vertex staging shadow [n] (delayed modes that stage there), a
// vertex-order staging copy of the result [n] (host output only), and the
// per-sweep state (stopping flags, worker counts, per-worker partials).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "dg.h"
#include "dg_graph.hpp"
#include "dg_host.hpp"
#include "dg_internal.hpp"

namespace dg {
namespace {

constexpr size_t kScratchBytes = DG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr uint32_t kNoAllocMaxSweeps = 65535;
constexpr uint32_t kFirstChunk = 4, kMaxChunk = 32;

// The scratch array.  Host code never uses its name as an address: it uses
// the device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up on the first
// call on the device (with that device current).
dg_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return host::fail(DG_ERR_DEVICE, "no usable HIP device: %s", hipGetErrorString(e));
  }
  if (dev < 0 || dev >= kMaxDevices) return host::fail(DG_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return host::fail(DG_ERR_DEVICE, "looking up the scratch array failed: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

// Bump allocation inside the scratch array (256-byte aligned parts).
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += (count * sizeof(T) + 255) & ~(size_t)255;
    return p;
  }
};

}  // namespace
}  // namespace dg

using dg::host::fail;

extern "C" dg_status dg_sssp_noalloc(dg_graph* g, uint32_t src, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                                     uint32_t* out_dist, int out_on_device, dg_stats* stats, void* hip_stream) {
  using namespace dg;
  host::g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (g->G) return fail(DG_ERR_UNSUPPORTED, "the union graph of a set is not supported");
  if (!g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "graph was created without weights");
  if (src >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "source %u >= n = %u", src, g->n);
  if (mode != DG_SYNC && mode != DG_ASYNC && mode != DG_DELAYED)
    return fail(DG_ERR_INVALID_ARGUMENT, "mode %d is not DG_SYNC, DG_ASYNC or DG_DELAYED", (int)mode);
  if (mode == DG_DELAYED && d == 0) return fail(DG_ERR_INVALID_ARGUMENT, "delayed mode needs d >= 1");
  if (max_sweeps == 0 || max_sweeps > kNoAllocMaxSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps must be in [1, %u]", kNoAllocMaxSweeps);
  if (!out_dist) return fail(DG_ERR_INVALID_ARGUMENT, "out_dist is NULL");

  // Staging of delayed commits, as dg_sssp chooses it.
  const uint32_t nres = std::min<uint32_t>(g->R, kResBytes / 4u);
  uint32_t d_eff = 0, cap = 0;
  bool use_shadow = false;
  if (mode == DG_DELAYED) host::staging(g, d, sizeof(uint32_t), nres, cap, d_eff, use_shadow);

  // Scratch needed; refused beyond the array's size.
  const size_t slots = (size_t)g->n + g->K;
  const size_t S1 = (size_t)max_sweeps + 1;
  auto part = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
  const size_t need = part(slots * 4) * (mode == DG_SYNC ? 2 : 1) + (use_shadow ? part((size_t)g->n * 4) : 0) +
                      (out_on_device ? 0 : part((size_t)g->n * 4)) + 2 * part(S1 * 8) + 2 * part(S1 * 4) +
                      part(3 * (size_t)g->P * 8);
  if (need > kScratchBytes)
    return fail(DG_ERR_UNSUPPORTED, "this call needs %zu bytes of scratch; the fixed scratch array holds %zu",
                need, kScratchBytes);
  void* base = nullptr;
  dg_status st = scratch_address(&base);
  if (st != DG_OK) return st;
  Carve cv{static_cast<unsigned char*>(base)};
  uint32_t* b0 = cv.take<uint32_t>(slots);
  uint32_t* b1 = mode == DG_SYNC ? cv.take<uint32_t>(slots) : nullptr;
  uint32_t* sh = use_shadow ? cv.take<uint32_t>(g->n) : nullptr;
  uint32_t* ostage = out_on_device ? nullptr : cv.take<uint32_t>(g->n);
  SweepState sst;
  sst.resid = cv.take<double>(S1);
  sst.dang = cv.take<double>(S1);
  sst.count = cv.take<uint32_t>(S1);
  sst.changed = cv.take<uint32_t>(S1);
  sst.part = cv.take<double>(3 * (size_t)g->P);
  sst.hresid = nullptr;
  sst.hchanged = nullptr;

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // Every state entry a sweep reads is written here (fill kernels, no memset).
  DG_HIP(launch_bf_init(b0, b1, g->cpos, g->n, src, sst, max_sweeps, s));
  BfArgs a;
  std::memset(&a, 0, sizeof a);
  a.g = host::topo(g);
  a.st = sst;
  a.d = d_eff;
  a.cap = cap;
  a.res = nres;
  a.shadow = sh;

  // Sweeps are queued in chunks of 4, 8, 16, then 32; each queued sweep
  // exits at once on the device if an earlier one made no update.  After a
  // chunk the host copies the chunk's stopping flags (into a stack array) and
  // looks for the first sweep that changed nothing.
  const auto t0 = std::chrono::steady_clock::now();
  uint32_t next = 0, chunk = kFirstChunk, sweeps = 0;
  bool conv = false;
  while (next < max_sweeps && !conv) {
    const uint32_t c = std::min(chunk, max_sweeps - next);
    for (uint32_t k = next; k < next + c; ++k) {
      if (mode == DG_SYNC) {
        a.din = (k & 1) ? b1 : b0;
        a.dout = (k & 1) ? b0 : b1;
      } else {
        a.din = b0;
        a.dout = b0;
      }
      a.k = k;
      DG_HIP(launch_bf_sweep((int)mode, a, s));
    }
    uint32_t flags[kMaxChunk];
    DG_HIP(hipMemcpyAsync(flags, sst.changed + next + 1, (size_t)c * 4, hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < c; ++i)
      if (flags[i] == 0) {  // sweep next+i changed nothing
        sweeps = next + i + 1;
        conv = true;
        break;
      }
    next += c;
    chunk = std::min(2 * chunk, kMaxChunk);
  }
  if (!conv) sweeps = max_sweeps;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

  // The last executed sweep k = sweeps-1 wrote buffer (k+1) % 2 in sync mode.
  const uint32_t* res = (mode == DG_SYNC && (sweeps & 1)) ? b1 : b0;
  uint32_t* dst = out_on_device ? out_dist : ostage;
  DG_HIP(launch_bf_gather(res, g->cpos, g->n, dst, s));
  if (!out_on_device) DG_HIP(hipMemcpyAsync(out_dist, dst, (size_t)g->n * 4, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->sweeps = sweeps;
    stats->workers = g->P;
    stats->tile_vertices = g->T ? (uint32_t)(((uint64_t)g->n + g->T / 2) / g->T) : 0u;
    stats->commits = mode == DG_DELAYED ? host::commits_per_sweep(g, d_eff, cap, use_shadow) : 0u;
    stats->commit_interval =
        stats->commits ? (uint32_t)(((uint64_t)g->n + stats->commits / 2) / stats->commits) : 0u;
    stats->seconds = secs;
    stats->edges_traversed = g->m * (uint64_t)sweeps;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "no convergence within %u sweeps", max_sweeps);
  return DG_OK;
}

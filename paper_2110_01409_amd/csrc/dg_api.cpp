// Host side of the C ABI declared in include/dg.h: argument validation,
// in-edge (CSC) construction, tiling and the blocked worker partition, device
// memory, and the sweep driver with device-side termination.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dg.h"
#include "dg_graph.hpp"
#include "dg_host.hpp"
#include "dg_internal.hpp"
#include "dg_plan.hpp"

using namespace dg;
using dg::host::fail;
using dg::host::g_last_error;

namespace {

std::mutex g_alloc_mu;
dg_alloc_fn g_alloc = nullptr;
dg_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;

}  // namespace

namespace dg {
namespace host {

thread_local std::string g_last_error;

dg_status fail(dg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

void current_allocator(dg_alloc_fn& alloc, dg_free_fn& free_fn, void*& ctx) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  alloc = g_alloc;
  free_fn = g_free;
  ctx = g_alloc_ctx;
}

}  // namespace host
}  // namespace dg


using dg::host::kMaxSweeps;
using dg::host::kEventRing;
using dg::host::kHostReactUs;
using dg::host::kMaxLookahead;
using dg::host::kWorkersPerCU;
using dg::host::kBatchSsspWorkersPerCU;
using dg::host::kBatchPprWorkersPerCU;
using dg::host::kBatchSssp;
using dg::host::kBatchPpr;
using dg::host::BatchPart;
using dg::host::kSetWorkersPerCU;
using dg::host::topo_batch;
using dg::host::build_layout;
using dg::host::build_workers;
using dg::host::build_workers_seg;
using dg::host::build_tiles;
using dg::host::plan_workers;
using dg::host::Layout;
using dg::host::validate_graph;

namespace dg {
namespace host {

void* dev_alloc(dg_graph* g, size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (g->alloc) {
    p = g->alloc(bytes, s, g->ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) g->owned.push_back(p);
  return p;
}

void dev_free(dg_graph* g, void* p) {
  if (!p) return;
  auto it = std::find(g->owned.begin(), g->owned.end(), p);
  if (it != g->owned.end()) g->owned.erase(it);
  if (g->free_fn) g->free_fn(p, g->create_stream, g->ctx);
  else (void)hipFree(p);
}

}  // namespace host
}  // namespace dg

namespace dg {
namespace host {

Topology topo(const dg_graph* g) {
  Topology t;
  t.in_ptr = g->in_ptr;
  t.in_src = g->in_src;
  t.in_w = g->in_w;
  t.in_w8 = g->in_w8;
  t.out_deg = g->out_deg;
  t.cpos = g->cpos;
  t.tile_v = g->tile_v;
  t.work_t = g->work_t;
  t.n = g->n;
  t.K = g->K;
  t.P = g->P;
  t.variant = g->variant;
  return t;
}

Topology topo_batch(const dg_graph* g, int which) {
  Topology t = topo(g);
  t.tile_v = g->btile_v;
  t.work_t = g->bp[which].work_t;
  t.P = g->bp[which].P;
  return t;
}

}  // namespace host
}  // namespace dg

using dg::host::dev_alloc;
using dg::host::dev_free;
using dg::host::topo;

namespace dg {
namespace host {

// Staging for a commit interval d.  LDS holds d values plus one more tile
// (each staged vertex keeps its value and the 4-byte slot it is committed
// to) when that fits next to the resident table (res values) and the
// kernel's static LDS in kLdsBudget (the compute unit's LDS, which one sweep
// workgroup fills), and in at most 16 KB; larger intervals stage in a global
// per-vertex shadow array.  Returns the LDS capacity (0 = global shadow) and the
// effective interval.
constexpr size_t kLdsStage = 16 * 1024;
constexpr size_t kStaticLds = 14 * 1024;  // bound on the sweep kernels' static LDS
void staging(const dg_graph* g, uint32_t d, size_t elem, uint32_t res, uint32_t& cap, uint32_t& d_eff,
             bool& shadow) {
  d_eff = std::min(d, g->max_block_v);
  if (d_eff < 1) d_eff = 1;
  const size_t need = ((size_t)d_eff + kTileV) * (elem + 4);
  const size_t room = std::min(kLdsStage, kLdsBudget - kStaticLds - (size_t)res * elem - 16);
  shadow = need > room;
  cap = shadow ? 0u : d_eff + kTileV;
}

// Commits per sweep of a delayed single-query sweep, counted as the kernels
// decide them: a worker commits at the end of the first tile that brings its
// staged count to >= d, of a tile after which the next one would overflow
// its LDS staging (cap, when not staging in the shadow), and of its last tile.
uint32_t commits_per_sweep(const dg_graph* g, uint32_t d, uint32_t cap, bool shadow) {
  uint32_t c = 0;
  const std::vector<uint32_t>& tv = g->tile_v_h;
  const std::vector<uint32_t>& wt = g->work_t_h;
  for (size_t w = 0; w + 1 < wt.size(); ++w) {
    uint32_t staged = 0;
    for (uint32_t t = wt[w]; t < wt[w + 1]; ++t) {
      const uint32_t nv = tv[t + 1] - tv[t];
      const bool more = t + 1 < wt[w + 1];
      const uint32_t nvn = more ? tv[t + 2] - tv[t + 1] : 0u;
      const bool flush = !more || staged + nv >= d || (!shadow && staged + nv + nvn > cap);
      staged += nv;
      if (flush) {
        ++c;
        staged = 0;
      }
    }
  }
  return c;
}

// Commits per sweep of one batch (64 queries) of a delayed batched sweep,
// counted as the kernels decide them: each of a batched worker's kWG / 64
// wavefronts stages the rows it updates (vertices v0 + wv, v0 + wv + kWG / 64,
// ... of each batched tile; wavefront 0 alone the row of a single-vertex
// tile) and
// commits them once ceil(d / (kWG / 64)) are staged, and at the end of the
// worker's block.
// Splits the batched tiles tv (first in-edges te0) into P batched workers
// (host side).
void plan_batch_part(const std::vector<uint32_t>& tv, const std::vector<uint32_t>& te0, uint32_t P, BatchPart& bp) {
  bp.P = P;
  build_workers(tv, te0, P, bp.work_t_h);
  bp.max_block_v = 1;
  for (uint32_t w = 0; w < P; ++w) bp.max_block_v = std::max(bp.max_block_v, tv[bp.work_t_h[w + 1]] - tv[bp.work_t_h[w]]);
}

// Default batched workers: per_cu 256-thread workgroups per compute unit,
// rounded down to a multiple of 8, at most one per batched tile.
uint32_t batch_workers(const dg_graph* g, uint32_t per_cu) {
  return batch_workers_for(g->cus, per_cu, (uint32_t)g->btile_v_h.size() - 1);
}

// Mean vertices per batched tile, rounded.
uint32_t batch_tile_vertices(const dg_graph* g) {
  const uint64_t Tb = g->btile_v_h.size() - 1;
  return (uint32_t)(((uint64_t)g->n + Tb / 2) / Tb);
}

uint32_t batch_commits_per_sweep(const dg_graph* g, int which, uint32_t d) {
  constexpr uint32_t waves = kWG / 64;
  const uint64_t per = ((uint64_t)d + waves - 1) / waves;
  const std::vector<uint32_t>& tv = g->btile_v_h;
  const std::vector<uint32_t>& wt = g->bp[which].work_t_h;
  uint64_t c = 0;
  for (size_t w = 0; w + 1 < wt.size(); ++w)
    for (uint32_t wv = 0; wv < waves; ++wv) {
      uint64_t rows = 0;
      for (uint32_t t = wt[w]; t < wt[w + 1]; ++t) {
        const uint32_t nv = tv[t + 1] - tv[t];
        rows += nv == 1 ? (wv == 0 ? 1u : 0u) : (nv > wv ? (nv - wv + waves - 1) / waves : 0u);
      }
      c += (rows + per - 1) / per;
    }
  return (uint32_t)std::min<uint64_t>(c, 0xFFFFFFFFu);
}

}  // namespace host
}  // namespace dg

using dg::host::commits_per_sweep;
using dg::host::staging;

namespace {

void release_all(dg_graph* g) {
  dg::host::drop_captures(g);
  if (g->cap_stream) {
    (void)hipStreamDestroy(g->cap_stream);
    g->cap_stream = nullptr;
  }
  if (g->events) {
    (void)hipEventDestroy(g->ev_start);
    for (auto& e : g->ev_sweep) (void)hipEventDestroy(e);
    g->events = false;
  }
  if (g->host_poll) {
    (void)hipHostFree(g->host_poll);
    g->host_poll = nullptr;
  }
  std::vector<void*> all = g->owned;
  for (void* p : all) dev_free(g, p);
  g->owned.clear();
}

// Pinned host memory, mapped into the device's address space and coherent,
// that kernels write with system-scope stores and the host reads once the
// writing sweep's event has completed.
hipError_t alloc_mapped(void** host, void** dev, size_t bytes) {
  hipError_t e = hipHostMalloc(host, bytes, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return e;
  e = hipHostGetDevicePointer(dev, *host, 0);
  if (e != hipSuccess) {
    (void)hipHostFree(*host);
    *host = nullptr;
  }
  return e;
}

dg_status ensure_workspace(dg_graph* g, uint32_t S, hipStream_t s) {
  if (!g->vals[0]) {
    const size_t bytes = ((size_t)g->n + g->K) * 8;
    for (auto& v : g->vals) {
      v = dev_alloc(g, bytes, s);
      if (!v) return fail(DG_ERR_OUT_OF_MEMORY, "workspace allocation of %zu bytes failed", bytes);
    }
    g->norm = static_cast<double*>(dev_alloc(g, (kNormBlocks + 1) * sizeof(double), s));
    g->part = static_cast<double*>(dev_alloc(g, 3 * (size_t)g->P * sizeof(double), s));
    if (!g->norm || !g->part) return fail(DG_ERR_OUT_OF_MEMORY, "workspace allocation failed");
  }
  if (!g->events) {
    DG_HIP(hipEventCreate(&g->ev_start));
    for (auto& e : g->ev_sweep) DG_HIP(hipEventCreate(&e));
    g->events = true;
  }
  if (g->ws_sweeps < S) {
    dev_free(g, g->resid);
    dev_free(g, g->scale);
    dev_free(g, g->dang);
    dev_free(g, g->count);
    dev_free(g, g->changed);
    if (g->host_poll) (void)hipHostFree(g->host_poll);
    g->host_poll = nullptr;
    g->host_poll_dev = nullptr;
    const size_t k = (size_t)S + 1;
    g->resid = static_cast<double*>(dev_alloc(g, k * sizeof(double), s));
    g->scale = static_cast<double*>(dev_alloc(g, k * sizeof(double), s));
    g->dang = static_cast<double*>(dev_alloc(g, k * sizeof(double), s));
    g->count = static_cast<uint32_t*>(dev_alloc(g, k * sizeof(uint32_t), s));
    g->changed = static_cast<uint32_t*>(dev_alloc(g, k * sizeof(uint32_t), s));
    if (!g->resid || !g->scale || !g->dang || !g->count || !g->changed) {
      g->ws_sweeps = 0;
      return fail(DG_ERR_OUT_OF_MEMORY, "sweep state allocation failed");
    }
    DG_HIP(alloc_mapped(&g->host_poll, &g->host_poll_dev, k * sizeof(double)));
    g->ws_sweeps = S;
  }
  return DG_OK;
}


SweepState state(const dg_graph* g) {
  SweepState st;
  st.resid = g->resid;
  st.hresid = static_cast<double*>(g->host_poll_dev);
  st.hchanged = static_cast<uint32_t*>(g->host_poll_dev);
  st.dang = g->dang;
  st.count = g->count;
  st.changed = g->changed;
  st.part = g->part;
  return st;
}

// local: whether the caller supports DG_DELAYED_LOCAL (single-query sweeps).
dg_status check_mode(dg_mode mode, uint32_t d, bool local = false) {
  if (mode == DG_DELAYED_LOCAL && !local)
    return fail(DG_ERR_INVALID_ARGUMENT, "DG_DELAYED_LOCAL is supported by dg_pagerank and dg_sssp only");
  if (mode != DG_SYNC && mode != DG_ASYNC && mode != DG_DELAYED && mode != DG_DELAYED_LOCAL)
    return fail(DG_ERR_INVALID_ARGUMENT, "mode %d is not DG_SYNC, DG_ASYNC, DG_DELAYED or DG_DELAYED_LOCAL",
                (int)mode);
  if ((mode == DG_DELAYED || mode == DG_DELAYED_LOCAL) && d == 0)
    return fail(DG_ERR_INVALID_ARGUMENT, "delayed mode needs a commit interval d >= 1");
  return DG_OK;
}

// Resident-table entries a sweep reads from LDS: the graph's R leading
// compact-region slots, as many as kResBytes holds at this element size.
uint32_t resident(const dg_graph* g, size_t elem) {
  return std::min(std::min<uint32_t>(g->R, kResBytes / (uint32_t)elem), g->res_limit);
}

// Fields of dg_stats that describe the partition and the commits.
void fill_shape(const dg_graph* g, bool delayed, uint32_t d_eff, uint32_t cap, bool shadow, dg_stats* st) {
  st->workers = g->P;
  st->tile_vertices = g->T ? (uint32_t)(((uint64_t)g->n + g->T / 2) / g->T) : 0u;
  st->commits = delayed ? commits_per_sweep(g, d_eff, cap, shadow) : 0u;
  st->commit_interval = st->commits ? (uint32_t)(((uint64_t)g->n + st->commits / 2) / st->commits) : 0u;
}

// err_bound of dg_pagerank / dg_ppr: ||T(y) - y||_1 / (1 - damping) for the
// float64 scores y (device, vertex order, sum 1) and the map T of global
// PageRank (psrc = kInf) or of personalised PageRank with restart vertex
// psrc, by one synchronous float64 sweep in the
// graph's workspace (its three value arrays; y may be one of them, and is
// read before any is written).  Synchronises the stream.
dg_status certify(dg_graph* g, const double* y, double damping, uint32_t psrc, const SweepState& sst, hipStream_t s,
                  double& bound) {
  double* x = static_cast<double*>(g->vals[0]);
  double* c0 = static_cast<double*>(y == g->vals[1] ? g->vals[2] : g->vals[1]);
  double* c1 = static_cast<double*>(c0 == g->vals[1] ? g->vals[2] : g->vals[1]);
  DG_HIP(launch_bound_setup(y, x, c0, g->out_deg, g->cpos, g->n, sst, g->norm, s));
  PrArgs a;
  std::memset(&a, 0, sizeof a);
  a.g = topo(g);
  a.st = sst;
  a.st.hresid = nullptr;
  a.st.hchanged = nullptr;
  a.x = x;
  a.cin = c0;
  a.cout = c1;
  a.alpha = damping;
  a.tol = 0.0;
  a.k = 0;
  a.res = resident(g, sizeof(double));
  a.psrc = psrc;
  DG_HIP(launch_pr_sweep(kSync, true, a, s));
  double r = 0.0;
  DG_HIP(hipMemcpyAsync(&r, sst.resid + 1, sizeof r, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  bound = r / (1.0 - damping);
  return DG_OK;
}

// Bytes that identify a call shape for captured launches: every value the
// call's launch(k, stream) reads besides k and the stream.
using CaptureKey = std::vector<unsigned char>;

template <typename T>
void key_add(CaptureKey& key, const T& v) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
  key.insert(key.end(), p, p + sizeof(T));
}

}  // namespace

namespace dg {
namespace host {

void drop_captures(dg_graph* g) {
  for (hipGraphExec_t& e : g->cap_exec)
    if (e) (void)hipGraphExecDestroy(e);
  g->cap_exec.clear();
  g->cap_key.clear();
}

}  // namespace host
}  // namespace dg

namespace {

using dg::host::drop_captures;
using dg::host::kMaxCaptureChunk;
using dg::host::kMaxCapturedChunks;

// Records sweeps k0 .. k1-1, as launch(k, stream) issues them, into a HIP
// graph on the graph's capture stream and instantiates it.
template <typename Launch>
dg_status record_chunk(dg_graph* g, uint32_t k0, uint32_t k1, Launch& launch, hipGraphExec_t* out) {
  if (!g->cap_stream) DG_HIP(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
  DG_HIP(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeRelaxed));
  hipError_t le = hipSuccess;
  for (uint32_t k = k0; k < k1 && le == hipSuccess; ++k) le = launch(k, g->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(g->cap_stream, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "recording sweeps %u..%u failed: %s", k0, k1 - 1,
                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  const hipError_t ie = hipGraphInstantiateWithFlags(out, graph, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "instantiating sweeps %u..%u failed: %s", k0, k1 - 1, hipGetErrorString(ie));
  }
  return DG_OK;
}

// Waits for the event after recorded chunk j (sweeps k0..k1-1).  A wait
// longer than 20 s prints one line naming the chunk to stderr, then goes on
// waiting: a chunk runs at most 64 sweeps, so this only shows on a stalled
// device or runtime.
dg_status wait_chunk(hipEvent_t e, uint32_t k0, uint32_t k1) {
  const auto t0 = std::chrono::steady_clock::now();
  bool warned = false;
  for (;;) {
    const hipError_t q = hipEventQuery(e);
    if (q == hipSuccess) return DG_OK;
    if (q != hipErrorNotReady) {
      (void)hipGetLastError();
      return fail(DG_ERR_DEVICE, "waiting for recorded sweeps %u..%u failed: %s", k0, k1 - 1, hipGetErrorString(q));
    }
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!warned && el > 20.0) {
      std::fprintf(stderr, "dg: recorded sweeps %u..%u not complete after %.0f s\n", k0, k1 - 1, el);
      std::fflush(stderr);
      warned = true;
    }
    if (el > 1e-3) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

// Convergence loop shared by every entry point.  launch(k, stream) enqueues
// sweep k, which writes the E stopping values of its row k+1 to the device
// state and, with system-scope stores, to the same row (`row` bytes) of the
// mapped host buffer `host`; rows are zeroed here before their sweep is
// enqueued, so a value a sweep does not write reads as 0, as on the device.
// done(row, k) tells whether sweep k met the stopping rule; it is called for
// k = 0, 1, ... in order until it says yes.
//
// Launched one by one (the default), the host waits for each sweep's event in
// turn and keeps up to `lookahead` sweeps queued beyond it, enough to cover
// its own reaction time at the measured sweep time, so the device does not
// wait for the host and at most that many sweeps are queued after the
// converging one (each exits at once on the device's own check).
//
// With captured launches (g->capture > 0 and a key), sweeps go in chunks of
// g->capture: chunk j is recorded once per call shape, on first use, and
// replayed with one hipGraphLaunch; two chunks are queued while the host
// reads the rows of the older one.  The replayed kernels are the ones the
// eager path launches, with the same arguments, so results do not change.
template <typename Launch, typename Done>
dg_status drive(dg_graph* g, uint32_t max_sweeps, hipStream_t s, size_t row, unsigned char* host, Launch launch,
                Done done, uint32_t& sweeps, double& seconds, bool& converged, const CaptureKey* key = nullptr) {
  static_assert(kMaxLookahead + 1 < kEventRing, "a queued sweep's event slot must not be reused before it is read");
  converged = false;
  sweeps = 0;
  dg_status st = DG_OK;
  int found = -1;
  uint32_t last_event = 0;  // event slot of the last sweep run (or of its chunk)
  DG_HIP(hipEventRecord(g->ev_start, s));
  if (key && g->capture) {
    const uint32_t C = g->capture;
    if (g->cap_key != *key) {
      drop_captures(g);
      g->cap_key = *key;
    }
    const uint32_t nchunks = (uint32_t)(((uint64_t)max_sweeps + C - 1) / C);
    uint32_t launched = 0;
    auto enqueue = [&]() -> dg_status {
      const uint32_t j = launched;
      const uint32_t k0 = j * C, k1 = std::min(k0 + C, max_sweeps);
      std::memset(host + (size_t)(k0 + 1) * row, 0, (size_t)(k1 - k0) * row);
      if (j < kMaxCapturedChunks) {
        if (g->cap_exec.size() <= j) g->cap_exec.resize(j + 1, nullptr);
        if (!g->cap_exec[j]) {
          const dg_status rs = record_chunk(g, k0, k1, launch, &g->cap_exec[j]);
          if (rs != DG_OK) return rs;
        }
        DG_HIP(hipGraphLaunch(g->cap_exec[j], s));
      } else {
        for (uint32_t k = k0; k < k1; ++k) {
          const hipError_t e = launch(k, s);
          if (e != hipSuccess) return fail(DG_ERR_DEVICE, "sweep launch failed: %s", hipGetErrorString(e));
        }
      }
      DG_HIP(hipEventRecord(g->ev_sweep[j % kEventRing], s));
      ++launched;
      return DG_OK;
    };
    while (launched < nchunks && launched < 2)
      if ((st = enqueue()) != DG_OK) return st;
    for (uint32_t j = 0; j < launched && found < 0; ++j) {
      const uint32_t k1 = std::min((j + 1) * C, max_sweeps);
      if ((st = wait_chunk(g->ev_sweep[j % kEventRing], j * C, k1)) != DG_OK) return st;
      last_event = j % kEventRing;
      for (uint32_t k = j * C; k < k1; ++k)
        if (done(host + (size_t)(k + 1) * row, k)) {
          found = (int)k;
          break;
        }
      if (found < 0 && launched < nchunks)
        if ((st = enqueue()) != DG_OK) return st;
    }
  } else {
    uint32_t look = std::max(1u, std::min(g->lookahead, kMaxLookahead));
    uint32_t next = 0;  // next sweep to enqueue
    auto enqueue = [&]() -> dg_status {
      std::memset(host + (size_t)(next + 1) * row, 0, row);
      const hipError_t e = launch(next, s);
      if (e != hipSuccess) return fail(DG_ERR_DEVICE, "sweep launch failed: %s", hipGetErrorString(e));
      DG_HIP(hipEventRecord(g->ev_sweep[next % kEventRing], s));
      ++next;
      return DG_OK;
    };
    while (next < max_sweeps && next < 1 + look)
      if ((st = enqueue()) != DG_OK) return st;
    for (uint32_t k = 0; k < next; ++k) {
      DG_HIP(hipEventSynchronize(g->ev_sweep[k % kEventRing]));
      last_event = k % kEventRing;
      if (k == 0) {
        // The first sweep's time (from the stream reaching it) sets how far
        // ahead to queue, here and in the graph's next call.
        float ms = 0.f;
        DG_HIP(hipEventElapsedTime(&ms, g->ev_start, g->ev_sweep[0]));
        const double us = std::max(1.0, (double)ms * 1e3);
        look = (uint32_t)std::min<double>(kMaxLookahead, std::max(2.0, std::ceil(kHostReactUs / us) + 1.0));
        g->lookahead = look;
      }
      if (done(host + (size_t)(k + 1) * row, k)) {
        found = (int)k;
        break;
      }
      while (next < max_sweeps && next < k + 2 + look)
        if ((st = enqueue()) != DG_OK) return st;
    }
  }
  DG_HIP(hipStreamSynchronize(s));
  const uint32_t last = found >= 0 ? (uint32_t)found : max_sweeps - 1;
  converged = found >= 0;
  sweeps = last + 1;
  // Time to the event after the converging sweep (captured: after its chunk,
  // whose later sweeps exit at once).
  float ms = 0.f;
  DG_HIP(hipEventElapsedTime(&ms, g->ev_start, g->ev_sweep[last_event]));
  seconds = ms * 1e-3;
  return DG_OK;
}

// Pinned host buffer for the batched entry points' state polls.
struct PinnedBuf {
  void* p = nullptr;
  void* dev = nullptr;  // device address of p
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
};

// Device allocations of one batched call, released when the call returns.
struct CallAllocs {
  dg_graph* g;
  std::vector<void*> ptrs;
  explicit CallAllocs(dg_graph* gg) : g(gg) {}
  void* get(size_t bytes, hipStream_t s) {
    void* p = dev_alloc(g, bytes, s);
    if (p) ptrs.push_back(p);
    return p;
  }
  ~CallAllocs() {
    if (!ptrs.empty()) (void)hipDeviceSynchronize();
    for (void* p : ptrs) dev_free(g, p);
  }
};

}  // namespace

namespace {

// Tuning results cached in-process by (graph content, algorithm, dtype,
// tolerance, source).
struct TuneEntry {
  uint64_t hash;
  int algo, dtype;
  double tol;
  uint32_t src;
  dg_tuning t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune_cache;

bool tune_find(uint64_t hash, int algo, int dtype, double tol, uint32_t src, dg_tuning& out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& e : g_tune_cache)
    if (e.hash == hash && e.algo == algo && e.dtype == dtype && e.tol == tol && e.src == src) {
      out = e.t;
      return true;
    }
  return false;
}

void tune_put(const TuneEntry& n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& e : g_tune_cache)
    if (e.hash == n.hash && e.algo == n.algo && e.dtype == n.dtype && e.tol == n.tol && e.src == n.src) {
      e = n;
      return;
    }
  g_tune_cache.push_back(n);
}

uint32_t default_workers(const dg_graph* g, uint32_t per_cu) {
  uint32_t P = std::max(1u, std::min(g->cus * per_cu, g->T));
  if (P > 8) P &= ~7u;
  return P;
}

}  // namespace

extern "C" {

const char* dg_version(void) { return "dg 0.1 (gfx950)"; }

const char* dg_last_error(void) { return g_last_error.c_str(); }

const char* dg_status_str(dg_status s) {
  switch (s) {
    case DG_OK: return "DG_OK";
    case DG_ERR_INVALID_ARGUMENT: return "DG_ERR_INVALID_ARGUMENT";
    case DG_ERR_OUT_OF_MEMORY: return "DG_ERR_OUT_OF_MEMORY";
    case DG_ERR_DEVICE: return "DG_ERR_DEVICE";
    case DG_ERR_NOT_CONVERGED: return "DG_ERR_NOT_CONVERGED";
    case DG_ERR_UNSUPPORTED: return "DG_ERR_UNSUPPORTED";
  }
  return "DG_ERR_UNKNOWN";
}

dg_status dg_set_allocator(dg_alloc_fn alloc, dg_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(DG_ERR_INVALID_ARGUMENT, "alloc and free hooks must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_ctx = ctx;
  return DG_OK;
}

dg_status dg_graph_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                          const uint32_t* w, const dg_graph_opts* opts, void* hip_stream, dg_graph** out) {
  g_last_error.clear();
  if (!opts || opts->arrays_on_device == 0)
    return dg::host::graph_create(n, m, layout, ptr, idx, w, opts, nullptr, hip_stream, out);
  if (opts->arrays_on_device != 1)
    return fail(DG_ERR_INVALID_ARGUMENT, "arrays_on_device = %u, expected 0 or 1", opts->arrays_on_device);
  // Device arrays: checked for what can be checked without reading them,
  // then copied to the host, where the layout is built as for host input.
  if (!out) return fail(DG_ERR_INVALID_ARGUMENT, "out is NULL");
  if (n == 0 || n > 0xFFFFFFFEu) return fail(DG_ERR_INVALID_ARGUMENT, "n = %u outside [1, 2^32-2]", n);
  if (m >= (uint64_t)0xFFFFFFFFu - 2 * kEdgePad)
    return fail(DG_ERR_INVALID_ARGUMENT, "m = %llu too large", (unsigned long long)m);
  if (!ptr) return fail(DG_ERR_INVALID_ARGUMENT, "ptr is NULL");
  if (m > 0 && !idx) return fail(DG_ERR_INVALID_ARGUMENT, "idx is NULL");
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "no usable HIP device: %s", hipGetErrorString(he));
  }
  struct Arr {
    const void* p;
    size_t bytes;
    const char* name;
  } arrs[] = {{ptr, ((size_t)n + 1) * sizeof(uint64_t), "ptr"},
              {idx, (size_t)m * sizeof(uint32_t), "idx"},
              {w, (size_t)m * sizeof(uint32_t), "w"}};
  for (const Arr& a : arrs) {
    if (!a.p || a.bytes == 0) continue;
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof at);
    he = hipPointerGetAttributes(&at, a.p);
    if (he != hipSuccess || (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)) {
      (void)hipGetLastError();
      return fail(DG_ERR_INVALID_ARGUMENT, "%s is not device memory (arrays_on_device = 1)", a.name);
    }
  }
  std::vector<uint64_t> hptr;
  std::vector<uint32_t> hidx, hw;
  try {
    hptr.resize((size_t)n + 1);
    hidx.resize((size_t)m);
    if (w) hw.resize(m ? (size_t)m : 1u);  // non-empty, so that a weighted graph without edges keeps w != NULL
  } catch (const std::bad_alloc&) {
    return fail(DG_ERR_OUT_OF_MEMORY, "host copy of the device arrays failed");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  DG_HIP(hipMemcpyAsync(hptr.data(), ptr, hptr.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  if (m) DG_HIP(hipMemcpyAsync(hidx.data(), idx, (size_t)m * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  if (w && m) DG_HIP(hipMemcpyAsync(hw.data(), w, (size_t)m * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  dg_graph_opts host_opts = *opts;
  host_opts.arrays_on_device = 0;
  const uint32_t* wp = w ? hw.data() : nullptr;
  return dg::host::graph_create(n, m, layout, hptr.data(), m ? hidx.data() : nullptr, wp, &host_opts, nullptr,
                                hip_stream, out);
}

}  // extern "C"

namespace dg {
namespace host {

dg_status graph_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                       const uint32_t* w, const dg_graph_opts* opts, const std::vector<uint32_t>* seg_v,
                       void* hip_stream, dg_graph** out) {
  if (!out) return fail(DG_ERR_INVALID_ARGUMENT, "out is NULL");
  dg_status st = validate_graph(n, m, layout, ptr, idx);
  if (st != DG_OK) return st;

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  dg_graph* g = new (std::nothrow) dg_graph;
  if (!g) return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g->alloc = g_alloc;
    g->free_fn = g_free;
    g->ctx = g_alloc_ctx;
  }
  g->create_stream = s;
  g->n = n;
  g->m = m;
  g->has_w = (w != nullptr);

  // Device sizes.  Without a device (or on error) nothing below leaks.
  int dev = 0, cus = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int lds = 0;
  if (he == hipSuccess) he = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    delete g;
    return fail(DG_ERR_DEVICE, "no usable HIP device: %s", hipGetErrorString(he));
  }
  g->cus = (uint32_t)cus;
  g->lds_per_block = (size_t)lds;

  // The layout every sweep reads (the same construction dg_plan_create
  // returns without a device).
  const uint32_t per_cu = seg_v ? kSetWorkersPerCU : kWorkersPerCU;
  Layout L;
  if ((st = build_layout(n, m, layout, ptr, idx, w, opts, opts && opts->workers ? opts->workers : g->cus * per_cu, L,
                         seg_v)) != DG_OK) {
    delete g;
    return st;
  }
  g->K = L.K;
  g->R = L.R;
  g->hot_edges = L.hot_edges;
  g->res_edges = L.res_edges;
  g->max_in_deg = L.max_in_deg;
  g->n_dangling = L.n_dangling;
  g->hash = L.hash;
  g->T = L.T();
  g->variant = L.variant;
  g->variant0 = L.variant;
  g->tile_v_h = L.tile_v;
  g->tile_e0_h = L.tile_e0;
  if (!seg_v) g->in_ptr_h = L.in_ptr;
  uint32_t P = plan_workers(L, opts ? opts->workers : 0u, g->cus, per_cu);
  std::vector<uint32_t> work_t;
  if (seg_v) {
    g->G = (uint32_t)seg_v->size() - 1;
    g->seg_v = *seg_v;
    build_workers_seg(L.tile_v, L.tile_e0, *seg_v, std::max(P, g->G), work_t, g->wseg_h);
    P = g->wseg_h.back();
    g->wgraph_h.resize(P);
    for (uint32_t gi = 0; gi < g->G; ++gi)
      for (uint32_t wk = g->wseg_h[gi]; wk < g->wseg_h[gi + 1]; ++wk) g->wgraph_h[wk] = gi;
  } else {
    build_workers(L.tile_v, L.tile_e0, P, work_t);
  }
  g->P = P;
  g->work_t_h = work_t;
  for (uint32_t wk = 0; wk < P; ++wk)
    g->max_block_v = std::max(g->max_block_v, L.tile_v[work_t[wk + 1]] - L.tile_v[work_t[wk]]);
  dg::host::build_batch_tiles(L.tile_v, L.in_ptr, dg::host::kBatchTileE, g->btile_v_h, g->btile_e0_h);
  dg::host::plan_batch_part(g->btile_v_h, g->btile_e0_h, dg::host::batch_workers(g, kBatchSsspWorkersPerCU),
                            g->bp[kBatchSssp]);
  dg::host::plan_batch_part(g->btile_v_h, g->btile_e0_h, dg::host::batch_workers(g, kBatchPprWorkersPerCU),
                            g->bp[kBatchPpr]);

  uint32_t* w8_words = nullptr;
  struct Up {
    uint32_t** dst;
    const std::vector<uint32_t>* src;
  } ups[] = {{&g->in_ptr, &L.in_ptr}, {&g->in_src, &L.in_src}, {&g->in_w, &L.in_w}, {&w8_words, &L.w8pack},
             {&g->out_deg, &L.out_deg}, {&g->cpos, &L.cpos}, {&g->tile_v, &L.tile_v}, {&g->work_t, &work_t},
             {&g->wseg, &g->wseg_h}, {&g->wgraph, &g->wgraph_h}, {&g->btile_v, &g->btile_v_h},
             {&g->bp[kBatchSssp].work_t, &g->bp[kBatchSssp].work_t_h},
             {&g->bp[kBatchPpr].work_t, &g->bp[kBatchPpr].work_t_h}, {&g->segv_d, &g->seg_v}};
  for (auto& u : ups) {
    if (u.src->empty()) continue;
    const size_t bytes = u.src->size() * sizeof(uint32_t);
    *u.dst = static_cast<uint32_t*>(dev_alloc(g, bytes, s));
    if (!*u.dst) {
      release_all(g);
      delete g;
      return fail(DG_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", bytes);
    }
    g->graph_bytes += bytes;
    he = hipMemcpyAsync(*u.dst, u.src->data(), bytes, hipMemcpyHostToDevice, s);
    if (he != hipSuccess) break;
  }
  g->in_w8 = reinterpret_cast<uint8_t*>(w8_words);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    release_all(g);
    delete g;
    return fail(DG_ERR_DEVICE, "graph upload failed: %s", hipGetErrorString(he));
  }
  if (g->G) {
    g->gsweeps = static_cast<uint32_t*>(dev_alloc(g, (size_t)g->G * sizeof(uint32_t), s));
    g->gdang = static_cast<double*>(dev_alloc(g, (size_t)2 * g->G * sizeof(double), s));
    if (!g->gsweeps || !g->gdang) {
      release_all(g);
      delete g;
      return fail(DG_ERR_OUT_OF_MEMORY, "device allocation failed");
    }
    // Dangling mass of each graph at x = 1/n (the union's first iterate).
    g->gdang0.assign(g->G, 0.0);
    for (uint32_t gi = 0; gi < g->G; ++gi) {
      uint32_t nd = 0;
      for (uint32_t v = g->seg_v[gi]; v < g->seg_v[gi + 1]; ++v) nd += L.out_deg[v] == 0;
      g->gdang0[gi] = (double)nd / (double)n;
    }
  }
  *out = g;
  return DG_OK;
}

}  // namespace host
}  // namespace dg

extern "C" {

dg_status dg_graph_destroy(dg_graph* g) {
  if (!g) return DG_OK;
  (void)hipDeviceSynchronize();
  release_all(g);
  delete g;
  return DG_OK;
}

dg_status dg_graph_info_get(const dg_graph* g, dg_graph_info* info) {
  if (!g || !info) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  info->n = g->n;
  info->m = g->m;
  info->workers = g->P;
  info->tiles = g->T;
  info->max_in_degree = g->max_in_deg;
  info->dangling = g->n_dangling;
  info->has_weights = g->has_w ? 1u : 0u;
  info->compute_units = g->cus;
  info->hot_vertices = g->K;
  info->hot_edges = g->hot_edges;
  info->resident_vertices = g->R;
  info->resident_edges = g->res_edges;
  info->weight_bytes = g->in_w8 ? 1u : (g->in_w ? 4u : 0u);
  info->device_bytes = g->graph_bytes;
  info->sweep_variant = g->variant;
  info->batch_tiles = (uint32_t)g->btile_v_h.size() - 1;
  return DG_OK;
}

dg_status dg_graph_partition(const dg_graph* g, uint32_t* out_first_vertex, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out_first_vertex) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::vector<uint32_t> wt(g->P + 1), tv((size_t)g->T + 1);
  DG_HIP(hipMemcpyAsync(wt.data(), g->work_t, wt.size() * 4, hipMemcpyDeviceToHost, s));
  DG_HIP(hipMemcpyAsync(tv.data(), g->tile_v, tv.size() * 4, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  for (uint32_t w = 0; w <= g->P; ++w) out_first_vertex[w] = tv[wt[w]];
  return DG_OK;
}

dg_status dg_access_matrix(dg_graph* g, uint32_t groups, uint64_t* out_counts, dg_access_stats* stats,
                           void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (groups < 1 || groups > 64 || groups > g->P)
    return fail(DG_ERR_INVALID_ARGUMENT, "groups = %u outside [1, min(64, workers = %u)]", groups, g->P);
  if (!out_counts && !stats) return fail(DG_ERR_INVALID_ARGUMENT, "nothing to return");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  CallAllocs al(g);
  uint32_t* vw = static_cast<uint32_t*>(al.get((size_t)g->n * 4, s));
  uint32_t* inv = static_cast<uint32_t*>(al.get((size_t)std::max(g->K, 1u) * 4, s));
  unsigned long long* cnt = static_cast<unsigned long long*>(al.get(((size_t)groups * groups + 1) * 8, s));
  if (!vw || !inv || !cnt) return fail(DG_ERR_OUT_OF_MEMORY, "access matrix workspace allocation failed");
  DG_HIP(hipMemsetAsync(cnt, 0, ((size_t)groups * groups + 1) * 8, s));
  DG_HIP(launch_access_matrix(topo(g), vw, inv, groups, cnt, cnt + (size_t)groups * groups, s));
  std::vector<unsigned long long> h((size_t)groups * groups + 1);
  DG_HIP(hipMemcpyAsync(h.data(), cnt, h.size() * 8, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  uint64_t total = 0, diag = 0;
  std::vector<double> row(groups, 0.0), col(groups, 0.0);
  for (uint32_t r = 0; r < groups; ++r)
    for (uint32_t c = 0; c < groups; ++c) {
      const uint64_t x = h[(size_t)r * groups + c];
      total += x;
      if (r == c) diag += x;
      row[r] += (double)x;
      col[c] += (double)x;
      if (out_counts) out_counts[(size_t)r * groups + c] = x;
    }
  if (stats) {
    stats->reads = total;
    stats->same_worker = h.back();
    stats->diagonal = diag;
    stats->groups = groups;
    stats->workers = g->P;
    stats->self_share = total ? (double)h.back() / (double)total : 0.0;
    stats->diagonal_share = total ? (double)diag / (double)total : 0.0;
    double u = 0.0;
    for (uint32_t r = 0; r < groups; ++r) u += row[r] * col[r];
    stats->uniform_diagonal = total ? u / ((double)total * (double)total) : 0.0;
  }
  return DG_OK;
}

dg_status dg_predict_mode(dg_graph* g, dg_prediction* out, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  dg_access_stats st{};
  const uint32_t groups = std::min(8u, g->P);
  const dg_status r = dg_access_matrix(g, groups, nullptr, &st, hip_stream);
  if (r != DG_OK) return r;
  dg_prediction p{};
  p.groups = groups;
  p.diagonal_share = st.diagonal_share;
  p.uniform_diagonal = st.uniform_diagonal;
  p.lift = st.uniform_diagonal > 0.0 ? st.diagonal_share / st.uniform_diagonal : 1.0;
  p.self_share = st.self_share;
  if (p.lift >= DG_PREDICT_CLUSTER_LIFT) {
    p.mode = DG_ASYNC;
    p.d = 0;
  } else {
    p.mode = DG_DELAYED;
    p.d = 64;
  }
  *out = p;
  return DG_OK;
}

dg_status dg_pagerank(dg_graph* g, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                      uint32_t max_sweeps, double* out_scores, int out_on_device, dg_stats* stats,
                      void* hip_stream) {
  return dg::host::pr_run(g, kInf, damping, tol, mode, d, dtype, max_sweeps, out_scores, out_on_device, stats,
                          hip_stream);
}

dg_status dg_error_bound(dg_graph* g, double damping, uint32_t restart, const double* scores, int scores_on_device,
                         double* out_bound, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (g->G) return fail(DG_ERR_UNSUPPORTED, "not supported on the union graph of a set");
  if (!(damping >= 0.0 && damping < 1.0)) return fail(DG_ERR_INVALID_ARGUMENT, "damping must be in [0, 1)");
  if (restart != DG_NO_RESTART && restart >= g->n)
    return fail(DG_ERR_INVALID_ARGUMENT, "restart vertex %u >= n = %u", restart, g->n);
  if (!scores || !out_bound) return fail(DG_ERR_INVALID_ARGUMENT, "NULL scores or out_bound");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  dg_status st = ensure_workspace(g, 1, s);
  if (st != DG_OK) return st;
  const double* y = scores;
  if (!scores_on_device) {
    DG_HIP(hipMemcpyAsync(g->vals[2], scores, (size_t)g->n * 8, hipMemcpyHostToDevice, s));
    y = static_cast<const double*>(g->vals[2]);
  }
  SweepState sst = state(g);
  sst.scale = g->scale;
  double bound = 0.0;
  if ((st = certify(g, y, damping, restart, sst, s, bound)) != DG_OK) return st;
  *out_bound = bound;
  return DG_OK;
}

dg_status dg_ppr(dg_graph* g, uint32_t src, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                 uint32_t max_sweeps, double* out_scores, int out_on_device, dg_stats* stats, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (g->G) return fail(DG_ERR_UNSUPPORTED, "personalised PageRank is not supported on the union graph of a set");
  if (src >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "restart vertex %u >= n = %u", src, g->n);
  return dg::host::pr_run(g, src, damping, tol, mode, d, dtype, max_sweeps, out_scores, out_on_device, stats,
                          hip_stream);
}

}  // extern "C"

namespace dg {
namespace host {

dg_status pr_run(dg_graph* g, uint32_t psrc, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                 uint32_t max_sweeps, double* out_scores, int out_on_device, dg_stats* stats, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!(damping >= 0.0 && damping < 1.0)) return fail(DG_ERR_INVALID_ARGUMENT, "damping must be in [0, 1)");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and >= 0");
  dg_status st = check_mode(mode, d, true);
  if (st != DG_OK) return st;
  if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "unknown dtype %d", (int)dtype);
  if (max_sweeps == 0 || max_sweeps > kMaxSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps must be in [1, %u]", kMaxSweeps);
  if (!out_scores) return fail(DG_ERR_INVALID_ARGUMENT, "out_scores is NULL");

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_workspace(g, max_sweeps, s)) != DG_OK) return st;
  const bool f64 = dtype == DG_F64;
  const size_t elem = f64 ? 8 : 4;
  uint32_t cap = 0, d_eff = 0;
  bool use_shadow = false;
  const bool delayed = mode == DG_DELAYED || mode == DG_DELAYED_LOCAL;
  const uint32_t nres = resident(g, elem);
  if (delayed) staging(g, d, elem, nres, cap, d_eff, use_shadow);
  if (mode == DG_DELAYED_LOCAL) {
    use_shadow = true;  // local reads look the worker's staged values up by vertex
    cap = 0;
  }
  void* x = g->vals[0];
  void* c0 = g->vals[1];
  void* c1 = mode == DG_SYNC ? g->vals[2] : nullptr;
  SweepState sst = state(g);
  double d0 = (double)g->n_dangling / (double)g->n;  // dangling mass of x = 1/n
  if (psrc != kInf) {
    // dangling mass of the one-hot start: 1 if the restart vertex is dangling
    uint32_t deg = 0;
    DG_HIP(hipMemcpyAsync(&deg, g->out_deg + psrc, sizeof deg, hipMemcpyDeviceToHost, s));
    DG_HIP(hipStreamSynchronize(s));
    d0 = deg ? 0.0 : 1.0;
    sst.scale = g->scale;
  }
  DG_HIP(launch_pr_init(f64, x, c0, c1, g->out_deg, g->cpos, g->n, sst, max_sweeps, d0, psrc, s));
  if (mode == DG_DELAYED_LOCAL) DG_HIP(launch_by_vertex(f64, c0, g->cpos, g->n, g->vals[2], s));

  PrArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: the bytes identify a captured call shape
  a.g = topo(g);
  a.st = sst;
  a.x = x;
  a.shadow = use_shadow ? g->vals[2] : nullptr;
  a.alpha = damping;
  a.tol = tol;
  a.d = d_eff;
  a.cap = cap;
  a.res = nres;
  a.wseg = g->G ? g->wseg : nullptr;
  a.wgraph = g->wgraph;
  a.G = g->G;
  a.gsweeps = g->gsweeps;
  a.voff = g->segv_d;
  a.gdang = g->gdang;
  a.psrc = psrc;
  if (g->G) {
    DG_HIP(launch_fill_u32(g->gsweeps, g->G, 0u, s));
    DG_HIP(hipMemcpyAsync(g->gdang, g->gdang0.data(), (size_t)g->G * sizeof(double), hipMemcpyHostToDevice, s));
  }
  CaptureKey key;
  key_add(key, 1);
  key_add(key, (int)mode);
  key_add(key, f64);
  key_add(key, max_sweeps);
  key_add(key, c0);
  key_add(key, c1);
  key_add(key, a);
  auto launch = [&](uint32_t k, hipStream_t q) {
    if (mode == DG_SYNC) {
      a.cin = (k & 1) ? c1 : c0;
      a.cout = (k & 1) ? c0 : c1;
    } else {
      a.cin = c0;
      a.cout = c0;
    }
    a.k = k;
    return launch_pr_sweep((int)mode, f64, a, q);
  };
  auto done = [&](const unsigned char* p, uint32_t) {
    double r;
    std::memcpy(&r, p, sizeof r);
    return !(r >= tol);
  };
  uint32_t sweeps = 0;
  double secs = 0.0, resid = 0.0;
  bool conv = false;
  unsigned char* poll = static_cast<unsigned char*>(g->host_poll);
  if ((st = drive(g, max_sweeps, s, sizeof(double), poll, launch, done, sweeps, secs, conv, &key)) != DG_OK)
    return st;
  std::memcpy(&resid, poll + (size_t)sweeps * sizeof(double), sizeof(double));
  resid = std::fabs(resid);  // negative: a float32 personalised sweep stopped at its rounding floor

  double* dst = out_on_device ? out_scores : static_cast<double*>(g->vals[1]);
  if (!out_on_device && mode != DG_SYNC) dst = static_cast<double*>(g->vals[2]);
  DG_HIP(launch_normalize(f64, x, g->n, dst, g->norm, s));
  if (!out_on_device) DG_HIP(hipMemcpyAsync(out_scores, dst, (size_t)g->n * 8, hipMemcpyDeviceToHost, s));
  double bound = 0.0;
  if (stats && (stats->request & DG_STATS_ERR_BOUND)) {
    if ((st = certify(g, dst, damping, psrc, sst, s, bound)) != DG_OK) return st;
  }
  DG_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->sweeps = sweeps;
    fill_shape(g, delayed, d_eff, cap, use_shadow, stats);
    stats->residual = resid;
    stats->seconds = secs;
    stats->edges_traversed = g->m * (uint64_t)sweeps;
    stats->err_bound = bound;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "no convergence within %u sweeps (last change %g)", max_sweeps, resid);
  return DG_OK;
}

}  // namespace host
}  // namespace dg

extern "C" {

dg_status dg_sssp(dg_graph* g, uint32_t src, dg_mode mode, uint32_t d, uint32_t max_sweeps, uint32_t* out_dist,
                  int out_on_device, dg_stats* stats, void* hip_stream) {
  return dg::host::sssp_run(g, src, nullptr, 0, mode, d, max_sweeps, out_dist, out_on_device, stats, hip_stream);
}

}  // extern "C"

namespace dg {
namespace host {

dg_status sssp_run(dg_graph* g, uint32_t src, const uint32_t* more_src, uint32_t n_more, dg_mode mode, uint32_t d,
                   uint32_t max_sweeps, uint32_t* out_dist, int out_on_device, dg_stats* stats, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "graph was created without weights");
  if (src >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "source %u >= n = %u", src, g->n);
  dg_status st = check_mode(mode, d, true);
  if (st != DG_OK) return st;
  if (max_sweeps == 0 || max_sweeps > kMaxSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps must be in [1, %u]", kMaxSweeps);
  if (!out_dist) return fail(DG_ERR_INVALID_ARGUMENT, "out_dist is NULL");

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_workspace(g, max_sweeps, s)) != DG_OK) return st;
  uint32_t cap = 0, d_eff = 0;
  bool use_shadow = false;
  const bool delayed = mode == DG_DELAYED || mode == DG_DELAYED_LOCAL;
  const uint32_t nres = resident(g, sizeof(uint32_t));
  if (delayed) staging(g, d, sizeof(uint32_t), nres, cap, d_eff, use_shadow);
  if (mode == DG_DELAYED_LOCAL) {
    use_shadow = true;  // local reads look the worker's staged values up by vertex
    cap = 0;
  }
  uint32_t* b0 = static_cast<uint32_t*>(g->vals[0]);
  uint32_t* b1 = mode == DG_SYNC ? static_cast<uint32_t*>(g->vals[1]) : nullptr;
  SweepState sst = state(g);
  DG_HIP(launch_bf_init(b0, b1, g->cpos, g->n, src, sst, max_sweeps, s));
  if (n_more) DG_HIP(launch_bf_more_sources(b0, b1, g->cpos, more_src, n_more, s));
  if (mode == DG_DELAYED_LOCAL)
    DG_HIP(launch_bf_gather(b0, g->cpos, g->n, static_cast<uint32_t*>(g->vals[2]), s));

  BfArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: the bytes identify a captured call shape
  a.g = topo(g);
  a.st = sst;
  a.d = d_eff;
  a.cap = cap;
  a.res = nres;
  a.shadow = use_shadow ? static_cast<uint32_t*>(g->vals[2]) : nullptr;
  a.wseg = g->G ? g->wseg : nullptr;
  a.wgraph = g->wgraph;
  a.G = g->G;
  a.gsweeps = g->gsweeps;
  if (g->G) DG_HIP(launch_fill_u32(g->gsweeps, g->G, 0u, s));
  CaptureKey key;
  key_add(key, 2);
  key_add(key, (int)mode);
  key_add(key, max_sweeps);
  key_add(key, b0);
  key_add(key, b1);
  key_add(key, a);
  auto launch = [&](uint32_t k, hipStream_t q) {
    if (mode == DG_SYNC) {
      a.din = (k & 1) ? b1 : b0;
      a.dout = (k & 1) ? b0 : b1;
    } else {
      a.din = b0;
      a.dout = b0;
    }
    a.k = k;
    return launch_bf_sweep((int)mode, a, q);
  };
  auto done = [&](const unsigned char* p, uint32_t) {
    uint32_t c;
    std::memcpy(&c, p, sizeof c);
    return c == 0;
  };
  uint32_t sweeps = 0;
  double secs = 0.0;
  bool conv = false;
  unsigned char* poll = static_cast<unsigned char*>(g->host_poll);
  if ((st = drive(g, max_sweeps, s, sizeof(uint32_t), poll, launch, done, sweeps, secs, conv, &key)) != DG_OK)
    return st;
  // The last executed sweep k = sweeps-1 wrote buffer (k+1) % 2 in sync mode.
  const uint32_t* res = (mode == DG_SYNC && (sweeps & 1)) ? b1 : b0;
  uint32_t* dst = out_on_device ? out_dist : static_cast<uint32_t*>(g->vals[2]);
  DG_HIP(launch_bf_gather(res, g->cpos, g->n, dst, s));
  if (!out_on_device)
    DG_HIP(hipMemcpyAsync(out_dist, dst, (size_t)g->n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->sweeps = sweeps;
    fill_shape(g, delayed, d_eff, cap, use_shadow, stats);
    stats->residual = 0.0;
    stats->seconds = secs;
    stats->edges_traversed = g->m * (uint64_t)sweeps;
    stats->err_bound = 0.0;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "no convergence within %u sweeps", max_sweeps);
  return DG_OK;
}

}  // namespace host
}  // namespace dg

extern "C" {

// ----------------------------------------------------------- batched --

namespace {
constexpr uint32_t kBatchQ = 64;
constexpr uint32_t kMaxBatchSweeps = 100000;

dg_status check_batch(dg_graph* g, const uint32_t* sources, uint32_t k, dg_mode mode, uint32_t d,
                      uint32_t max_sweeps, const void* out) {
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!sources || k == 0) return fail(DG_ERR_INVALID_ARGUMENT, "need k >= 1 sources");
  for (uint32_t i = 0; i < k; ++i)
    if (sources[i] >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "sources[%u] = %u >= n", i, sources[i]);
  dg_status st = check_mode(mode, d);
  if (st != DG_OK) return st;
  if (max_sweeps == 0 || max_sweeps > kMaxBatchSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps must be in [1, %u] for batched queries", kMaxBatchSweeps);
  if (!out) return fail(DG_ERR_INVALID_ARGUMENT, "output is NULL");
  const uint64_t NB = (k + kBatchQ - 1) / kBatchQ;
  if ((uint64_t)(g->n + g->K) * kBatchQ * 4u * NB >= (1ull << 40))
    return fail(DG_ERR_UNSUPPORTED, "batched values would exceed 1 TiB");
  return DG_OK;
}
}  // namespace

dg_status dg_sssp_batch(dg_graph* g, const uint32_t* sources, uint32_t k, dg_mode mode, uint32_t d,
                        uint32_t max_sweeps, uint32_t* out_dist, int out_on_device, dg_stats* stats,
                        void* hip_stream) {
  g_last_error.clear();
  dg_status st = check_batch(g, sources, k, mode, d, max_sweeps, out_dist);
  if (st != DG_OK) return st;
  if (!g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "graph was created without weights");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_workspace(g, 1, s)) != DG_OK) return st;
  const uint32_t NB = (k + kBatchQ - 1) / kBatchQ;
  const size_t vals = (size_t)NB * (g->n + g->K) * kBatchQ;
  CallAllocs al(g);
  uint32_t* srcd = static_cast<uint32_t*>(al.get((size_t)k * 4, s));
  uint32_t* b0 = static_cast<uint32_t*>(al.get(vals * 4, s));
  uint32_t* b1 = mode == DG_SYNC ? static_cast<uint32_t*>(al.get(vals * 4, s)) : nullptr;
  // Delayed commits stage in LDS up to kLdsStageMaxD, beyond in a shadow.
  const uint32_t d_eff = mode == DG_DELAYED ? std::max(1u, std::min(d, g->bp[kBatchSssp].max_block_v)) : 0u;
  const bool need_sh = mode == DG_DELAYED && d_eff > kLdsStageMaxD;
  uint32_t* sh = need_sh ? static_cast<uint32_t*>(al.get((size_t)NB * g->n * kBatchQ * 4, s)) : nullptr;
  uint32_t* changed = static_cast<uint32_t*>(al.get(((size_t)max_sweeps + 1) * NB * 4, s));
  uint32_t* outd = out_on_device ? out_dist : static_cast<uint32_t*>(al.get((size_t)k * g->n * 4, s));
  if (!srcd || !b0 || (mode == DG_SYNC && !b1) || (need_sh && !sh) || !changed || !outd)
    return fail(DG_ERR_OUT_OF_MEMORY, "batched SSSP workspace allocation failed");
  PinnedBuf poll;
  DG_HIP(alloc_mapped(&poll.p, &poll.dev, ((size_t)max_sweeps + 1) * NB * 4));
  DG_HIP(hipMemcpyAsync(srcd, sources, (size_t)k * 4, hipMemcpyHostToDevice, s));
  DG_HIP(launch_fill_u32(changed, ((size_t)max_sweeps + 1) * NB, 0u, s));
  DG_HIP(launch_fill_u32(changed, NB, 1u, s));
  DG_HIP(launch_mbf_init(b0, b1, g->cpos, srcd, k, g->n, g->K, NB, s));
  MbfArgs a;
  std::memset(&a, 0, sizeof a);  // call mode: no serving fields
  a.g = topo_batch(g, kBatchSssp);
  a.changed = changed;
  a.hchanged = static_cast<uint32_t*>(poll.dev);
  a.shadow = sh;
  a.d = d_eff;
  a.NB = NB;
  CaptureKey key;
  key_add(key, 3);
  key_add(key, (int)mode);
  key_add(key, max_sweeps);
  key_add(key, b0);
  key_add(key, b1);
  key_add(key, a);
  auto launch = [&](uint32_t kk, hipStream_t q) {
    if (mode == DG_SYNC) {
      a.din = (kk & 1) ? b1 : b0;
      a.dout = (kk & 1) ? b0 : b1;
    } else {
      a.din = b0;
      a.dout = b0;
    }
    a.k = kk;
    return launch_mbf_sweep((int)mode, a, q);
  };
  std::vector<uint32_t> bsweeps(NB, 0);
  auto done = [&](const unsigned char* p, uint32_t kk) {
    bool all = true;
    for (uint32_t b = 0; b < NB; ++b) {
      uint32_t c;
      std::memcpy(&c, p + 4 * b, 4);
      if (c == 0 && bsweeps[b] == 0) bsweeps[b] = kk + 1;
      all = all && c == 0;
    }
    return all;
  };
  uint32_t sweeps = 0;
  double secs = 0.0;
  bool conv = false;
  if ((st = drive(g, max_sweeps, s, (size_t)NB * 4, static_cast<unsigned char*>(poll.p), launch, done, sweeps, secs,
                  conv, &key)) != DG_OK)
    return st;
  // The buffer sweep `sweeps-1` wrote holds every batch's final distances:
  // converged batches skip later sweeps, and sync sweeps alternate buffers.
  const uint32_t* res = (mode == DG_SYNC && (sweeps & 1)) ? b1 : b0;
  if (mode == DG_SYNC) {
    // A batch that converged earlier stopped writing: its last write went to
    // the buffer of its own final sweep.  Copy those rows into `res`.
    for (uint32_t b = 0; b < NB; ++b) {
      const uint32_t sb = bsweeps[b] ? bsweeps[b] : sweeps;
      const uint32_t* own = (sb & 1) ? b1 : b0;
      if (own != res) {
        const size_t off = (size_t)b * (g->n + g->K) * kBatchQ;
        DG_HIP(hipMemcpyAsync(const_cast<uint32_t*>(res) + off, own + off, (size_t)(g->n + g->K) * kBatchQ * 4,
                              hipMemcpyDeviceToDevice, s));
      }
    }
  }
  DG_HIP(launch_mbf_out(res, g->cpos, g->n, g->K, k, NB, outd, s));
  if (!out_on_device) DG_HIP(hipMemcpyAsync(out_dist, outd, (size_t)k * g->n * 4, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  if (stats) {
    uint64_t qe = 0;
    for (uint32_t b = 0; b < NB; ++b) {
      const uint32_t nq = std::min(kBatchQ, k - b * kBatchQ);
      qe += (uint64_t)(bsweeps[b] ? bsweeps[b] : sweeps) * nq;
    }
    stats->sweeps = sweeps;
    stats->workers = g->bp[kBatchSssp].P;
    stats->tile_vertices = dg::host::batch_tile_vertices(g);
    stats->commits = mode == DG_DELAYED ? dg::host::batch_commits_per_sweep(g, kBatchSssp, a.d) : 0u;
    stats->commit_interval = stats->commits ? (uint32_t)(((uint64_t)g->n + stats->commits / 2) / stats->commits) : 0u;
    stats->err_bound = 0.0;
    stats->residual = 0.0;
    stats->seconds = secs;
    stats->edges_traversed = g->m * qe;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "no convergence within %u sweeps", max_sweeps);
  return DG_OK;
}

dg_status dg_ppr_batch(dg_graph* g, const uint32_t* sources, uint32_t k, double damping, double tol, dg_mode mode,
                       uint32_t d, dg_dtype dtype, uint32_t max_sweeps, double* out_scores, int out_on_device,
                       dg_stats* stats, void* hip_stream) {
  g_last_error.clear();
  dg_status st = check_batch(g, sources, k, mode, d, max_sweeps, out_scores);
  if (st != DG_OK) return st;
  if (!(damping >= 0.0 && damping < 1.0)) return fail(DG_ERR_INVALID_ARGUMENT, "damping must be in [0, 1)");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and >= 0");
  if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "dtype must be DG_F32 or DG_F64");
  const bool f64 = dtype == DG_F64;
  const size_t esz = f64 ? 8 : 4;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_workspace(g, 1, s)) != DG_OK) return st;
  const uint32_t NB = (k + kBatchQ - 1) / kBatchQ;
  const size_t vals = (size_t)NB * (g->n + g->K) * kBatchQ;
  const size_t xs = (size_t)NB * g->n * kBatchQ;
  CallAllocs al(g);
  uint32_t* srcd = static_cast<uint32_t*>(al.get((size_t)k * 4, s));
  void* x = al.get(xs * esz, s);
  void* c0 = al.get(vals * esz, s);
  void* c1 = mode == DG_SYNC ? al.get(vals * esz, s) : nullptr;
  const uint32_t d_eff = mode == DG_DELAYED ? std::max(1u, std::min(d, g->bp[kBatchPpr].max_block_v)) : 0u;
  // Delayed commits stage in LDS up to kLdsStageMaxD, beyond in a shadow.
  const bool need_sh = mode == DG_DELAYED && d_eff > kLdsStageMaxD;
  void* sh = need_sh ? al.get(xs * esz, s) : nullptr;
  double* resid = static_cast<double*>(al.get(((size_t)max_sweeps + 1) * NB * 8, s));
  uint32_t* count = static_cast<uint32_t*>(al.get(((size_t)max_sweeps + 1) * NB * 4, s));
  double* dang = static_cast<double*>(al.get((size_t)2 * NB * kBatchQ * 8, s));
  double* scale = static_cast<double*>(al.get((size_t)2 * NB * kBatchQ * 8, s));
  double* rhist = f64 ? nullptr : static_cast<double*>(al.get((size_t)2 * NB * kBatchQ * 8, s));
  uint32_t* qdone = static_cast<uint32_t*>(al.get((size_t)NB * kBatchQ * 4, s));
  double* part = static_cast<double*>(al.get((size_t)g->bp[kBatchPpr].P * NB * 3 * kBatchQ * 8, s));
  double* qsum = static_cast<double*>(al.get((size_t)NB * kBatchQ * 8, s));
  double* qpart = static_cast<double*>(al.get((size_t)NB * 256 * kBatchQ * 8, s));
  double* outd = out_on_device ? out_scores : static_cast<double*>(al.get((size_t)k * g->n * 8, s));
  if (!srcd || !x || !c0 || (mode == DG_SYNC && !c1) || (need_sh && !sh) || !resid || !count || !dang ||
      !scale || (!f64 && !rhist) || !qdone || !part || !qsum || !qpart || !outd)
    return fail(DG_ERR_OUT_OF_MEMORY, "batched PageRank workspace allocation failed");
  PinnedBuf poll;
  DG_HIP(alloc_mapped(&poll.p, &poll.dev, ((size_t)max_sweeps + 1) * NB * 8));
  DG_HIP(hipMemcpyAsync(srcd, sources, (size_t)k * 4, hipMemcpyHostToDevice, s));
  DG_HIP(launch_fill_f64(resid, ((size_t)max_sweeps + 1) * NB, 0.0, s));
  DG_HIP(launch_fill_f64(resid, NB, __builtin_inf(), s));
  DG_HIP(launch_fill_u32(count, ((size_t)max_sweeps + 1) * NB, 0u, s));
  DG_HIP(launch_fill_f64(dang, (size_t)2 * NB * kBatchQ, 0.0, s));
  DG_HIP(launch_fill_f64(scale, (size_t)2 * NB * kBatchQ, 1.0, s));
  if (rhist) DG_HIP(launch_fill_f64(rhist, (size_t)2 * NB * kBatchQ, __builtin_inf(), s));
  // padding lanes of the last batch start frozen
  DG_HIP(launch_fill_u32(qdone, (size_t)k, 0u, s));
  if ((size_t)NB * kBatchQ > k) DG_HIP(launch_fill_u32(qdone + k, (size_t)NB * kBatchQ - k, 1u, s));
  DG_HIP(launch_mppr_init(f64, x, c0, c1, g->out_deg, g->cpos, srcd, k, g->n, g->K, NB, dang, s));
  MpprArgs a;
  std::memset(&a, 0, sizeof a);  // call mode: no serving fields
  a.g = topo_batch(g, kBatchPpr);
  a.x = x;
  a.shadow = sh;
  a.src = srcd;
  a.resid = resid;
  a.hresid = static_cast<double*>(poll.dev);
  a.dang = dang;
  a.scale = scale;
  a.rhist = rhist;
  a.qdone = qdone;
  a.count = count;
  a.part = part;
  a.alpha = damping;
  a.tol = tol;
  a.nq = k;
  a.d = d_eff;
  a.NB = NB;
  CaptureKey key;
  key_add(key, 4);
  key_add(key, (int)mode);
  key_add(key, f64);
  key_add(key, max_sweeps);
  key_add(key, c0);
  key_add(key, c1);
  key_add(key, a);
  auto launch = [&](uint32_t kk, hipStream_t q) {
    if (mode == DG_SYNC) {
      a.cin = (kk & 1) ? c1 : c0;
      a.cout = (kk & 1) ? c0 : c1;
    } else {
      a.cin = c0;
      a.cout = c0;
    }
    a.k = kk;
    return launch_mppr_sweep((int)mode, f64, a, q);
  };
  std::vector<uint32_t> bsweeps(NB, 0);
  double last_r = 0.0;
  auto done = [&](const unsigned char* p, uint32_t kk) {
    bool all = true;
    last_r = 0.0;
    for (uint32_t b = 0; b < NB; ++b) {
      double r;
      std::memcpy(&r, p + 8 * b, 8);
      const bool ok = !(r >= tol);
      if (ok && bsweeps[b] == 0) bsweeps[b] = kk + 1;
      if (!ok) last_r = std::max(last_r, r);
      all = all && ok;
    }
    return all;
  };
  uint32_t sweeps = 0;
  double secs = 0.0;
  bool conv = false;
  if ((st = drive(g, max_sweeps, s, (size_t)NB * 8, static_cast<unsigned char*>(poll.p), launch, done, sweeps, secs,
                  conv, &key)) != DG_OK)
    return st;
  DG_HIP(launch_mppr_out(f64, x, qpart, qsum, g->n, k, NB, outd, s));
  if (!out_on_device) DG_HIP(hipMemcpyAsync(out_scores, outd, (size_t)k * g->n * 8, hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  if (stats) {
    uint64_t qe = 0;
    for (uint32_t b = 0; b < NB; ++b) {
      const uint32_t nq = std::min(kBatchQ, k - b * kBatchQ);
      qe += (uint64_t)(bsweeps[b] ? bsweeps[b] : sweeps) * nq;
    }
    stats->sweeps = sweeps;
    stats->workers = g->bp[kBatchPpr].P;
    stats->tile_vertices = dg::host::batch_tile_vertices(g);
    stats->commits = mode == DG_DELAYED ? dg::host::batch_commits_per_sweep(g, kBatchPpr, a.d) : 0u;
    stats->commit_interval = stats->commits ? (uint32_t)(((uint64_t)g->n + stats->commits / 2) / stats->commits) : 0u;
    stats->err_bound = 0.0;
    stats->residual = last_r;
    stats->seconds = secs;
    stats->edges_traversed = g->m * qe;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "no convergence within %u sweeps", max_sweeps);
  return DG_OK;
}

dg_status dg_graph_repartition(dg_graph* g, uint32_t workers, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  uint32_t P = workers ? std::max(1u, std::min(workers, g->T))
                       : default_workers(g, g->G ? kSetWorkersPerCU : kWorkersPerCU);
  std::vector<uint32_t> work_t, wseg, wgraph;
  if (g->G) {
    // a set's union graph: every graph keeps worker blocks of its own
    build_workers_seg(g->tile_v_h, g->tile_e0_h, g->seg_v, std::max(P, g->G), work_t, wseg);
    P = wseg.back();
    wgraph.resize(P);
    for (uint32_t gi = 0; gi < g->G; ++gi)
      for (uint32_t wk = wseg[gi]; wk < wseg[gi + 1]; ++wk) wgraph[wk] = gi;
  }
  if (P == g->P) return DG_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!g->G) build_workers(g->tile_v_h, g->tile_e0_h, P, work_t);
  uint32_t mbv = 1;
  for (uint32_t w = 0; w < P; ++w) mbv = std::max(mbv, g->tile_v_h[work_t[w + 1]] - g->tile_v_h[work_t[w]]);
  DG_HIP(hipStreamSynchronize(s));
  uint32_t* wt = static_cast<uint32_t*>(dev_alloc(g, (size_t)(P + 1) * 4, s));
  double* part = g->part ? static_cast<double*>(dev_alloc(g, 3 * (size_t)P * sizeof(double), s)) : nullptr;
  uint32_t* wsd = g->G ? static_cast<uint32_t*>(dev_alloc(g, wseg.size() * 4, s)) : nullptr;
  uint32_t* wgd = g->G ? static_cast<uint32_t*>(dev_alloc(g, (size_t)P * 4, s)) : nullptr;
  if (!wt || (g->part && !part) || (g->G && (!wsd || !wgd))) {
    dev_free(g, wt);
    dev_free(g, part);
    dev_free(g, wsd);
    dev_free(g, wgd);
    return fail(DG_ERR_OUT_OF_MEMORY, "repartition allocation failed");
  }
  DG_HIP(hipMemcpyAsync(wt, work_t.data(), (size_t)(P + 1) * 4, hipMemcpyHostToDevice, s));
  if (g->G) {
    DG_HIP(hipMemcpyAsync(wsd, wseg.data(), wseg.size() * 4, hipMemcpyHostToDevice, s));
    DG_HIP(hipMemcpyAsync(wgd, wgraph.data(), (size_t)P * 4, hipMemcpyHostToDevice, s));
  }
  DG_HIP(hipStreamSynchronize(s));
  g->graph_bytes += 4 * ((uint64_t)work_t.size() + wseg.size() + wgraph.size());
  g->graph_bytes -= 4 * ((uint64_t)g->work_t_h.size() + (g->G ? g->wseg_h.size() + g->wgraph_h.size() : 0u));
  dev_free(g, g->work_t);
  g->work_t = wt;
  g->work_t_h = work_t;
  if (g->part) {
    dev_free(g, g->part);
    g->part = part;
  }
  if (g->G) {
    dev_free(g, g->wseg);
    dev_free(g, g->wgraph);
    g->wseg = wsd;
    g->wgraph = wgd;
    g->wseg_h.swap(wseg);
    g->wgraph_h.swap(wgraph);
  }
  g->P = P;
  g->max_block_v = mbv;
  dg::host::drop_captures(g);
  return DG_OK;
}

dg_status dg_graph_set_capture(dg_graph* g, uint32_t chunk_sweeps) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (chunk_sweeps > kMaxCaptureChunk)
    return fail(DG_ERR_INVALID_ARGUMENT, "chunk_sweeps = %u beyond %u", chunk_sweeps, kMaxCaptureChunk);
  if (chunk_sweeps != g->capture) dg::host::drop_captures(g);
  g->capture = chunk_sweeps;
  return DG_OK;
}

dg_status dg_graph_set_mapping(dg_graph* g, uint32_t sweep_variant, uint32_t resident_vertices, uint32_t workers,
                               void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (g->G) return fail(DG_ERR_UNSUPPORTED, "a set's union graph keeps its own mapping");
  if (sweep_variant > DG_SWEEP_NARROW)
    return fail(DG_ERR_INVALID_ARGUMENT, "unknown sweep_variant %u", sweep_variant);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const uint32_t want = sweep_variant == DG_SWEEP_AUTO ? g->variant0 : sweep_variant;
  const bool narrow_now = g->variant == kNarrow, narrow_want = want == kNarrow;
  if (narrow_now != narrow_want) {
    // The narrow variant has its own tile cap: rebuild the tiles, the batched
    // tiles split from them, and every partition over either.
    std::vector<uint32_t> tv, te0, btv, bte0;
    BatchPart nb[2];
    try {
      build_tiles(g->in_ptr_h, g->n, tv, nullptr, narrow_want ? (uint32_t)kTileENarrow : (uint32_t)kTileE);
      te0.resize(tv.size());
      for (size_t t = 0; t < tv.size(); ++t) te0[t] = g->in_ptr_h[tv[t]];
      dg::host::build_batch_tiles(tv, g->in_ptr_h, dg::host::kBatchTileE, btv, bte0);
    } catch (const std::bad_alloc&) {
      return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    const uint32_t T = (uint32_t)tv.size() - 1, Tb = (uint32_t)btv.size() - 1;
    for (int b : {kBatchSssp, kBatchPpr}) {
      const uint32_t Pb =
          dg::host::batch_workers_for(g->cus, b == kBatchSssp ? kBatchSsspWorkersPerCU : kBatchPprWorkersPerCU, Tb);
      dg::host::plan_batch_part(btv, bte0, Pb, nb[b]);
    }
    DG_HIP(hipStreamSynchronize(s));
    uint32_t* tvd = static_cast<uint32_t*>(dev_alloc(g, tv.size() * 4, s));
    uint32_t* btvd = static_cast<uint32_t*>(dev_alloc(g, btv.size() * 4, s));
    for (BatchPart& b : nb) b.work_t = static_cast<uint32_t*>(dev_alloc(g, b.work_t_h.size() * 4, s));
    if (!tvd || !btvd || !nb[0].work_t || !nb[1].work_t) {
      dev_free(g, tvd);
      dev_free(g, btvd);
      for (BatchPart& b : nb) dev_free(g, b.work_t);
      return fail(DG_ERR_OUT_OF_MEMORY, "re-tiling allocation failed");
    }
    DG_HIP(hipMemcpyAsync(tvd, tv.data(), tv.size() * 4, hipMemcpyHostToDevice, s));
    DG_HIP(hipMemcpyAsync(btvd, btv.data(), btv.size() * 4, hipMemcpyHostToDevice, s));
    for (BatchPart& b : nb)
      DG_HIP(hipMemcpyAsync(b.work_t, b.work_t_h.data(), b.work_t_h.size() * 4, hipMemcpyHostToDevice, s));
    DG_HIP(hipStreamSynchronize(s));
    g->graph_bytes += 4 * ((uint64_t)tv.size() + btv.size() + nb[0].work_t_h.size() + nb[1].work_t_h.size());
    g->graph_bytes -= 4 * ((uint64_t)g->tile_v_h.size() + g->btile_v_h.size() + g->bp[0].work_t_h.size() +
                           g->bp[1].work_t_h.size());
    dev_free(g, g->tile_v);
    g->tile_v = tvd;
    dev_free(g, g->btile_v);
    g->btile_v = btvd;
    for (int b : {kBatchSssp, kBatchPpr}) {
      dev_free(g, g->bp[b].work_t);
      g->bp[b] = std::move(nb[b]);
    }
    g->tile_v_h.swap(tv);
    g->tile_e0_h.swap(te0);
    g->btile_v_h.swap(btv);
    g->btile_e0_h.swap(bte0);
    g->T = T;
    g->P = 0;  // forces the repartition below
  }
  g->variant = want;
  g->res_limit = resident_vertices == DG_RESIDENT_AUTO ? 0xFFFFFFFFu : resident_vertices;
  dg::host::drop_captures(g);
  return dg_graph_repartition(g, workers, hip_stream);
}

}  // extern "C"

namespace {

// Median, min and max of a few timed runs.
struct Spread {
  double med = 0.0, lo = 0.0, hi = 0.0;
};
Spread spread_of(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  Spread sp;
  if (v.empty()) return sp;
  sp.lo = v.front();
  sp.hi = v.back();
  sp.med = v.size() % 2 ? v[v.size() / 2] : 0.5 * (v[v.size() / 2 - 1] + v[v.size() / 2]);
  return sp;
}

constexpr uint32_t kTuneRepeats = 3;
constexpr uint32_t kTuneCaptureChunk = 16;  // sweeps per captured chunk tried by the tuner

}  // namespace

extern "C" {

dg_status dg_tune(dg_graph* g, dg_algo algo, dg_dtype dtype, double tol, uint32_t src, uint32_t flags,
                  dg_tuning* out, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  if (algo != DG_ALGO_PAGERANK && algo != DG_ALGO_SSSP) return fail(DG_ERR_INVALID_ARGUMENT, "unknown algorithm");
  if (flags & ~(uint32_t)(DG_TUNE_NO_CACHE | DG_TUNE_KEEP_WORKERS))
    return fail(DG_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
  if (algo == DG_ALGO_PAGERANK) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and > 0");
    if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "dtype must be DG_F32 or DG_F64");
    src = 0;
  } else {
    if (src >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "source %u >= n", src);
    if (!g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "the graph was created without weights");
    dtype = DG_F32;
    tol = 0.0;
  }
  const bool keep = (flags & DG_TUNE_KEEP_WORKERS) != 0;
  const bool can_map = g->G == 0 && !keep;  // sets keep their per-graph mapping
  dg_tuning cached;
  if (!(flags & DG_TUNE_NO_CACHE) && tune_find(g->hash, (int)algo, (int)dtype, tol, src, cached)) {
    if (!keep) {
      dg_status st = can_map ? dg_graph_set_mapping(g, cached.sweep_variant, cached.resident_vertices, cached.workers,
                                                    hip_stream)
                             : dg_graph_repartition(g, cached.workers, hip_stream);
      if (st == DG_OK) st = dg_graph_set_capture(g, cached.capture_chunk);
      if (st != DG_OK) return st;
    }
    *out = cached;
    out->from_cache = 1;
    out->workers = g->P;
    return DG_OK;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  CallAllocs al(g);
  void* scratch = al.get((size_t)g->n * 8, s);
  if (!scratch) return fail(DG_ERR_OUT_OF_MEMORY, "tuning scratch allocation failed");
  const uint32_t full = algo == DG_ALGO_PAGERANK ? 10000u : std::min<uint32_t>(g->n + 1, kMaxSweeps);
  // one run: status DG_OK or DG_ERR_NOT_CONVERGED (probes) fill st
  auto run = [&](dg_mode mode, uint32_t d, double tl, uint32_t ms, dg_stats& st) -> dg_status {
    dg_status r = algo == DG_ALGO_PAGERANK
                      ? dg_pagerank(g, 0.85, tl, mode, d, dtype, ms, static_cast<double*>(scratch), 1, &st, hip_stream)
                      : dg_sssp(g, src, mode, d, ms, static_cast<uint32_t*>(scratch), 1, &st, hip_stream);
    if (r == DG_ERR_NOT_CONVERGED) r = DG_OK;
    return r;
  };
  // kTuneRepeats full runs: the spread of their times to convergence
  auto timed = [&](dg_mode mode, uint32_t d, Spread& sp, uint32_t& sweeps) -> dg_status {
    std::vector<double> t;
    for (uint32_t i = 0; i < kTuneRepeats; ++i) {
      dg_stats x{};
      dg_status r = run(mode, d, tol, full, x);
      if (r != DG_OK) return r;
      t.push_back(x.seconds);
      sweeps = x.sweeps;
    }
    sp = spread_of(t);
    return DG_OK;
  };
  dg_status st;
  // Every stage but the last measures one launch per sweep.
  const uint32_t cap0 = g->capture;
  if ((st = dg_graph_set_capture(g, 0)) != DG_OK) return st;
  // The default the choice is compared with: the creation-time mapping and
  // partition, delayed d = 64.
  const uint32_t P0 = g->P, var0 = g->variant, res0 = g->res_limit;
  Spread def{};
  uint32_t def_sweeps = 0;
  if (can_map && (st = dg_graph_set_mapping(g, DG_SWEEP_AUTO, DG_RESIDENT_AUTO, 0, hip_stream)) != DG_OK) return st;
  if ((st = timed(DG_DELAYED, 64, def, def_sweeps)) != DG_OK) return st;
  if (can_map && (st = dg_graph_set_mapping(g, var0, res0, P0, hip_stream)) != DG_OK) return st;

  struct Cand {
    dg_mode mode;
    uint32_t d;
    uint32_t sweeps;
  };
  std::vector<Cand> cands = {{DG_SYNC, 1, 0},      {DG_ASYNC, 1, 0},     {DG_DELAYED, 16, 0},
                             {DG_DELAYED, 64, 0},  {DG_DELAYED, 256, 0}, {DG_DELAYED, 1024, 0},
                             {DG_DELAYED, 4096, 0}, {DG_DELAYED, DG_D_WHOLE, 0}};
  // Stage 1, commit mode and interval: sweep counts from a full run of each
  // candidate at the current mapping.
  for (auto& c : cands) {
    dg_stats x{};
    if ((st = run(c.mode, c.d, tol, full, x)) != DG_OK) return st;
    c.sweeps = x.sweeps;
  }
  // Stage 2, partition size: time per sweep from short fixed-length probes
  // (tol 0 for PageRank) of every candidate for every size, best of two; the
  // least predicted time to convergence wins.
  std::vector<uint32_t> Ps;
  if (keep) {
    Ps.push_back(g->P);
  } else {
    for (uint32_t per_cu : {1u, 2u, 3u, 4u}) {
      const uint32_t P = default_workers(g, per_cu);
      if (std::find(Ps.begin(), Ps.end(), P) == Ps.end()) Ps.push_back(P);
    }
  }
  const uint32_t probe = 6;
  double best = 1e300;
  uint32_t bestP = g->P, bestc = 0, evaluated = 0;
  for (uint32_t P : Ps) {
    if ((st = dg_graph_repartition(g, P, hip_stream)) != DG_OK) return st;
    for (uint32_t i = 0; i < cands.size(); ++i) {
      double ts = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        dg_stats x{};
        if ((st = run(cands[i].mode, cands[i].d, algo == DG_ALGO_PAGERANK ? 0.0 : tol, probe, x)) != DG_OK)
          return st;
        if (x.sweeps) ts = std::min(ts, x.seconds / x.sweeps);
      }
      const double pred = ts * cands[i].sweeps;
      ++evaluated;
      if (pred < best) {
        best = pred;
        bestP = P;
        bestc = i;
      }
    }
  }
  if ((st = dg_graph_repartition(g, bestP, hip_stream)) != DG_OK) return st;
  const dg_mode mode = cands[bestc].mode;
  const uint32_t d = cands[bestc].d;
  // Stage 3, the mapping of edges onto the workgroup (sweep variant) and the
  // size of the resident table, for the chosen mode, d and partition: each
  // candidate timed kTuneRepeats times to convergence (their sweep counts
  // depend on the mapping in the asynchronous modes), the least median wins.
  uint32_t best_var = g->variant, best_res = g->res_limit, sweeps = 0;
  Spread chosen{};
  if ((st = timed(mode, d, chosen, sweeps)) != DG_OK) return st;
  ++evaluated;
  if (can_map) {
    const uint32_t R = g->R;
    std::vector<uint32_t> res_c = {DG_RESIDENT_AUTO};
    if (R >= 2) res_c.push_back(R / 2);
    if (R > 0) res_c.push_back(0);
    for (uint32_t var : {DG_SWEEP_WIDE, DG_SWEEP_WIDE_INFLIGHT, DG_SWEEP_NARROW}) {
      for (uint32_t res : res_c) {
        const uint32_t res_l = res == DG_RESIDENT_AUTO ? 0xFFFFFFFFu : res;
        if (var == best_var && res_l == best_res) continue;  // the current mapping, timed above
        if ((st = dg_graph_set_mapping(g, var, res, bestP, hip_stream)) != DG_OK) return st;
        Spread sp{};
        uint32_t sw = 0;
        if ((st = timed(mode, d, sp, sw)) != DG_OK) return st;
        ++evaluated;
        if (sp.med < chosen.med) {
          chosen = sp;
          sweeps = sw;
          best_var = var;
          best_res = res_l;
        }
      }
    }
    if ((st = dg_graph_set_mapping(g, best_var, best_res == 0xFFFFFFFFu ? DG_RESIDENT_AUTO : best_res, bestP,
                                   hip_stream)) != DG_OK)
      return st;
  }
  // Stage 4, the launch: chunks of captured sweeps against one launch per
  // sweep for the chosen configuration (a first, untimed call records the
  // chunks); the lesser median wins and the graph keeps it.
  uint32_t cap = 0;
  if (!keep) {
    if ((st = dg_graph_set_capture(g, kTuneCaptureChunk)) != DG_OK) return st;
    dg_stats x{};
    Spread sp{};
    uint32_t sw = 0;
    st = run(mode, d, tol, full, x);
    if (st == DG_OK) st = timed(mode, d, sp, sw);
    if (st != DG_OK) {
      (void)dg_graph_set_capture(g, 0);
      return st;
    }
    ++evaluated;
    if (sp.med < chosen.med) {
      chosen = sp;
      sweeps = sw;
      cap = kTuneCaptureChunk;
    } else if ((st = dg_graph_set_capture(g, 0)) != DG_OK) {
      return st;
    }
  } else if ((st = dg_graph_set_capture(g, cap0)) != DG_OK) {
    return st;
  }
  dg_tuning t{};
  t.workers = g->P;
  t.mode = mode;
  t.d = d;
  t.sweeps = sweeps;
  t.seconds = chosen.med;
  t.seconds_min = chosen.lo;
  t.seconds_max = chosen.hi;
  t.predicted_seconds = best;
  t.candidates = evaluated;
  t.from_cache = 0;
  t.graph_hash = g->hash;
  t.sweep_variant = g->variant;
  t.resident_vertices = best_res == 0xFFFFFFFFu ? DG_RESIDENT_AUTO : best_res;
  t.repeats = kTuneRepeats;
  t.capture_chunk = cap;
  t.default_seconds = def.med;
  t.default_seconds_min = def.lo;
  t.default_seconds_max = def.hi;
  tune_put(TuneEntry{g->hash, (int)algo, (int)dtype, tol, src, t});
  *out = t;
  return DG_OK;
}

}  // extern "C"

namespace {

// Re-partitions the batched tiles of batched partition `which` over Pb
// workers.
dg_status set_batch_workers(dg_graph* g, int which, uint32_t Pb, hipStream_t s) {
  Pb = std::max(1u, std::min(Pb, (uint32_t)g->btile_v_h.size() - 1));
  if (Pb == g->bp[which].P) return DG_OK;
  BatchPart nb;
  dg::host::plan_batch_part(g->btile_v_h, g->btile_e0_h, Pb, nb);
  DG_HIP(hipStreamSynchronize(s));
  nb.work_t = static_cast<uint32_t*>(dev_alloc(g, nb.work_t_h.size() * 4, s));
  if (!nb.work_t) return fail(DG_ERR_OUT_OF_MEMORY, "batched partition allocation failed");
  DG_HIP(hipMemcpyAsync(nb.work_t, nb.work_t_h.data(), nb.work_t_h.size() * 4, hipMemcpyHostToDevice, s));
  DG_HIP(hipStreamSynchronize(s));
  g->graph_bytes += 4 * (uint64_t)nb.work_t_h.size();
  g->graph_bytes -= 4 * (uint64_t)g->bp[which].work_t_h.size();
  dev_free(g, g->bp[which].work_t);
  g->bp[which] = std::move(nb);
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_graph_repartition_batch(dg_graph* g, dg_algo algo, uint32_t workers, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(DG_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (algo != DG_ALGO_PAGERANK && algo != DG_ALGO_SSSP) return fail(DG_ERR_INVALID_ARGUMENT, "unknown algorithm");
  const int which = algo == DG_ALGO_SSSP ? kBatchSssp : kBatchPpr;
  const uint32_t P = workers ? workers
                             : dg::host::batch_workers(g, which == kBatchSssp ? kBatchSsspWorkersPerCU
                                                                              : kBatchPprWorkersPerCU);
  return set_batch_workers(g, which, P, static_cast<hipStream_t>(hip_stream));
}

dg_status dg_tune_batch(dg_graph* g, dg_algo algo, dg_dtype dtype, double tol, const uint32_t* sources, uint32_t k,
                        uint32_t flags, dg_tuning* out, void* hip_stream) {
  g_last_error.clear();
  if (!g || !out || !sources) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  if (algo != DG_ALGO_PAGERANK && algo != DG_ALGO_SSSP) return fail(DG_ERR_INVALID_ARGUMENT, "unknown algorithm");
  if (k == 0 || k > 1024) return fail(DG_ERR_INVALID_ARGUMENT, "k = %u outside [1, 1024]", k);
  if (flags != 0) return fail(DG_ERR_INVALID_ARGUMENT, "flags must be 0 (got 0x%x)", flags);
  for (uint32_t i = 0; i < k; ++i)
    if (sources[i] >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "sources[%u] = %u >= n", i, sources[i]);
  if (algo == DG_ALGO_PAGERANK) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and > 0");
    if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "dtype must be DG_F32 or DG_F64");
  } else if (!g->has_w) {
    return fail(DG_ERR_INVALID_ARGUMENT, "the graph was created without weights");
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  CallAllocs al(g);
  void* outd = al.get((size_t)k * g->n * (algo == DG_ALGO_PAGERANK ? 8 : 4), s);
  if (!outd) return fail(DG_ERR_OUT_OF_MEMORY, "tuning output allocation failed");
  auto timed = [&](dg_mode mode, uint32_t d, Spread& sp, uint32_t& sweeps) -> dg_status {
    std::vector<double> t;
    for (uint32_t i = 0; i < kTuneRepeats; ++i) {
      dg_stats x{};
      dg_status r = algo == DG_ALGO_PAGERANK
                        ? dg_ppr_batch(g, sources, k, 0.85, tol, mode, d, dtype, 10000, static_cast<double*>(outd), 1,
                                       &x, hip_stream)
                        : dg_sssp_batch(g, sources, k, mode, d, std::min<uint32_t>(g->n + 1, 100000),
                                        static_cast<uint32_t*>(outd), 1, &x, hip_stream);
      if (r == DG_ERR_NOT_CONVERGED) r = DG_OK;
      if (r != DG_OK) return r;
      t.push_back(x.seconds);
      sweeps = x.sweeps;
    }
    sp = spread_of(t);
    return DG_OK;
  };
  dg_status st;
  const int which = algo == DG_ALGO_SSSP ? kBatchSssp : kBatchPpr;
  const uint32_t Pb_def =
      dg::host::batch_workers(g, which == kBatchSssp ? kBatchSsspWorkersPerCU : kBatchPprWorkersPerCU);
  Spread def{};
  uint32_t sw_def = 0;
  if ((st = set_batch_workers(g, which, Pb_def, s)) != DG_OK) return st;
  if ((st = timed(DG_DELAYED, 64, def, sw_def)) != DG_OK) return st;
  struct Cand {
    dg_mode mode;
    uint32_t d;
  };
  const Cand cands[] = {{DG_SYNC, 1},       {DG_ASYNC, 1},        {DG_DELAYED, 16},
                        {DG_DELAYED, 64},   {DG_DELAYED, 256},    {DG_DELAYED, DG_D_WHOLE}};
  Spread best{};
  best.med = 1e300;
  uint32_t bestP = Pb_def, best_sw = 0, evaluated = 0;
  Cand bestc = {DG_DELAYED, 64};
  for (uint32_t per_cu : {3u, 5u, 8u}) {
    const uint32_t Pb = dg::host::batch_workers(g, per_cu);
    if ((st = set_batch_workers(g, which, Pb, s)) != DG_OK) return st;
    for (const Cand& c : cands) {
      Spread sp{};
      uint32_t sw = 0;
      if (Pb == Pb_def && c.mode == DG_DELAYED && c.d == 64) {
        sp = def;
        sw = sw_def;
      } else if ((st = timed(c.mode, c.d, sp, sw)) != DG_OK) {
        return st;
      }
      ++evaluated;
      if (sp.med < best.med) {
        best = sp;
        bestP = g->bp[which].P;
        bestc = c;
        best_sw = sw;
      }
    }
  }
  if ((st = set_batch_workers(g, which, bestP, s)) != DG_OK) return st;
  dg_tuning t{};
  t.workers = g->bp[which].P;
  t.mode = bestc.mode;
  t.d = bestc.d;
  t.sweeps = best_sw;
  t.seconds = best.med;
  t.seconds_min = best.lo;
  t.seconds_max = best.hi;
  t.predicted_seconds = best.med;
  t.candidates = evaluated;
  t.graph_hash = g->hash;
  t.sweep_variant = g->variant;
  t.resident_vertices = DG_RESIDENT_AUTO;
  t.repeats = kTuneRepeats;
  t.default_seconds = def.med;
  t.default_seconds_min = def.lo;
  t.default_seconds_max = def.hi;
  *out = t;
  return DG_OK;
}

dg_status dg_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
  return DG_OK;
}

dg_status dg_tune_cache_save(const char* path) {
  g_last_error.clear();
  if (!path) return fail(DG_ERR_INVALID_ARGUMENT, "path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(DG_ERR_INVALID_ARGUMENT, "cannot open %s for writing", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::fprintf(f, "# dg tuning cache: hash algo dtype tol src workers mode d sweeps seconds variant resident capture\n");
  for (const auto& e : g_tune_cache)
    std::fprintf(f, "%016llx %d %d %.17g %u %u %d %u %u %.9g %u %u %u\n", (unsigned long long)e.hash, e.algo, e.dtype,
                 e.tol, e.src, e.t.workers, (int)e.t.mode, e.t.d, e.t.sweeps, e.t.seconds, e.t.sweep_variant,
                 e.t.resident_vertices, e.t.capture_chunk);
  const bool ok = std::fclose(f) == 0;
  return ok ? DG_OK : fail(DG_ERR_INVALID_ARGUMENT, "writing %s failed", path);
}

dg_status dg_tune_cache_load(const char* path) {
  g_last_error.clear();
  if (!path) return fail(DG_ERR_INVALID_ARGUMENT, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(DG_ERR_INVALID_ARGUMENT, "cannot open %s", path);
  char line[512];
  uint32_t bad = 0;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    unsigned long long h = 0;
    int algo = 0, dtype = 0, mode = 0;
    double tol = 0.0, secs = 0.0;
    unsigned src = 0, workers = 0, d = 0, sweeps = 0, variant = DG_SWEEP_AUTO, res = DG_RESIDENT_AUTO, cap = 0;
    const int got = std::sscanf(line, "%llx %d %d %lg %u %u %d %u %u %lg %u %u %u", &h, &algo, &dtype, &tol, &src,
                                &workers, &mode, &d, &sweeps, &secs, &variant, &res, &cap);
    if ((got != 10 && got != 12 && got != 13) || variant > DG_SWEEP_NARROW || cap > kMaxCaptureChunk ||
        (algo != DG_ALGO_PAGERANK && algo != DG_ALGO_SSSP) || mode < DG_SYNC || mode > DG_DELAYED || workers == 0 ||
        (mode == DG_DELAYED && d == 0)) {
      ++bad;
      continue;
    }
    dg_tuning t{};
    t.workers = workers;
    t.mode = (dg_mode)mode;
    t.d = d;
    t.sweeps = sweeps;
    t.seconds = secs;
    t.graph_hash = h;
    t.sweep_variant = variant;
    t.resident_vertices = res;
    t.capture_chunk = cap;
    tune_put(TuneEntry{(uint64_t)h, algo, dtype, tol, src, t});
  }
  std::fclose(f);
  if (bad) return fail(DG_ERR_INVALID_ARGUMENT, "%u malformed line(s) in %s skipped", bad, path);
  return DG_OK;
}

}  // extern "C"

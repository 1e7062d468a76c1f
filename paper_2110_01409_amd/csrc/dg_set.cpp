// Host side of graph sets (dg_set_*): many graphs resident as one union
// graph, swept together in one launch per sweep, with each graph stopping on
// its own rule.  Chunks of sweeps are launched eagerly or as a captured HIP
// graph that is instantiated once and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dg.h"
#include "dg_host.hpp"
#include "dg_internal.hpp"

using namespace dg;
using dg::host::fail;
using dg::host::g_last_error;

namespace {

constexpr uint32_t kSetChunk = 8;       // sweeps per launch chunk (and per captured graph)
constexpr uint32_t kSetWorkersPerCU = 5;
constexpr uint32_t kSetMaxSweeps = 1000000;
// Set sweeps are switched off: their first GPU run (synchronous Bellman-Ford
// through a captured chunk) stopped making progress and no cause has been
// identified in this code yet.  dg_set_pagerank / dg_set_sssp validate their
// arguments and then return DG_ERR_UNSUPPORTED without touching the device.
constexpr bool kSetSweepsEnabled = false;

}  // namespace

struct dg_set {
  uint32_t G = 0, N = 0, T = 0, P = 0, cus = 0;
  uint64_t M = 0;
  bool has_w = false;
  dg_alloc_fn alloc = nullptr;
  dg_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  hipStream_t own = nullptr;  // non-blocking stream every call runs on (capturable)
  std::vector<void*> owned;
  uint64_t bytes = 0;
  std::vector<uint32_t> voff;  // host copy of g_voff
  std::vector<uint64_t> gm;    // edges of each graph
  // resident arrays
  uint32_t *in_ptr = nullptr, *in_src = nullptr, *in_w = nullptr, *out_deg = nullptr;
  uint32_t *tile_v = nullptr, *tile_g = nullptr, *g_voff = nullptr, *g_toff = nullptr;
  double* dang0 = nullptr;  // [G] dangling fraction of each graph (initial spread mass)
  // workspace
  void* vals[4] = {nullptr, nullptr, nullptr, nullptr};  // 8N bytes each
  double *tpart = nullptr, *gdang = nullptr, *gres = nullptr;
  uint32_t *tchg = nullptr, *gdone = nullptr, *srcd = nullptr, *cur = nullptr;
  uint32_t ws_sweeps = 0;
  uint32_t *next = nullptr, *live = nullptr, *fcount = nullptr;
  uint32_t* host_live = nullptr;       // mapped pinned [S+1]
  uint32_t* host_live_dev = nullptr;   // its device address
  hipEvent_t ev_in = nullptr, ev_start = nullptr, ev_chunk[2] = {nullptr, nullptr};
  // cached executable graph of one chunk and the launch it was captured from
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> exec_key;
};

namespace {

void* set_alloc(dg_set* s, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (s->alloc) {
    p = s->alloc(bytes, s->own, s->ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) s->owned.push_back(p);
  return p;
}

void set_free(dg_set* s, void* p) {
  if (!p) return;
  auto it = std::find(s->owned.begin(), s->owned.end(), p);
  if (it != s->owned.end()) s->owned.erase(it);
  if (s->free_fn) s->free_fn(p, s->own, s->ctx);
  else (void)hipFree(p);
}

void set_release(dg_set* s) {
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  s->exec = nullptr;
  if (s->host_live) (void)hipHostFree(s->host_live);
  s->host_live = nullptr;
  std::vector<void*> all = s->owned;
  for (void* p : all) set_free(s, p);
  s->owned.clear();
  for (hipEvent_t* e : {&s->ev_in, &s->ev_start, &s->ev_chunk[0], &s->ev_chunk[1]})
    if (*e) (void)hipEventDestroy(*e), *e = nullptr;
  if (s->own) (void)hipStreamDestroy(s->own);
  s->own = nullptr;
}

dg_status set_workspace(dg_set* s, uint32_t S) {
  if (!s->vals[0]) {
    for (auto& v : s->vals)
      if (!(v = set_alloc(s, (size_t)s->N * 8))) return fail(DG_ERR_OUT_OF_MEMORY, "set workspace allocation failed");
    s->tpart = static_cast<double*>(set_alloc(s, (size_t)s->T * 16));
    s->tchg = static_cast<uint32_t*>(set_alloc(s, (size_t)s->T * 4));
    s->gdang = static_cast<double*>(set_alloc(s, (size_t)s->G * 16));
    s->gres = static_cast<double*>(set_alloc(s, (size_t)s->G * 8));
    s->gdone = static_cast<uint32_t*>(set_alloc(s, (size_t)s->G * 4));
    s->srcd = static_cast<uint32_t*>(set_alloc(s, (size_t)s->G * 4));
    s->cur = static_cast<uint32_t*>(set_alloc(s, 4));
    if (!s->tpart || !s->tchg || !s->gdang || !s->gres || !s->gdone || !s->srcd || !s->cur)
      return fail(DG_ERR_OUT_OF_MEMORY, "set workspace allocation failed");
  }
  if (s->ws_sweeps < S) {
    if (s->exec) (void)hipGraphExecDestroy(s->exec);  // captured with the old arrays
    s->exec = nullptr;
    s->exec_key.clear();
    set_free(s, s->next);
    set_free(s, s->live);
    set_free(s, s->fcount);
    if (s->host_live) (void)hipHostFree(s->host_live);
    s->host_live = nullptr;
    s->ws_sweeps = 0;
    const size_t k = (size_t)S + 1;
    s->next = static_cast<uint32_t*>(set_alloc(s, k * 4));
    s->live = static_cast<uint32_t*>(set_alloc(s, k * 4));
    s->fcount = static_cast<uint32_t*>(set_alloc(s, k * 4));
    if (!s->next || !s->live || !s->fcount) return fail(DG_ERR_OUT_OF_MEMORY, "set sweep state allocation failed");
    DG_HIP(hipHostMalloc((void**)&s->host_live, k * 4, hipHostMallocMapped | hipHostMallocCoherent));
    DG_HIP(hipHostGetDevicePointer((void**)&s->host_live_dev, s->host_live, 0));
    s->ws_sweeps = S;
  }
  return DG_OK;
}

SetTopo set_topo(const dg_set* s) {
  SetTopo t;
  t.in_ptr = s->in_ptr;
  t.in_src = s->in_src;
  t.in_w = s->in_w;
  t.out_deg = s->out_deg;
  t.tile_v = s->tile_v;
  t.tile_g = s->tile_g;
  t.g_voff = s->g_voff;
  t.g_toff = s->g_toff;
  t.N = s->N;
  t.T = s->T;
  t.G = s->G;
  t.P = s->P;
  return t;
}

SetCtl set_ctl(const dg_set* s, uint32_t S) {
  SetCtl c;
  c.cur = s->cur;
  c.next = s->next;
  c.live = s->live;
  c.fcount = s->fcount;
  c.gdone = s->gdone;
  c.host_live = s->host_live_dev;
  c.S = S;
  return c;
}

// Runs chunks of kSetChunk sweeps on s->own until every graph has stopped or
// S sweeps ran.  launch(stream) enqueues one sweep.  With a captured graph
// the chunk is recorded once (per distinct launch, identified by key) and
// replayed; two chunks are in flight while the host reads the live count the
// device wrote into mapped memory.
template <typename Launch>
dg_status run_chunks(dg_set* s, uint32_t S, bool eager, const std::vector<unsigned char>& key, Launch launch,
                     uint32_t& chunks_run, double& seconds, bool& converged) {
  const uint32_t C = kSetChunk;
  if (!eager && (!s->exec || s->exec_key != key)) {
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    s->exec = nullptr;
    hipGraph_t graph = nullptr;
    DG_HIP(hipStreamBeginCapture(s->own, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (uint32_t j = 0; j < C && le == hipSuccess; ++j) le = launch(s->own);
    const hipError_t ce = hipStreamEndCapture(s->own, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return fail(DG_ERR_DEVICE, "capture of a sweep chunk failed: %s",
                  hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ie = hipGraphInstantiate(&s->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      s->exec = nullptr;
      (void)hipGetLastError();
      return fail(DG_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    }
    s->exec_key = key;
  }
  auto enqueue = [&](uint32_t c) -> dg_status {
    if (eager) {
      for (uint32_t j = 0; j < C; ++j) {
        const hipError_t e = launch(s->own);
        if (e != hipSuccess) return fail(DG_ERR_DEVICE, "sweep launch failed: %s", hipGetErrorString(e));
      }
    } else {
      DG_HIP(hipGraphLaunch(s->exec, s->own));
    }
    DG_HIP(hipEventRecord(s->ev_chunk[c & 1], s->own));
    return DG_OK;
  };
  const uint32_t nchunks = (S + C - 1) / C;
  std::memset(s->host_live, 0xFF, ((size_t)S + 1) * 4);
  DG_HIP(hipEventRecord(s->ev_start, s->own));
  dg_status st = enqueue(0);
  if (st != DG_OK) return st;
  uint32_t launched = 1;
  if (nchunks > 1) {
    if ((st = enqueue(1)) != DG_OK) return st;
    launched = 2;
  }
  converged = false;
  uint32_t polled = 0;
  for (;;) {
    DG_HIP(hipEventSynchronize(s->ev_chunk[polled & 1]));
    ++polled;
    const uint32_t k_end = std::min(C * polled, S);
    const uint32_t live = __atomic_load_n(s->host_live + k_end, __ATOMIC_ACQUIRE);
    if (live == 0) {
      converged = true;
      break;
    }
    if (polled >= nchunks) break;
    if (launched < nchunks) {
      // the event slot is reused: the chunk it belonged to has been polled
      if ((st = enqueue(launched)) != DG_OK) return st;
      ++launched;
    }
  }
  DG_HIP(hipStreamSynchronize(s->own));
  float ms = 0.f;
  DG_HIP(hipEventElapsedTime(&ms, s->ev_start, s->ev_chunk[(polled - 1) & 1]));
  seconds = ms * 1e-3;
  chunks_run = polled;
  return DG_OK;
}

template <typename T>
void append_key(std::vector<unsigned char>& key, const T& v) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
  key.insert(key.end(), p, p + sizeof(T));
}

dg_status set_check_mode(dg_mode mode, uint32_t d, uint32_t max_sweeps) {
  if (mode != DG_SYNC && mode != DG_ASYNC && mode != DG_DELAYED)
    return fail(DG_ERR_INVALID_ARGUMENT, "mode %d is not DG_SYNC, DG_ASYNC or DG_DELAYED", (int)mode);
  if (mode == DG_DELAYED && d == 0) return fail(DG_ERR_INVALID_ARGUMENT, "delayed mode needs d >= 1");
  if (max_sweeps < 1 || max_sweeps > kSetMaxSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps = %u outside [1, %u]", max_sweeps, kSetMaxSweeps);
  return DG_OK;
}

// Enter the call's stream order: s->own waits for work already queued on the
// caller's stream.
dg_status enter(dg_set* s, void* hip_stream) {
  DG_HIP(hipEventRecord(s->ev_in, static_cast<hipStream_t>(hip_stream)));
  DG_HIP(hipStreamWaitEvent(s->own, s->ev_in, 0));
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_set_create(uint32_t count, const dg_graph_desc* graphs, const dg_set_opts* opts, void* hip_stream,
                        dg_set** out) {
  g_last_error.clear();
  if (!out) return fail(DG_ERR_INVALID_ARGUMENT, "out is NULL");
  if (count == 0 || !graphs) return fail(DG_ERR_INVALID_ARGUMENT, "a set needs at least one graph");
  uint64_t N = 0, M = 0;
  int weighted = -1;
  for (uint32_t i = 0; i < count; ++i) {
    const dg_graph_desc& d = graphs[i];
    if (d.n == 0) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u has no vertices", i);
    if (!d.ptr || (d.m > 0 && !d.idx)) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u: NULL ptr or idx", i);
    if (d.ptr[0] != 0 || d.ptr[d.n] != d.m)
      return fail(DG_ERR_INVALID_ARGUMENT, "graph %u: ptr[0] must be 0 and ptr[n] = m", i);
    for (uint32_t v = 0; v < d.n; ++v)
      if (d.ptr[v + 1] < d.ptr[v]) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u: ptr decreases at %u", i, v);
    for (uint64_t e = 0; e < d.m; ++e)
      if (d.idx[e] >= d.n) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u: idx[%llu] >= n", i, (unsigned long long)e);
    const int wi = d.w != nullptr;
    if (weighted >= 0 && wi != weighted)
      return fail(DG_ERR_INVALID_ARGUMENT, "either every graph of a set has weights or none has");
    weighted = wi;
    N += d.n;
    M += d.m;
  }
  if (N >= (1ull << 31)) return fail(DG_ERR_INVALID_ARGUMENT, "the set has %llu vertices (limit 2^31)",
                                     (unsigned long long)N);
  if (M + kEdgePad >= (1ull << 32))
    return fail(DG_ERR_INVALID_ARGUMENT, "the set has %llu edges (limit 2^32 - %u)", (unsigned long long)M,
                kEdgePad);

  dg_set* s = new (std::nothrow) dg_set;
  if (!s) return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
  dg::host::current_allocator(s->alloc, s->free_fn, s->ctx);
  s->G = count;
  s->N = (uint32_t)N;
  s->M = M;
  s->has_w = weighted == 1;

  std::vector<uint32_t> in_ptr, in_src, in_w, out_deg, tile_v, tile_g, g_toff;
  std::vector<double> dang0(count);
  try {
    s->voff.assign(count + 1, 0);
    s->gm.assign(count, 0);
    for (uint32_t i = 0; i < count; ++i) {
      s->voff[i + 1] = s->voff[i] + graphs[i].n;
      s->gm[i] = graphs[i].m;
    }
    in_ptr.assign((size_t)N + 1, 0);
    in_src.assign((size_t)M + kEdgePad, 0);
    if (s->has_w) in_w.assign((size_t)M + kEdgePad, 0);
    out_deg.assign(N, 0);
    for (uint32_t i = 0; i < count; ++i) {
      const dg_graph_desc& d = graphs[i];
      const uint32_t o = s->voff[i];
      uint32_t dangling = 0;
      for (uint32_t u = 0; u < d.n; ++u) {
        out_deg[o + u] = (uint32_t)(d.ptr[u + 1] - d.ptr[u]);
        dangling += out_deg[o + u] == 0;
      }
      dang0[i] = (double)dangling / (double)d.n;
      for (uint64_t e = 0; e < d.m; ++e) ++in_ptr[(size_t)o + d.idx[e] + 1];
    }
    for (uint64_t v = 0; v < N; ++v) in_ptr[v + 1] += in_ptr[v];
    std::vector<uint32_t> pos(in_ptr.begin(), in_ptr.end() - 1);
    for (uint32_t i = 0; i < count; ++i) {
      const dg_graph_desc& d = graphs[i];
      const uint32_t o = s->voff[i];
      for (uint32_t u = 0; u < d.n; ++u)
        for (uint64_t e = d.ptr[u]; e < d.ptr[u + 1]; ++e) {
          const uint32_t p = pos[o + d.idx[e]]++;
          in_src[p] = o + u;
          if (s->has_w) in_w[p] = d.w[e];
        }
    }
    // tiles per graph, so that none spans two graphs
    tile_v.push_back(0);
    g_toff.push_back(0);
    std::vector<uint32_t> local, lt;
    for (uint32_t i = 0; i < count; ++i) {
      const uint32_t o = s->voff[i], n = graphs[i].n;
      local.assign(in_ptr.begin() + o, in_ptr.begin() + o + n + 1);
      dg::host::build_tiles(local, n, lt);
      for (size_t t = 1; t < lt.size(); ++t) {
        tile_v.push_back(o + lt[t]);
        tile_g.push_back(i);
      }
      g_toff.push_back((uint32_t)tile_g.size());
    }
  } catch (const std::bad_alloc&) {
    delete s;
    return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed while building the set");
  }
  s->T = (uint32_t)tile_g.size();

  int dev = 0, cus = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventCreate(&s->ev_start);
  if (he == hipSuccess) he = hipEventCreate(&s->ev_chunk[0]);
  if (he == hipSuccess) he = hipEventCreate(&s->ev_chunk[1]);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    set_release(s);
    delete s;
    return fail(DG_ERR_DEVICE, "no usable HIP device: %s", hipGetErrorString(he));
  }
  s->cus = (uint32_t)cus;
  const uint32_t want = opts ? opts->workers : 0u;
  s->P = std::max(1u, std::min(want ? want : s->cus * kSetWorkersPerCU, s->T));

  if (enter(s, hip_stream) != DG_OK) {
    set_release(s);
    delete s;
    return DG_ERR_DEVICE;
  }
  struct Up {
    void** dst;
    const void* src;
    size_t bytes;
  } ups[] = {{(void**)&s->in_ptr, in_ptr.data(), in_ptr.size() * 4},
             {(void**)&s->in_src, in_src.data(), in_src.size() * 4},
             {(void**)&s->in_w, in_w.data(), in_w.size() * 4},
             {(void**)&s->out_deg, out_deg.data(), out_deg.size() * 4},
             {(void**)&s->tile_v, tile_v.data(), tile_v.size() * 4},
             {(void**)&s->tile_g, tile_g.data(), tile_g.size() * 4},
             {(void**)&s->g_voff, s->voff.data(), s->voff.size() * 4},
             {(void**)&s->g_toff, g_toff.data(), g_toff.size() * 4},
             {(void**)&s->dang0, dang0.data(), dang0.size() * 8}};
  for (auto& u : ups) {
    if (u.bytes == 0) continue;
    *u.dst = set_alloc(s, u.bytes);
    if (!*u.dst) {
      (void)hipStreamSynchronize(s->own);
      set_release(s);
      delete s;
      return fail(DG_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes failed", u.bytes);
    }
    s->bytes += u.bytes;
    he = hipMemcpyAsync(*u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s->own);
    if (he != hipSuccess) break;
  }
  if (he == hipSuccess) he = hipStreamSynchronize(s->own);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    set_release(s);
    delete s;
    return fail(DG_ERR_DEVICE, "set upload failed: %s", hipGetErrorString(he));
  }
  *out = s;
  return DG_OK;
}

dg_status dg_set_destroy(dg_set* s) {
  if (!s) return DG_OK;
  if (s->own) (void)hipStreamSynchronize(s->own);
  set_release(s);
  delete s;
  return DG_OK;
}

dg_status dg_set_info_get(const dg_set* s, dg_set_info* info) {
  if (!s || !info) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  info->graphs = s->G;
  info->n = s->N;
  info->m = s->M;
  info->tiles = s->T;
  info->workers = s->P;
  info->has_weights = s->has_w ? 1u : 0u;
  info->device_bytes = s->bytes;
  return DG_OK;
}

dg_status dg_set_pagerank(dg_set* s, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                          uint32_t max_sweeps, uint32_t flags, double* out_scores, int out_on_device,
                          uint32_t* out_sweeps, dg_stats* stats, void* hip_stream) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "set is NULL");
  if (!out_scores) return fail(DG_ERR_INVALID_ARGUMENT, "out_scores is NULL");
  if (!(damping >= 0.0 && damping < 1.0)) return fail(DG_ERR_INVALID_ARGUMENT, "damping must be in [0, 1)");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and >= 0");
  if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "dtype must be DG_F32 or DG_F64");
  if (flags & ~(uint32_t)DG_SET_EAGER) return fail(DG_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
  dg_status st = set_check_mode(mode, d, max_sweeps);
  if (st != DG_OK) return st;
  if (!kSetSweepsEnabled) return fail(DG_ERR_UNSUPPORTED, "set sweeps are switched off in this build");
  if ((st = set_workspace(s, max_sweeps)) != DG_OK) return st;
  if ((st = enter(s, hip_stream)) != DG_OK) return st;
  const bool f64 = dtype == DG_F64;
  SetPrArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: the bytes identify the captured chunk
  a.g = set_topo(s);
  a.c = set_ctl(s, max_sweeps);
  a.c0 = s->vals[0];
  a.c1 = mode == DG_SYNC ? s->vals[1] : nullptr;
  a.x = s->vals[2];
  a.shadow = mode == DG_DELAYED ? s->vals[3] : nullptr;
  a.tpart = s->tpart;
  a.gdang = s->gdang;
  a.gres = s->gres;
  a.alpha = damping;
  a.tol = tol;
  a.d = mode == DG_DELAYED ? d : 0u;
  DG_HIP(launch_set_pr_init(f64, a, s->dang0, s->own));
  std::vector<unsigned char> key;
  append_key(key, 1);
  append_key(key, (int)mode);
  append_key(key, f64);
  append_key(key, a);
  uint32_t chunks = 0;
  double secs = 0.0;
  bool conv = false;
  st = run_chunks(s, max_sweeps, (flags & DG_SET_EAGER) != 0, key,
                  [&](hipStream_t q) { return launch_set_pr_sweep((int)mode, f64, a, q); }, chunks, secs, conv);
  if (st != DG_OK) return st;
  double* outd = out_scores;
  void* tmp = nullptr;
  if (!out_on_device) {
    tmp = set_alloc(s, (size_t)s->N * 8);
    if (!tmp) return fail(DG_ERR_OUT_OF_MEMORY, "output staging allocation failed");
    outd = static_cast<double*>(tmp);
  }
  std::vector<uint32_t> gs(s->G);
  hipError_t e = launch_set_pr_out(f64, a, outd, s->own);
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(out_scores, outd, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->own);
  if (e == hipSuccess) e = hipMemcpyAsync(gs.data(), s->gdone, (size_t)s->G * 4, hipMemcpyDeviceToHost, s->own);
  if (e == hipSuccess) e = hipStreamSynchronize(s->own);
  if (tmp) set_free(s, tmp);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "set PageRank output failed: %s", hipGetErrorString(e));
  }
  uint32_t most = 0;
  uint64_t edges = 0;
  for (uint32_t i = 0; i < s->G; ++i) {
    const uint32_t sw = gs[i] ? gs[i] : max_sweeps;
    most = std::max(most, sw);
    edges += s->gm[i] * sw;
    if (out_sweeps) out_sweeps[i] = gs[i];
  }
  if (stats) {
    stats->sweeps = most;
    stats->workers = s->P;
    stats->tile_vertices = kTileV;
    stats->commit_interval = a.d;
    stats->residual = 0.0;
    stats->seconds = secs;
    stats->edges_traversed = edges;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "some graphs did not converge within %u sweeps", max_sweeps);
  return DG_OK;
}

dg_status dg_set_sssp(dg_set* s, const uint32_t* sources, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                      uint32_t flags, uint32_t* out_dist, int out_on_device, uint32_t* out_sweeps, dg_stats* stats,
                      void* hip_stream) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "set is NULL");
  if (!s->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "the set was created without weights");
  if (!sources || !out_dist) return fail(DG_ERR_INVALID_ARGUMENT, "NULL sources or out_dist");
  if (flags & ~(uint32_t)DG_SET_EAGER) return fail(DG_ERR_INVALID_ARGUMENT, "unknown flags 0x%x", flags);
  for (uint32_t i = 0; i < s->G; ++i)
    if (sources[i] >= s->voff[i + 1] - s->voff[i])
      return fail(DG_ERR_INVALID_ARGUMENT, "source %u of graph %u is not a vertex of it", sources[i], i);
  dg_status st = set_check_mode(mode, d, max_sweeps);
  if (st != DG_OK) return st;
  if (!kSetSweepsEnabled) return fail(DG_ERR_UNSUPPORTED, "set sweeps are switched off in this build");
  if ((st = set_workspace(s, max_sweeps)) != DG_OK) return st;
  if ((st = enter(s, hip_stream)) != DG_OK) return st;
  std::vector<uint32_t> usrc(s->G);
  for (uint32_t i = 0; i < s->G; ++i) usrc[i] = s->voff[i] + sources[i];
  DG_HIP(hipMemcpyAsync(s->srcd, usrc.data(), (size_t)s->G * 4, hipMemcpyHostToDevice, s->own));
  SetBfArgs a;
  std::memset(&a, 0, sizeof a);
  a.g = set_topo(s);
  a.c = set_ctl(s, max_sweeps);
  a.c0 = static_cast<uint32_t*>(s->vals[0]);
  a.c1 = mode == DG_SYNC ? static_cast<uint32_t*>(s->vals[1]) : nullptr;
  a.shadow = mode == DG_DELAYED ? static_cast<uint32_t*>(s->vals[3]) : nullptr;
  a.tchg = s->tchg;
  a.d = mode == DG_DELAYED ? d : 0u;
  DG_HIP(launch_set_bf_init(a, s->srcd, s->own));
  std::vector<unsigned char> key;
  append_key(key, 2);
  append_key(key, (int)mode);
  append_key(key, a);
  uint32_t chunks = 0;
  double secs = 0.0;
  bool conv = false;
  st = run_chunks(s, max_sweeps, (flags & DG_SET_EAGER) != 0, key,
                  [&](hipStream_t q) { return launch_set_bf_sweep((int)mode, a, q); }, chunks, secs, conv);
  if (st != DG_OK) return st;
  uint32_t* outd = out_dist;
  void* tmp = nullptr;
  if (!out_on_device) {
    tmp = set_alloc(s, (size_t)s->N * 4);
    if (!tmp) return fail(DG_ERR_OUT_OF_MEMORY, "output staging allocation failed");
    outd = static_cast<uint32_t*>(tmp);
  }
  const uint32_t last_k = std::min(chunks * kSetChunk, max_sweeps) - 1;
  std::vector<uint32_t> gs(s->G);
  hipError_t e = launch_set_bf_out((int)mode, a, last_k, outd, s->own);
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(out_dist, outd, (size_t)s->N * 4, hipMemcpyDeviceToHost, s->own);
  if (e == hipSuccess) e = hipMemcpyAsync(gs.data(), s->gdone, (size_t)s->G * 4, hipMemcpyDeviceToHost, s->own);
  if (e == hipSuccess) e = hipStreamSynchronize(s->own);
  if (tmp) set_free(s, tmp);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "set SSSP output failed: %s", hipGetErrorString(e));
  }
  uint32_t most = 0;
  uint64_t edges = 0;
  for (uint32_t i = 0; i < s->G; ++i) {
    const uint32_t sw = gs[i] ? gs[i] : max_sweeps;
    most = std::max(most, sw);
    edges += s->gm[i] * sw;
    if (out_sweeps) out_sweeps[i] = gs[i];
  }
  if (stats) {
    stats->sweeps = most;
    stats->workers = s->P;
    stats->tile_vertices = kTileV;
    stats->commit_interval = a.d;
    stats->residual = 0.0;
    stats->seconds = secs;
    stats->edges_traversed = edges;
  }
  if (!conv) return fail(DG_ERR_NOT_CONVERGED, "some graphs did not converge within %u sweeps", max_sweeps);
  return DG_OK;
}

}  // extern "C"

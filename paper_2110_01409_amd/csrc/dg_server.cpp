// Host side of the serving loop (dg_server_*): resident graphs, a queue of
// requests per (graph, query kind), and continuous batching.  Each pool of a
// (graph, kind) owns batches of 64 lanes swept by the batched kernels in
// serving mode; at every sweep boundary of the pool queued requests take free
// lanes (a lane is initialised for its source while the others keep
// running), finished lanes hand their row to the request and become free, and
// the pool grows by one batch when it has no free lane and the state budget
// allows.  Pools run on streams of their own and advance independently, so a
// small graph's queries are not paced by a large graph's sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "dg.h"
#include "dg_graph.hpp"
#include "dg_host.hpp"
#include "dg_internal.hpp"

using namespace dg;
using dg::host::dev_alloc;
using dg::host::dev_free;
using dg::host::fail;
using dg::host::g_last_error;
using dg::host::topo;
using dg::host::topo_batch;
using dg::host::kBatchSssp;
using dg::host::kBatchPpr;

namespace {

constexpr uint32_t kLanes = 64;
constexpr uint32_t kNone = 0xFFFFFFFFu;

struct Pool {
  dg_graph* g = nullptr;
  int kind = 0;
  uint32_t NB = 0;     // batches allocated
  uint32_t k = 0;      // sweeps run (ring parity, double-buffer parity)
  size_t per_batch = 0;
  // SSSP: distances (two buffers when synchronous), delayed staging, per-lane change flags
  uint32_t *b0 = nullptr, *b1 = nullptr, *sh = nullptr, *lchg = nullptr;
  // PPR: scores, contributions, staging, per-lane scalars, partials, worker counter ring
  void *x = nullptr, *c0 = nullptr, *c1 = nullptr, *psh = nullptr;
  uint32_t *src = nullptr, *qdone = nullptr, *count = nullptr;
  double *dang = nullptr, *scale = nullptr, *part = nullptr;
  uint32_t part_P = 0;      // batched workers `part` was sized for
  double* rhist = nullptr;  // float32 storage: [2][NB][64] changes two sweeps back (stall rule)
  // both kinds
  uint32_t *bactive = nullptr, *lane_src = nullptr, *blist = nullptr;
  uint32_t* flags_h = nullptr;  // pinned [NB * 64] readback
  hipStream_t st = nullptr;     // the pool's stream
  hipEvent_t ev = nullptr;      // recorded after a sweep's readback
  bool inflight = false;        // a sweep was launched and not yet retired
  uint64_t launched_at = 0;     // launch order (the oldest is waited for)
  double* qpart = nullptr;      // [256] normalisation partials (PPR)
  std::vector<int64_t> lane_req;  // request id in each lane, -1 if free
  std::vector<uint32_t> lane_k0;  // pool sweep count when the lane was admitted
  std::deque<uint64_t> queue;
};

struct Req {
  uint32_t graph = 0;
  dg_query kind = DG_QUERY_SSSP;
  uint32_t source = 0;
  uint64_t submit_step = 0, admit_step = 0, finish_step = 0;
  uint32_t sweeps = 0;
  int state = 0;  // 0 queued, 1 running, 2 finished, 3 fetched
  void* result = nullptr;
};

}  // namespace

struct dg_server {
  std::vector<dg_graph*> graphs;
  dg_server_opts o{};
  hipStream_t s = nullptr;
  std::vector<Pool> pools;  // index 2 * graph + kind
  std::vector<Req> reqs;    // index id - 1
  std::deque<uint64_t> finished;
  uint64_t steps = 0, state_bytes = 0, launches = 0;
  int64_t starved = -1;  // pool that has queued requests but no batch and no budget, else -1
};

namespace {

bool f64(const dg_server* s) { return s->o.dtype == DG_F64; }

// The graph's batched partition for a pool of this kind.
int batch_part(int kind) { return kind == DG_QUERY_SSSP ? kBatchSssp : kBatchPpr; }

// Commit interval of a pool's delayed sweeps: d, at most a worker's block.
uint32_t pool_d(const dg_server* s, const dg_graph* g, int kind) {
  return std::max(1u, std::min(s->o.d, g->bp[batch_part(kind)].max_block_v));
}

// Delayed commits stage per wavefront in LDS up to kLdsStageMaxD, and need
// the per-batch shadow array only beyond.
bool delayed_shadow(const dg_server* s, const dg_graph* g, int kind) {
  return s->o.mode == DG_DELAYED && pool_d(s, g, kind) > kLdsStageMaxD;
}

size_t batch_bytes(const dg_server* s, const dg_graph* g, int kind) {
  const size_t n = g->n, slots = (size_t)g->n + g->K;
  const bool sync = s->o.mode == DG_SYNC;
  if (kind == DG_QUERY_SSSP)
    return (slots * (sync ? 2 : 1) + (delayed_shadow(s, g, kind) ? n : 0)) * kLanes * 4 + kLanes * 8 + 16;
  const size_t e = f64(s) ? 8 : 4;
  return (n + slots * (sync ? 2 : 1) + (delayed_shadow(s, g, kind) ? n : 0)) * kLanes * e + kLanes * (4 + 4 + 6 * 8 + 4) +
         (size_t)g->bp[kBatchPpr].P * 3 * kLanes * 8 + 16;
}

void free_pool(Pool& p) {
  for (void* q : {(void*)p.b0, (void*)p.b1, (void*)p.sh, (void*)p.lchg, p.x, p.c0, p.c1, p.psh, (void*)p.src,
                  (void*)p.qdone, (void*)p.count, (void*)p.dang, (void*)p.scale, (void*)p.rhist, (void*)p.part,
                  (void*)p.bactive,
                  (void*)p.lane_src, (void*)p.blist})
    dev_free(p.g, q);
  if (p.flags_h) (void)hipHostFree(p.flags_h);
  p.flags_h = nullptr;
  dev_free(p.g, p.qpart);
  p.qpart = nullptr;
  if (p.ev) (void)hipEventDestroy(p.ev);
  if (p.st) (void)hipStreamDestroy(p.st);
  p.ev = nullptr;
  p.st = nullptr;
}

// Re-allocates a [NB] x stride array for NBn batches, keeping the first
// min(NB, NBn) batches (none when copy is false); NBn = 0 frees it.
template <typename T>
dg_status reshape(Pool& p, T*& arr, size_t stride_bytes, uint32_t NBn, bool copy) {
  T* na = nullptr;
  if (NBn) {
    na = static_cast<T*>(dev_alloc(p.g, (size_t)NBn * stride_bytes, p.st));
    if (!na) return fail(DG_ERR_OUT_OF_MEMORY, "serving state allocation failed");
    const size_t keep = (size_t)std::min(p.NB, NBn) * stride_bytes;
    if (arr && copy && keep) DG_HIP(hipMemcpyAsync(na, arr, keep, hipMemcpyDeviceToDevice, p.st));
  }
  dev_free(p.g, arr);
  arr = na;
  return DG_OK;
}

// The same for a [2][NB] x stride ring (both slots keep their batches).
template <typename T>
dg_status reshape_ring(Pool& p, T*& arr, size_t stride_bytes, uint32_t NBn) {
  T* na = nullptr;
  if (NBn) {
    na = static_cast<T*>(dev_alloc(p.g, 2 * (size_t)NBn * stride_bytes, p.st));
    if (!na) return fail(DG_ERR_OUT_OF_MEMORY, "serving state allocation failed");
    const size_t keep = (size_t)std::min(p.NB, NBn) * stride_bytes;
    if (arr && keep) {
      auto* src = reinterpret_cast<unsigned char*>(arr);
      auto* dst = reinterpret_cast<unsigned char*>(na);
      DG_HIP(hipMemcpyAsync(dst, src, keep, hipMemcpyDeviceToDevice, p.st));
      DG_HIP(hipMemcpyAsync(dst + (size_t)NBn * stride_bytes, src + (size_t)p.NB * stride_bytes, keep,
                            hipMemcpyDeviceToDevice, p.st));
    }
  }
  dev_free(p.g, arr);
  arr = na;
  return DG_OK;
}

// Resizes a pool to NBn batches of 64 lanes.  Growing adds free lanes;
// shrinking drops trailing batches, whose lanes must all be free (0 releases
// the pool's whole state).  The budget account follows.
dg_status resize(dg_server* s, Pool& p, uint32_t NBn) {
  dg_graph* g = p.g;
  const size_t n = g->n, slots = (size_t)g->n + g->K;
  const bool sync = s->o.mode == DG_SYNC;
  dg_status st;
  if (!p.st) {
    DG_HIP(hipStreamCreateWithFlags(&p.st, hipStreamNonBlocking));
    DG_HIP(hipEventCreateWithFlags(&p.ev, hipEventDisableTiming));
    p.qpart = static_cast<double*>(dev_alloc(g, 256 * 8, p.st));
    if (!p.qpart) return fail(DG_ERR_OUT_OF_MEMORY, "serving state allocation failed");
  }
  if (p.kind == DG_QUERY_SSSP) {
    if ((st = reshape(p, p.b0, slots * kLanes * 4, NBn, true)) != DG_OK) return st;
    if (sync && (st = reshape(p, p.b1, slots * kLanes * 4, NBn, true)) != DG_OK) return st;
    if (delayed_shadow(s, g, p.kind) && (st = reshape(p, p.sh, n * kLanes * 4, NBn, false)) != DG_OK) return st;
    if ((st = reshape(p, p.lchg, kLanes * 4, NBn, false)) != DG_OK) return st;
  } else {
    const size_t e = f64(s) ? 8 : 4;
    if ((st = reshape(p, p.x, n * kLanes * e, NBn, true)) != DG_OK) return st;
    if ((st = reshape(p, p.c0, slots * kLanes * e, NBn, true)) != DG_OK) return st;
    if (sync && (st = reshape(p, p.c1, slots * kLanes * e, NBn, true)) != DG_OK) return st;
    if (delayed_shadow(s, g, p.kind) && (st = reshape(p, p.psh, n * kLanes * e, NBn, false)) != DG_OK) return st;
    if ((st = reshape(p, p.src, kLanes * 4, NBn, true)) != DG_OK) return st;
    if ((st = reshape(p, p.qdone, kLanes * 4, NBn, true)) != DG_OK) return st;
    if ((st = reshape_ring(p, p.dang, kLanes * 8, NBn)) != DG_OK) return st;
    if ((st = reshape_ring(p, p.scale, kLanes * 8, NBn)) != DG_OK) return st;
    if (!f64(s) && (st = reshape_ring(p, p.rhist, kLanes * 8, NBn)) != DG_OK) return st;
    if ((st = reshape_ring(p, p.count, 4, NBn)) != DG_OK) return st;
    p.part_P = g->bp[kBatchPpr].P;
    if ((st = reshape(p, p.part, (size_t)p.part_P * 3 * kLanes * 8, NBn, false)) != DG_OK) return st;
    // new batches: lanes frozen and unassigned
    for (uint32_t b = p.NB; b < NBn; ++b) {
      DG_HIP(launch_fill_u32(p.qdone + (size_t)b * kLanes, kLanes, 1u, p.st));
      DG_HIP(launch_fill_u32(p.src + (size_t)b * kLanes, kLanes, kInf, p.st));
      DG_HIP(launch_fill_f64(p.scale + (size_t)b * kLanes, kLanes, 1.0, p.st));
      DG_HIP(launch_fill_f64(p.scale + (size_t)(NBn + b) * kLanes, kLanes, 1.0, p.st));
      DG_HIP(launch_fill_f64(p.dang + (size_t)b * kLanes, kLanes, 0.0, p.st));
      DG_HIP(launch_fill_f64(p.dang + (size_t)(NBn + b) * kLanes, kLanes, 0.0, p.st));
      if (p.rhist) {
        DG_HIP(launch_fill_f64(p.rhist + (size_t)b * kLanes, kLanes, __builtin_inf(), p.st));
        DG_HIP(launch_fill_f64(p.rhist + (size_t)(NBn + b) * kLanes, kLanes, __builtin_inf(), p.st));
      }
    }
  }
  if ((st = reshape(p, p.bactive, 4, NBn, false)) != DG_OK) return st;
  if ((st = reshape(p, p.lane_src, kLanes * 4, NBn, false)) != DG_OK) return st;
  if ((st = reshape(p, p.blist, 4, NBn, false)) != DG_OK) return st;
  DG_HIP(hipStreamSynchronize(p.st));  // copies done before the old arrays' memory is reused
  if (p.flags_h) (void)hipHostFree(p.flags_h);
  p.flags_h = nullptr;
  if (NBn) DG_HIP(hipHostMalloc((void**)&p.flags_h, (size_t)NBn * kLanes * 4, hipHostMallocDefault));
  s->state_bytes = s->state_bytes + (size_t)NBn * p.per_batch - (size_t)p.NB * p.per_batch;
  p.NB = NBn;
  p.lane_req.resize((size_t)NBn * kLanes, -1);
  p.lane_k0.resize((size_t)NBn * kLanes, 0);
  return DG_OK;
}

bool budget_allows(const dg_server* s, const Pool& p) {
  if (s->o.max_batches && p.NB >= s->o.max_batches) return false;
  return !s->o.hbm_budget || s->state_bytes + p.per_batch <= s->o.hbm_budget;
}

bool lanes_free(const Pool& p, uint32_t b) {
  for (uint32_t i = 0; i < kLanes; ++i)
    if (p.lane_req[(size_t)b * kLanes + i] >= 0) return false;
  return true;
}

// While a pool starves (queued requests, no batch, no budget), only it may grow.
bool can_grow(const dg_server* s, const Pool& p) {
  if (s->starved >= 0 && &s->pools[(size_t)s->starved] != &p) return false;
  return budget_allows(s, p);
}

// Admission, one sweep and retirement for one pool.  Returns the number of
// lanes that ran (0 = nothing to do).
dg_status pool_sweep(dg_server* s, Pool& p, bool& ran) {
  ran = false;
  dg_graph* g = p.g;
  // admission: queued requests take free lanes, the pool grows if it may
  std::vector<uint32_t> lane_src;
  std::vector<uint32_t> blist;
  size_t cursor = 0;
  // while another pool starves, every other pool keeps its last batch free
  // of new queries so that it can be released (a pool of one batch then
  // drains and, if requests still wait, starves in turn: the pool of the
  // oldest waiting request is served first)
  const bool donor = s->starved >= 0 && &s->pools[(size_t)s->starved] != &p && p.NB >= 1;
  while (!p.queue.empty()) {
    const size_t limit = donor ? (size_t)(p.NB - 1) * kLanes : p.lane_req.size();
    while (cursor < limit && p.lane_req[cursor] >= 0) ++cursor;
    if (cursor >= limit) {
      if (donor || !can_grow(s, p)) break;
      dg_status st = resize(s, p, p.NB + 1);
      if (st != DG_OK) return st;
    }
    const uint64_t id = p.queue.front();
    p.queue.pop_front();
    Req& r = s->reqs[id - 1];
    if (lane_src.empty() || lane_src.size() < p.lane_req.size()) lane_src.resize(p.lane_req.size(), kNone);
    lane_src[cursor] = r.source;
    p.lane_req[cursor] = (int64_t)id;
    p.lane_k0[cursor] = p.k;
    r.state = 1;
    r.admit_step = s->steps;
    const uint32_t b = (uint32_t)(cursor / kLanes);
    if (blist.empty() || blist.back() != b) blist.push_back(b);
  }
  std::vector<uint32_t> active(p.NB, 0);
  bool any = false;
  for (size_t i = 0; i < p.lane_req.size(); ++i)
    if (p.lane_req[i] >= 0) active[i / kLanes] = 1, any = true;
  if (!any) return DG_OK;
  hipStream_t q = p.st;
  const Topology t = topo_batch(g, batch_part(p.kind));
  if (!blist.empty()) {
    lane_src.resize((size_t)p.NB * kLanes, kNone);
    DG_HIP(hipMemcpyAsync(p.lane_src, lane_src.data(), lane_src.size() * 4, hipMemcpyHostToDevice, q));
    DG_HIP(hipMemcpyAsync(p.blist, blist.data(), blist.size() * 4, hipMemcpyHostToDevice, q));
    if (p.kind == DG_QUERY_SSSP)
      DG_HIP(launch_mbf_lane_init(p.b0, p.b1, g->cpos, g->n, g->K, p.lane_src, p.blist, (uint32_t)blist.size(), q));
    else
      DG_HIP(launch_mppr_lane_init(f64(s), p.x, p.c0, p.c1, g->out_deg, g->cpos, g->n, g->K, p.NB, p.lane_src,
                                   p.blist, (uint32_t)blist.size(), p.src, p.dang, p.scale, p.qdone, p.rhist, q));
  }
  DG_HIP(hipMemcpyAsync(p.bactive, active.data(), active.size() * 4, hipMemcpyHostToDevice, q));
  const bool sync = s->o.mode == DG_SYNC;
  if (p.kind == DG_QUERY_SSSP) {
    DG_HIP(launch_fill_u32(p.lchg, (size_t)p.NB * kLanes, 0u, q));
    MbfArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = t;
    a.din = sync && (p.k & 1u) ? p.b1 : p.b0;
    a.dout = sync ? ((p.k & 1u) ? p.b0 : p.b1) : p.b0;
    a.shadow = p.sh;
    a.lchg = p.lchg;
    a.bactive = p.bactive;
    a.k = p.k;
    a.d = s->o.mode == DG_DELAYED ? pool_d(s, g, p.kind) : 0u;
    a.NB = p.NB;
    DG_HIP(launch_mbf_sweep((int)s->o.mode, a, q));
    DG_HIP(hipMemcpyAsync(p.flags_h, p.lchg, (size_t)p.NB * kLanes * 4, hipMemcpyDeviceToHost, q));
  } else {
    if (p.part_P != t.P) {
      // the graph was re-partitioned (dg_tune_batch) since the partials were sized
      dg_status rs = reshape(p, p.part, (size_t)t.P * 3 * kLanes * 8, p.NB, false);
      if (rs != DG_OK) return rs;
      p.part_P = t.P;
    }
    DG_HIP(launch_fill_u32(p.count, 2 * (size_t)p.NB, 0u, q));
    MpprArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = t;
    a.cin = sync && (p.k & 1u) ? p.c1 : p.c0;
    a.cout = sync ? ((p.k & 1u) ? p.c0 : p.c1) : p.c0;
    a.x = p.x;
    a.shadow = p.psh;
    a.src = p.src;
    a.dang = p.dang;
    a.scale = p.scale;
    a.qdone = p.qdone;
    a.rhist = p.rhist;
    a.count = p.count;
    a.part = p.part;
    a.bactive = p.bactive;
    a.alpha = s->o.damping;
    a.tol = s->o.tol;
    a.nq = p.NB * kLanes;
    a.k = p.k;
    a.d = s->o.mode == DG_DELAYED ? pool_d(s, g, p.kind) : 0u;
    a.NB = p.NB;
    DG_HIP(launch_mppr_sweep((int)s->o.mode, f64(s), a, q));
    DG_HIP(hipMemcpyAsync(p.flags_h, p.qdone, (size_t)p.NB * kLanes * 4, hipMemcpyDeviceToHost, q));
  }
  ++p.k;
  ran = true;
  return DG_OK;
}

// After the step's sweeps: lanes whose query stopped hand over their rows.
dg_status pool_retire(dg_server* s, Pool& p) {
  dg_graph* g = p.g;
  for (size_t i = 0; i < p.lane_req.size(); ++i) {
    if (p.lane_req[i] < 0) continue;
    const bool done = p.kind == DG_QUERY_SSSP ? p.flags_h[i] == 0 : p.flags_h[i] != 0;
    if (!done) continue;
    const uint64_t id = (uint64_t)p.lane_req[i];
    Req& r = s->reqs[id - 1];
    const uint32_t b = (uint32_t)(i / kLanes), lane = (uint32_t)(i % kLanes);
    r.result = dev_alloc(g, (size_t)g->n * (p.kind == DG_QUERY_SSSP ? 4 : 8), p.st);
    if (!r.result) return fail(DG_ERR_OUT_OF_MEMORY, "result allocation failed");
    if (p.kind == DG_QUERY_SSSP) {
      // no distance changed in the last sweep, so both buffers hold the result
      DG_HIP(launch_mbf_lane_out(p.b0, g->cpos, g->n, g->K, b, lane, static_cast<uint32_t*>(r.result), p.st));
    } else {
      DG_HIP(launch_mppr_lane_out(f64(s), p.x, g->n, b, lane, p.qpart, static_cast<double*>(r.result), p.st));
    }
    r.state = 2;
    r.finish_step = s->steps;
    r.sweeps = p.k - p.lane_k0[i];
    p.lane_req[i] = -1;
    s->finished.push_back(id);
  }
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_server_create(dg_graph* const* graphs, uint32_t count, const dg_server_opts* opts, void* hip_stream,
                           dg_server** out) {
  g_last_error.clear();
  if (!out || !graphs || count == 0 || !opts) return fail(DG_ERR_INVALID_ARGUMENT, "NULL or empty argument");
  for (uint32_t i = 0; i < count; ++i)
    if (!graphs[i]) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u is NULL", i);
  if (opts->mode != DG_SYNC && opts->mode != DG_ASYNC && opts->mode != DG_DELAYED)
    return fail(DG_ERR_INVALID_ARGUMENT, "unknown mode %d", (int)opts->mode);
  if (opts->mode == DG_DELAYED && opts->d == 0) return fail(DG_ERR_INVALID_ARGUMENT, "delayed mode needs d >= 1");
  if (!(opts->damping >= 0.0 && opts->damping < 1.0)) return fail(DG_ERR_INVALID_ARGUMENT, "damping must be in [0, 1)");
  if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite, > 0");
  if (opts->dtype != DG_F32 && opts->dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "unknown dtype");
  dg_server* s = new (std::nothrow) dg_server;
  if (!s) return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->graphs.assign(graphs, graphs + count);
  s->o = *opts;
  s->s = static_cast<hipStream_t>(hip_stream);
  s->pools.resize(2 * (size_t)count);
  for (uint32_t i = 0; i < count; ++i)
    for (int kind = 0; kind < 2; ++kind) {
      Pool& p = s->pools[2 * i + kind];
      p.g = graphs[i];
      p.kind = kind;
      p.per_batch = batch_bytes(s, graphs[i], kind);
    }
  *out = s;
  return DG_OK;
}

dg_status dg_server_destroy(dg_server* s) {
  if (!s) return DG_OK;
  for (auto& p : s->pools)
    if (p.st) (void)hipStreamSynchronize(p.st);
  for (auto& r : s->reqs)
    if (r.result) dev_free(s->graphs[r.graph], r.result);
  for (auto& p : s->pools) free_pool(p);
  delete s;
  return DG_OK;
}

dg_status dg_server_submit(dg_server* s, uint32_t graph, dg_query kind, uint32_t source, uint64_t* out_id) {
  g_last_error.clear();
  if (!s || !out_id) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  if (graph >= s->graphs.size()) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u out of range", graph);
  if (kind != DG_QUERY_SSSP && kind != DG_QUERY_PPR) return fail(DG_ERR_INVALID_ARGUMENT, "unknown query kind");
  const dg_graph* g = s->graphs[graph];
  if (source >= g->n) return fail(DG_ERR_INVALID_ARGUMENT, "source %u >= n", source);
  if (kind == DG_QUERY_SSSP && !g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "graph %u has no weights", graph);
  Pool& p = s->pools[2 * (size_t)graph + kind];
  if (p.NB == 0 && s->o.hbm_budget && p.per_batch > s->o.hbm_budget)
    return fail(DG_ERR_OUT_OF_MEMORY, "the state budget is below one batch (%zu bytes)", p.per_batch);
  Req r;
  r.graph = graph;
  r.kind = kind;
  r.source = source;
  r.submit_step = s->steps;
  s->reqs.push_back(r);
  const uint64_t id = s->reqs.size();
  p.queue.push_back(id);
  *out_id = id;
  return DG_OK;
}

dg_status dg_server_step(dg_server* s, uint64_t* out_finished, uint32_t cap, uint32_t* out_count) {
  g_last_error.clear();
  if (!s || !out_count || (cap && !out_finished)) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  ++s->steps;
  // A pool whose sweep has finished retires its finished lanes; the rows are
  // complete when the extraction on its stream is.
  auto retire = [&](Pool& p) -> dg_status {
    dg_status st = pool_retire(s, p);
    if (st != DG_OK) return st;
    DG_HIP(hipStreamSynchronize(p.st));
    p.inflight = false;
    return DG_OK;
  };
  bool retired = false;
  for (auto& p : s->pools) {
    if (!p.inflight) continue;
    const hipError_t q = hipEventQuery(p.ev);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();  // not an error: keep it out of later launch checks
      continue;
    }
    DG_HIP(q);
    dg_status st = retire(p);
    if (st != DG_OK) return st;
    retired = true;
  }
  // Budget: a pool with nothing running and nothing queued releases its
  // state; a pool that has queued requests but no batch and no budget starves,
  // and then other pools do not grow and give up trailing batches that
  // emptied (their last one included), until it fits.
  for (auto& p : s->pools) {
    if (p.inflight || p.NB == 0 || !p.queue.empty()) continue;
    bool idle = true;
    for (int64_t r : p.lane_req) idle = idle && r < 0;
    if (idle) {
      dg_status st = resize(s, p, 0);
      if (st != DG_OK) return st;
    }
  }
  s->starved = -1;
  uint64_t oldest = ~0ull;
  for (size_t i = 0; i < s->pools.size(); ++i) {
    const Pool& p = s->pools[i];
    if (p.NB == 0 && !p.queue.empty() && !budget_allows(s, p) && p.queue.front() < oldest) {
      oldest = p.queue.front();
      s->starved = (int64_t)i;
    }
  }
  if (s->starved >= 0) {
    const Pool& hungry = s->pools[(size_t)s->starved];
    for (auto& p : s->pools) {
      if (budget_allows(s, hungry)) break;
      if (&p == &hungry) continue;
      while (!p.inflight && p.NB >= 1 && lanes_free(p, p.NB - 1) && !budget_allows(s, hungry)) {
        dg_status st = resize(s, p, p.NB - 1);
        if (st != DG_OK) return st;
      }
    }
  }
  // Every idle pool with work admits queued requests and starts its next sweep.
  auto launch = [&](Pool& p) -> dg_status {
    bool ran = false;
    dg_status st = pool_sweep(s, p, ran);
    if (st != DG_OK) return st;
    if (ran) {
      DG_HIP(hipEventRecord(p.ev, p.st));
      p.inflight = true;
      p.launched_at = ++s->launches;
    }
    return DG_OK;
  };
  for (auto& p : s->pools) {
    if (p.inflight) continue;
    dg_status st = launch(p);
    if (st != DG_OK) return st;
  }
  // Nothing retired in this call: wait for the oldest sweep, retire it and
  // start its pool's next one, so every call makes progress.
  if (!retired) {
    Pool* oldest = nullptr;
    for (auto& p : s->pools)
      if (p.inflight && (!oldest || p.launched_at < oldest->launched_at)) oldest = &p;
    if (oldest) {
      DG_HIP(hipEventSynchronize(oldest->ev));
      dg_status st = retire(*oldest);
      if (st == DG_OK) st = launch(*oldest);
      if (st != DG_OK) return st;
    }
  }
  uint32_t c = 0;
  while (c < cap && !s->finished.empty()) {
    out_finished[c++] = s->finished.front();
    s->finished.pop_front();
  }
  *out_count = c;
  return DG_OK;
}

dg_status dg_server_fetch(dg_server* s, uint64_t id, void* out, int out_on_device, dg_request_info* info) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "server is NULL");
  if (id == 0 || id > s->reqs.size()) return fail(DG_ERR_INVALID_ARGUMENT, "unknown request %llu",
                                                  (unsigned long long)id);
  Req& r = s->reqs[id - 1];
  if (info) {
    info->graph = r.graph;
    info->kind = r.kind;
    info->source = r.source;
    info->sweeps = r.sweeps;
    info->state = (uint32_t)r.state;
    info->submit_step = r.submit_step;
    info->admit_step = r.admit_step;
    info->finish_step = r.finish_step;
  }
  if (!out) return DG_OK;  // status only
  if (r.state != 2) return fail(DG_ERR_INVALID_ARGUMENT, "request %llu has no result to fetch (state %d)",
                                (unsigned long long)id, r.state);
  dg_graph* g = s->graphs[r.graph];
  const size_t bytes = (size_t)g->n * (r.kind == DG_QUERY_SSSP ? 4 : 8);
  DG_HIP(hipMemcpyAsync(out, r.result, bytes, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        s->s));
  DG_HIP(hipStreamSynchronize(s->s));
  dev_free(g, r.result);
  r.result = nullptr;
  r.state = 3;
  return DG_OK;
}

dg_status dg_server_status_get(const dg_server* s, dg_server_status* st) {
  if (!s || !st) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  std::memset(st, 0, sizeof *st);
  for (const auto& r : s->reqs) {
    st->queued += r.state == 0;
    st->running += r.state == 1;
    st->finished += r.state == 2;
  }
  for (const auto& p : s->pools) st->batches += p.NB;
  st->state_bytes = s->state_bytes;
  st->steps = s->steps;
  return DG_OK;
}

}  // extern "C"

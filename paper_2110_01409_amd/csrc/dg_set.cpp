// Host side of graph sets (dg_set_*): many graphs of uneven size resident as
// one union graph and swept together, one launch per sweep for all of them,
// by the single-graph kernels.
//
// Bellman-Ford: the union is swept from every graph's own source at once;
// no edge crosses two graphs, so each graph's distances are its own.
//
// PageRank: the union's PageRank, restricted to one graph and renormalised,
// is that graph's PageRank.  Inside graph g the union's fixed point reads
// x_v = alpha * (pulled) + c with the same constant c = ((1 - alpha) + alpha
// D) / N for every vertex, and g's mass balance M_g (1 - alpha) + alpha D_g =
// n_g ((1 - alpha) + alpha D) / N makes x / M_g solve g's own equation
// x_v = alpha * (pulled) + ((1 - alpha) + alpha D_g / M_g) / n_g.  Worker
// blocks never cross a graph boundary, so the sweep kernel sums each graph's
// L1 change and mass separately: a sweep's stopping value is the largest
// change over M_g, i.e. the largest change of a graph's normalised scores,
// and the set stops when every graph has met the single-graph rule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
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

struct dg_set {
  dg_graph* g = nullptr;       // the union graph
  uint32_t G = 0, n_min = 0;
  std::vector<uint32_t> voff;  // first vertex of each graph, and the total
  std::vector<uint64_t> gm;    // edges of each graph
  uint32_t* voff_d = nullptr;  // device copy of voff (allocated through g)
  uint32_t* src_d = nullptr;   // [G] device sources of an SSSP call
};

namespace {

// Float32 scores cannot settle below about 1e-7 of L1 change (their rounding).
constexpr double kF32Floor = 1e-7;

dg_status set_check_mode(dg_mode mode, uint32_t d, uint32_t max_sweeps) {
  if (mode != DG_SYNC && mode != DG_ASYNC && mode != DG_DELAYED)
    return fail(DG_ERR_INVALID_ARGUMENT, "mode %d is not DG_SYNC, DG_ASYNC or DG_DELAYED", (int)mode);
  if (mode == DG_DELAYED && d == 0) return fail(DG_ERR_INVALID_ARGUMENT, "delayed mode needs d >= 1");
  if (max_sweeps < 1 || max_sweeps > dg::host::kMaxSweeps)
    return fail(DG_ERR_INVALID_ARGUMENT, "max_sweeps = %u outside [1, %u]", max_sweeps, dg::host::kMaxSweeps);
  return DG_OK;
}

// The first sweep that took each graph below tol (PageRank) or in which it
// changed no distance (Bellman-Ford); 0: none within max_sweeps.
dg_status per_graph_sweeps(const dg_set* s, uint32_t* out_sweeps, hipStream_t q) {
  if (!out_sweeps) return DG_OK;
  DG_HIP(hipMemcpyAsync(out_sweeps, s->g->gsweeps, (size_t)s->G * 4, hipMemcpyDeviceToHost, q));
  DG_HIP(hipStreamSynchronize(q));
  return DG_OK;
}

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

constexpr uint32_t kSetTuneRepeats = 3;

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
  s->G = count;
  std::vector<uint64_t> ptr;
  std::vector<uint32_t> idx, w;
  try {
    s->voff.assign(count + 1, 0);
    s->gm.assign(count, 0);
    ptr.assign(N + 1, 0);
    idx.resize(M);
    if (weighted == 1) w.resize(M);
    uint64_t e0 = 0;
    s->n_min = 0xFFFFFFFFu;
    for (uint32_t i = 0; i < count; ++i) {
      const dg_graph_desc& d = graphs[i];
      const uint32_t o = s->voff[i];
      s->voff[i + 1] = o + d.n;
      s->gm[i] = d.m;
      s->n_min = std::min(s->n_min, d.n);
      for (uint32_t v = 0; v < d.n; ++v) ptr[(size_t)o + v + 1] = e0 + d.ptr[v + 1];
      for (uint64_t e = 0; e < d.m; ++e) idx[e0 + e] = o + d.idx[e];
      if (weighted == 1) std::copy(d.w, d.w + d.m, w.begin() + e0);
      e0 += d.m;
    }
  } catch (const std::bad_alloc&) {
    delete s;
    return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed while building the set");
  }
  dg_graph_opts go{};
  go.workers = opts ? opts->workers : 0u;
  go.hot_vertices = DG_HOT_AUTO;
  go.resident_vertices = DG_RESIDENT_AUTO;
  go.sweep_variant = DG_SWEEP_AUTO;
  dg_status st = dg::host::graph_create((uint32_t)N, M, DG_CSR, ptr.data(), M ? idx.data() : nullptr,
                                        weighted == 1 ? w.data() : nullptr, &go, &s->voff, hip_stream, &s->g);
  if (st != DG_OK) {
    delete s;
    return st;
  }
  hipStream_t q = static_cast<hipStream_t>(hip_stream);
  s->voff_d = static_cast<uint32_t*>(dev_alloc(s->g, (size_t)(count + 1) * 4, q));
  s->src_d = static_cast<uint32_t*>(dev_alloc(s->g, (size_t)count * 4, q));
  hipError_t he = (s->voff_d && s->src_d) ? hipSuccess : hipErrorOutOfMemory;
  if (he == hipSuccess)
    he = hipMemcpyAsync(s->voff_d, s->voff.data(), (size_t)(count + 1) * 4, hipMemcpyHostToDevice, q);
  if (he == hipSuccess) he = hipStreamSynchronize(q);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    dg_graph_destroy(s->g);
    delete s;
    return fail(he == hipErrorOutOfMemory ? DG_ERR_OUT_OF_MEMORY : DG_ERR_DEVICE, "set upload failed: %s",
                hipGetErrorString(he));
  }
  *out = s;
  return DG_OK;
}

dg_status dg_set_destroy(dg_set* s) {
  if (!s) return DG_OK;
  dg_graph_destroy(s->g);  // also frees voff_d and src_d
  delete s;
  return DG_OK;
}

dg_status dg_set_info_get(const dg_set* s, dg_set_info* info) {
  if (!s || !info) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  dg_graph_info gi;
  dg_status st = dg_graph_info_get(s->g, &gi);
  if (st != DG_OK) return st;
  info->graphs = s->G;
  info->n = gi.n;
  info->m = gi.m;
  info->tiles = gi.tiles;
  info->workers = gi.workers;
  info->has_weights = gi.has_weights;
  info->device_bytes = gi.device_bytes;
  return DG_OK;
}

dg_status dg_set_repartition(dg_set* s, uint32_t workers, void* hip_stream) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "set is NULL");
  return dg_graph_repartition(s->g, workers, hip_stream);
}

dg_status dg_set_tune(dg_set* s, dg_algo algo, dg_dtype dtype, double tol, const uint32_t* sources, uint32_t flags,
                      dg_tuning* out, void* hip_stream) {
  g_last_error.clear();
  if (!s || !out) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  if (algo != DG_ALGO_PAGERANK && algo != DG_ALGO_SSSP) return fail(DG_ERR_INVALID_ARGUMENT, "unknown algorithm");
  if (flags != 0) return fail(DG_ERR_INVALID_ARGUMENT, "flags must be 0 (got 0x%x)", flags);
  if (algo == DG_ALGO_PAGERANK) {
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(DG_ERR_INVALID_ARGUMENT, "tol must be finite and > 0");
    if (dtype != DG_F32 && dtype != DG_F64) return fail(DG_ERR_INVALID_ARGUMENT, "dtype must be DG_F32 or DG_F64");
    if (dtype == DG_F32 && tol < kF32Floor)
      return fail(DG_ERR_UNSUPPORTED, "float32 scores cannot settle below an L1 change of %.0e", kF32Floor);
  } else {
    if (!s->g->has_w) return fail(DG_ERR_INVALID_ARGUMENT, "the set was created without weights");
    if (!sources) return fail(DG_ERR_INVALID_ARGUMENT, "sources is NULL");
    for (uint32_t i = 0; i < s->G; ++i)
      if (sources[i] >= s->voff[i + 1] - s->voff[i])
        return fail(DG_ERR_INVALID_ARGUMENT, "source %u of graph %u is not a vertex of it", sources[i], i);
  }
  hipStream_t q = static_cast<hipStream_t>(hip_stream);
  const uint32_t N = s->voff.back();
  void* outd = dev_alloc(s->g, (size_t)N * (algo == DG_ALGO_PAGERANK ? 8 : 4), q);
  if (!outd) return fail(DG_ERR_OUT_OF_MEMORY, "tuning output allocation failed");
  uint32_t n_max = 0;
  for (uint32_t i = 0; i < s->G; ++i) n_max = std::max(n_max, s->voff[i + 1] - s->voff[i]);
  const uint32_t max_sw = algo == DG_ALGO_PAGERANK ? 10000u : std::min<uint32_t>(n_max + 1, dg::host::kMaxSweeps);
  auto timed = [&](dg_mode mode, uint32_t d, Spread& sp, uint32_t& sweeps) -> dg_status {
    std::vector<double> t;
    for (uint32_t i = 0; i <= kSetTuneRepeats; ++i) {  // the first run is a warm-up
      dg_stats x{};
      dg_status r = algo == DG_ALGO_PAGERANK
                        ? dg_set_pagerank(s, 0.85, tol, mode, d, dtype, 10000, 0, static_cast<double*>(outd), 1,
                                          nullptr, &x, hip_stream)
                        : dg_set_sssp(s, sources, mode, d, max_sw, 0, static_cast<uint32_t*>(outd), 1, nullptr, &x,
                                      hip_stream);
      if (r == DG_ERR_NOT_CONVERGED) r = DG_OK;
      if (r != DG_OK) return r;
      if (i) t.push_back(x.seconds);
      sweeps = x.sweeps;
    }
    sp = spread_of(t);
    return DG_OK;
  };
  struct Cand {
    dg_mode mode;
    uint32_t d;
  };
  const Cand cands[] = {{DG_SYNC, 1},      {DG_ASYNC, 1},       {DG_DELAYED, 16},        {DG_DELAYED, 64},
                        {DG_DELAYED, 256}, {DG_DELAYED, 1024}, {DG_DELAYED, DG_D_WHOLE}};
  const uint32_t P0 = s->g->P;  // the partition chosen at creation (or the current one)
  dg_status st = DG_OK;
  Spread def{}, best{};
  best.med = 1e300;
  uint32_t sw_def = 0, best_sw = 0, bestP = P0, evaluated = 0;
  Cand bestc = {DG_DELAYED, 64};
  std::vector<uint32_t> parts = {P0};
  for (uint32_t per_cu : {2u, 3u, 5u, 8u}) {
    uint32_t P = std::max(1u, std::min(s->g->cus * per_cu, s->g->T));
    if (P > 8) P &= ~7u;
    if (std::find(parts.begin(), parts.end(), P) == parts.end()) parts.push_back(P);
  }
  for (uint32_t P : parts) {
    if ((st = dg_graph_repartition(s->g, P, hip_stream)) != DG_OK) break;
    for (const Cand& c : cands) {
      Spread sp{};
      uint32_t sw = 0;
      if ((st = timed(c.mode, c.d, sp, sw)) != DG_OK) break;
      ++evaluated;
      if (P == parts[0] && c.mode == DG_DELAYED && c.d == 64) {
        def = sp;
        sw_def = sw;
      }
      if (sp.med < best.med) {
        best = sp;
        bestP = s->g->P;
        bestc = c;
        best_sw = sw;
      }
    }
    if (st != DG_OK) break;
  }
  dev_free(s->g, outd);
  if (st == DG_OK) st = dg_graph_repartition(s->g, bestP, hip_stream);
  if (st != DG_OK) {
    (void)dg_graph_repartition(s->g, P0, hip_stream);
    return st;
  }
  dg_tuning t{};
  t.workers = s->g->P;
  t.mode = bestc.mode;
  t.d = bestc.d;
  t.sweeps = best_sw;
  t.seconds = best.med;
  t.seconds_min = best.lo;
  t.seconds_max = best.hi;
  t.predicted_seconds = best.med;
  t.candidates = evaluated;
  t.graph_hash = s->g->hash;
  t.sweep_variant = s->g->variant;
  t.resident_vertices = DG_RESIDENT_AUTO;
  t.repeats = kSetTuneRepeats;
  t.default_seconds = def.med;
  t.default_seconds_min = def.lo;
  t.default_seconds_max = def.hi;
  (void)sw_def;
  *out = t;
  return DG_OK;
}

dg_status dg_set_set_capture(dg_set* s, uint32_t chunk_sweeps) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "set is NULL");
  return dg_graph_set_capture(s->g, chunk_sweeps);
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
  if (flags != 0) return fail(DG_ERR_INVALID_ARGUMENT, "flags must be 0 (got 0x%x)", flags);
  dg_status st = set_check_mode(mode, d, max_sweeps);
  if (st != DG_OK) return st;
  const uint32_t N = s->voff.back();
  if (dtype == DG_F32 && tol > 0.0 && tol < kF32Floor)
    return fail(DG_ERR_UNSUPPORTED, "float32 scores cannot settle below an L1 change of %.0e (tol %.3g); use DG_F64",
                kF32Floor, tol);
  hipStream_t q = static_cast<hipStream_t>(hip_stream);
  double* outd = out_scores;
  if (!out_on_device) {
    outd = static_cast<double*>(dev_alloc(s->g, (size_t)N * 8, q));
    if (!outd) return fail(DG_ERR_OUT_OF_MEMORY, "output staging allocation failed");
  }
  dg_stats x{};
  const dg_status run = dg_pagerank(s->g, damping, tol, mode, d, dtype, max_sweeps, outd, 1, &x, hip_stream);
  hipError_t he = hipSuccess;
  if (run == DG_OK || run == DG_ERR_NOT_CONVERGED) {
    he = launch_segment_normalize(outd, s->voff_d, s->G, q);
    if (he == hipSuccess && !out_on_device)
      he = hipMemcpyAsync(out_scores, outd, (size_t)N * 8, hipMemcpyDeviceToHost, q);
    if (he == hipSuccess) he = hipStreamSynchronize(q);
  }
  if (!out_on_device) dev_free(s->g, outd);
  if (run != DG_OK && run != DG_ERR_NOT_CONVERGED) return run;
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(DG_ERR_DEVICE, "set normalisation failed: %s", hipGetErrorString(he));
  }
  const dg_status ps = per_graph_sweeps(s, out_sweeps, q);
  if (ps != DG_OK) return ps;
  if (stats) *stats = x;
  if (run != DG_OK) return fail(run, "the set did not converge within %u sweeps", max_sweeps);
  return DG_OK;
}

dg_status dg_set_sssp(dg_set* s, const uint32_t* sources, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                      uint32_t flags, uint32_t* out_dist, int out_on_device, uint32_t* out_sweeps, dg_stats* stats,
                      void* hip_stream) {
  g_last_error.clear();
  if (!s) return fail(DG_ERR_INVALID_ARGUMENT, "set is NULL");
  if (!sources || !out_dist) return fail(DG_ERR_INVALID_ARGUMENT, "NULL sources or out_dist");
  if (flags != 0) return fail(DG_ERR_INVALID_ARGUMENT, "flags must be 0 (got 0x%x)", flags);
  for (uint32_t i = 0; i < s->G; ++i)
    if (sources[i] >= s->voff[i + 1] - s->voff[i])
      return fail(DG_ERR_INVALID_ARGUMENT, "source %u of graph %u is not a vertex of it", sources[i], i);
  dg_status st = set_check_mode(mode, d, max_sweeps);
  if (st != DG_OK) return st;
  hipStream_t q = static_cast<hipStream_t>(hip_stream);
  std::vector<uint32_t> usrc(s->G);
  for (uint32_t i = 0; i < s->G; ++i) usrc[i] = s->voff[i] + sources[i];
  if (s->G > 1) DG_HIP(hipMemcpyAsync(s->src_d, usrc.data() + 1, (size_t)(s->G - 1) * 4, hipMemcpyHostToDevice, q));
  dg_stats x{};
  st = dg::host::sssp_run(s->g, usrc[0], s->src_d, s->G - 1, mode, d, max_sweeps, out_dist, out_on_device, &x,
                          hip_stream);
  if (st != DG_OK && st != DG_ERR_NOT_CONVERGED) return st;
  const dg_status ps = per_graph_sweeps(s, out_sweeps, q);
  if (ps != DG_OK) return ps;
  if (stats) *stats = x;
  return st;
}

}  // extern "C"

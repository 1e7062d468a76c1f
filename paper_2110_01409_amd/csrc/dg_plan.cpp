// Host-only construction of a graph's device layout (see dg_plan.hpp), and
// the dg_plan_* entry points that return it without touching a device.
#include "dg_plan.hpp"

#include <algorithm>
#include <new>

#include "dg_graph.hpp"
#include "dg_host.hpp"
#include "dg_internal.hpp"

namespace dg {
namespace host {

namespace {

// 64-bit FNV-1a over 8-byte words (the tail zero-padded) of a uint32 array,
// continuing from h.
uint64_t hash_words(uint64_t h, const uint32_t* p, size_t n) {
  const uint64_t prime = 0x100000001b3ull;
  size_t i = 0;
  for (; i + 2 <= n; i += 2) h = (h ^ ((uint64_t)p[i] | ((uint64_t)p[i + 1] << 32))) * prime;
  if (i < n) h = (h ^ (uint64_t)p[i]) * prime;
  return (h ^ (uint64_t)n) * prime;
}

}  // namespace

void build_tiles(const std::vector<uint32_t>& in_ptr, uint32_t n, std::vector<uint32_t>& tile_v,
                 const std::vector<uint32_t>* seg_v, uint32_t max_e) {
  tile_v.clear();
  tile_v.push_back(0);
  uint32_t nv = 0;
  uint64_t ne = 0;
  size_t next_seg = 1;  // index into seg_v of the next graph boundary
  for (uint32_t v = 0; v < n; ++v) {
    const uint64_t deg = in_ptr[v + 1] - in_ptr[v];
    bool boundary = false;
    if (seg_v) {
      while (next_seg < seg_v->size() && (*seg_v)[next_seg] <= v) {
        boundary |= (*seg_v)[next_seg] == v;
        ++next_seg;
      }
    }
    if (nv > 0 && (boundary || nv == (uint32_t)kTileV || ne + deg > (uint64_t)max_e)) {
      tile_v.push_back(v);
      nv = 0;
      ne = 0;
    }
    ++nv;
    ne += deg;
  }
  if (tile_v.back() != n) tile_v.push_back(n);
}

void build_batch_tiles(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& in_ptr, uint32_t max_e,
                       std::vector<uint32_t>& btile_v, std::vector<uint32_t>& btile_e0) {
  btile_v.clear();
  btile_v.push_back(0);
  for (size_t t = 0; t + 1 < tile_v.size(); ++t) {
    const uint32_t a = tile_v[t], b = tile_v[t + 1];
    uint64_t ne = 0;
    for (uint32_t v = a; v < b; ++v) {
      const uint64_t deg = in_ptr[v + 1] - in_ptr[v];
      if (v > btile_v.back() && ne + deg > (uint64_t)max_e) {
        btile_v.push_back(v);
        ne = 0;
      }
      ne += deg;
    }
    btile_v.push_back(b);
  }
  btile_e0.resize(btile_v.size());
  for (size_t t = 0; t < btile_v.size(); ++t) btile_e0[t] = in_ptr[btile_v[t]];
}

void build_workers(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& tile_e0, uint32_t P,
                   std::vector<uint32_t>& work_t) {
  const uint32_t T = (uint32_t)tile_v.size() - 1;
  std::vector<double> cum(T + 1, 0.0);
  for (uint32_t t = 0; t < T; ++t) {
    const double e = (double)(tile_e0[t + 1] - tile_e0[t]);
    const double v = (double)(tile_v[t + 1] - tile_v[t]);
    cum[t + 1] = cum[t] + 256.0 + e + 4.0 * v;
  }
  work_t.assign(P + 1, T);
  work_t[0] = 0;
  for (uint32_t w = 1; w < P; ++w) {
    const double target = cum[T] * (double)w / (double)P;
    uint32_t t = (uint32_t)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
    t = std::min(std::max(t, work_t[w - 1]), T);
    work_t[w] = t;
  }
  work_t[P] = T;
}

void build_workers_seg(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& tile_e0,
                       const std::vector<uint32_t>& seg_v, uint32_t P, std::vector<uint32_t>& work_t,
                       std::vector<uint32_t>& wseg) {
  const uint32_t G = (uint32_t)seg_v.size() - 1;
  // first tile of each graph (tiles never cross a graph boundary)
  std::vector<uint32_t> gt(G + 1);
  for (uint32_t i = 0; i <= G; ++i)
    gt[i] = (uint32_t)(std::lower_bound(tile_v.begin(), tile_v.end(), seg_v[i]) - tile_v.begin());
  std::vector<double> cost(G, 0.0);
  for (uint32_t i = 0; i < G; ++i)
    for (uint32_t t = gt[i]; t < gt[i + 1]; ++t)
      cost[i] += 256.0 + (double)(tile_e0[t + 1] - tile_e0[t]) + 4.0 * (double)(tile_v[t + 1] - tile_v[t]);
  // one worker each, the rest by largest remaining cost per worker
  std::vector<uint32_t> pw(G, 1u);
  for (uint32_t extra = P - G, i = 0; extra > 0; --extra) {
    uint32_t best = 0;
    double bq = -1.0;
    for (i = 0; i < G; ++i) {
      if (pw[i] >= gt[i + 1] - gt[i]) continue;  // no more workers than tiles
      const double q = cost[i] / (double)pw[i];
      if (q > bq) bq = q, best = i;
    }
    if (bq < 0.0) break;
    ++pw[best];
  }
  wseg.assign(G + 1, 0);
  work_t.clear();
  work_t.push_back(0);
  for (uint32_t i = 0; i < G; ++i) {
    wseg[i + 1] = wseg[i] + pw[i];
    std::vector<uint32_t> tv(tile_v.begin() + gt[i], tile_v.begin() + gt[i + 1] + 1);
    std::vector<uint32_t> te(tile_e0.begin() + gt[i], tile_e0.begin() + gt[i + 1] + 1);
    std::vector<uint32_t> wt;
    build_workers(tv, te, pw[i], wt);
    for (uint32_t k = 1; k <= pw[i]; ++k) work_t.push_back(gt[i] + wt[k]);
  }
}

dg_status validate_graph(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx) {
  if (n == 0 || n > 0xFFFFFFFEu) return fail(DG_ERR_INVALID_ARGUMENT, "n = %u outside [1, 2^32-2]", n);
  if (m >= (uint64_t)0xFFFFFFFFu - 2 * kEdgePad)
    return fail(DG_ERR_INVALID_ARGUMENT, "m = %llu too large", (unsigned long long)m);
  if (layout != DG_CSR && layout != DG_CSC) return fail(DG_ERR_INVALID_ARGUMENT, "unknown layout %d", (int)layout);
  if (!ptr) return fail(DG_ERR_INVALID_ARGUMENT, "ptr is NULL");
  if (m > 0 && !idx) return fail(DG_ERR_INVALID_ARGUMENT, "idx is NULL");
  if (ptr[0] != 0) return fail(DG_ERR_INVALID_ARGUMENT, "ptr[0] = %llu, expected 0", (unsigned long long)ptr[0]);
  for (uint32_t v = 0; v < n; ++v)
    if (ptr[v + 1] < ptr[v]) return fail(DG_ERR_INVALID_ARGUMENT, "ptr decreases at %u", v);
  if (ptr[n] != m)
    return fail(DG_ERR_INVALID_ARGUMENT, "ptr[n] = %llu, expected m = %llu", (unsigned long long)ptr[n],
                (unsigned long long)m);
  for (uint64_t e = 0; e < m; ++e)
    if (idx[e] >= n) return fail(DG_ERR_INVALID_ARGUMENT, "idx[%llu] = %u >= n", (unsigned long long)e, idx[e]);
  return DG_OK;
}

dg_status build_layout(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                       const uint32_t* w, const dg_graph_opts* opts, uint32_t workers, Layout& L,
                       const std::vector<uint32_t>* seg_v) {
  const uint32_t variant = opts ? opts->sweep_variant : DG_SWEEP_AUTO;
  if (variant > DG_SWEEP_NARROW) return fail(DG_ERR_INVALID_ARGUMENT, "unknown sweep_variant %u", variant);
  uint32_t hot_max = (!opts || opts->hot_vertices == DG_HOT_AUTO) ? 524288u : opts->hot_vertices;
  hot_max = std::min<uint32_t>(hot_max, 0xFFFFFFFEu - n);
  const bool res_auto = !opts || opts->resident_vertices == DG_RESIDENT_AUTO;
  const uint32_t res_max = std::min<uint32_t>(res_auto ? kResBytes / 4u : opts->resident_vertices, kResBytes / 4u);
  L = Layout();
  L.n = n;
  L.m = m;
  L.has_w = w != nullptr;
  try {
    // In-edge form (stable counting sort: in-edges of a vertex by ascending
    // source), with each source replaced by the slot of its published value.
    L.in_ptr.assign((size_t)n + 1, 0);
    L.in_src.assign((size_t)m + kEdgePad, 0);
    if (w) L.in_w.assign((size_t)m + kEdgePad, 0);
    L.out_deg.assign(n, 0);
    if (layout == DG_CSR) {
      for (uint32_t u = 0; u < n; ++u) L.out_deg[u] = (uint32_t)(ptr[u + 1] - ptr[u]);
    } else {
      for (uint64_t e = 0; e < m; ++e) ++L.out_deg[idx[e]];
    }
    // Compact region: the sources with the largest above-average out-degree,
    // in three runs, each in vertex order: the R/2 largest, the next R/2
    // (together the sweeps' LDS-resident table of R slots, of which a
    // float64 sweep keeps the first half), then the rest.  Vertex order keeps
    // each worker's hot vertices in a few contiguous runs of slots, so a
    // commit dirties few cache lines of the region everybody gathers from
    // (the reason the paper gives for blocked partitioning and line-sized
    // buffers); ordering the table by degree instead made asynchronous
    // sweeps 12% slower on R-MAT.
    L.cpos.resize(n);
    for (uint32_t v = 0; v < n; ++v) L.cpos[v] = v;
    {
      const double avg = (double)m / (double)n;
      std::vector<uint32_t> cand;
      for (uint32_t v = 0; v < n; ++v)
        if (L.out_deg[v] > 1 && (double)L.out_deg[v] > avg) cand.push_back(v);
      std::stable_sort(cand.begin(), cand.end(),
                       [&](uint32_t a, uint32_t b) { return L.out_deg[a] > L.out_deg[b]; });
      L.K = (uint32_t)std::min<size_t>(cand.size(), hot_max);
      cand.resize(L.K);
      L.R = std::min(L.K, res_max);
      // Automatic size: no table (and no reordering) unless it covers at
      // least 1/16 of the in-edges; below that its refreshes cost more than
      // the gathers it saves.
      if (res_auto) {
        uint64_t cover = 0;
        for (uint32_t r = 0; r < L.R; ++r) cover += L.out_deg[cand[r]];
        if (cover * 16 < m) L.R = 0;
      }
      const uint32_t half = (L.R + 1) / 2;
      std::sort(cand.begin(), cand.begin() + half);
      std::sort(cand.begin() + half, cand.begin() + L.R);
      std::sort(cand.begin() + L.R, cand.end());
      for (uint32_t r = 0; r < L.K; ++r) {
        L.cpos[cand[r]] = n + r;
        L.hot_edges += L.out_deg[cand[r]];
        if (r < L.R) L.res_edges += L.out_deg[cand[r]];
      }
    }
    if (layout == DG_CSR) {
      for (uint64_t e = 0; e < m; ++e) ++L.in_ptr[idx[e] + 1];
      for (uint32_t v = 0; v < n; ++v) L.in_ptr[v + 1] += L.in_ptr[v];
      std::vector<uint32_t> pos(L.in_ptr.begin(), L.in_ptr.end() - 1);
      for (uint32_t u = 0; u < n; ++u) {
        const uint32_t slot = L.cpos[u];
        for (uint64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
          const uint32_t p = pos[idx[e]]++;
          L.in_src[p] = slot;
          if (w) L.in_w[p] = w[e];
        }
      }
    } else {
      for (uint32_t v = 0; v <= n; ++v) L.in_ptr[v] = (uint32_t)ptr[v];
      for (uint64_t e = 0; e < m; ++e) L.in_src[e] = L.cpos[idx[e]];
      if (w) std::copy(w, w + m, L.in_w.begin());
    }
    for (uint32_t v = 0; v < n; ++v) {
      L.max_in_deg = std::max(L.max_in_deg, L.in_ptr[v + 1] - L.in_ptr[v]);
      L.n_dangling += L.out_deg[v] == 0;
    }
    // Sweep variant (SweepVariant): the wide tiles, or the narrow ones when
    // the wide give fewer than kNarrowBelow tiles per worker.
    build_tiles(L.in_ptr, n, L.tile_v, seg_v, (uint32_t)kTileE);
    const uint64_t T = L.tile_v.size() - 1, P = std::max(1u, workers);
    L.variant = variant != DG_SWEEP_AUTO ? variant
                : T < kNarrowBelow * P       ? (uint32_t)kNarrow
                : T <= kInFlightUpTo * P     ? (uint32_t)kWideInFlight
                                             : (uint32_t)kWide;
    if (L.variant == kNarrow) build_tiles(L.in_ptr, n, L.tile_v, seg_v, (uint32_t)kTileENarrow);
    L.tile_e0.resize(L.tile_v.size());
    for (size_t t = 0; t < L.tile_v.size(); ++t) L.tile_e0[t] = L.in_ptr[L.tile_v[t]];
    uint64_t h = 0xcbf29ce484222325ull;
    h = hash_words(h, L.in_ptr.data(), L.in_ptr.size());
    h = hash_words(h, L.in_src.data(), (size_t)m);
    if (w) h = hash_words(h, L.in_w.data(), (size_t)m);
    L.hash = hash_words(h, L.out_deg.data(), L.out_deg.size());
    // Weights that all fit a byte are stored as bytes (packed four to a
    // word here): a quarter of the weight stream's bytes per sweep.
    if (w && std::all_of(w, w + m, [](uint32_t x) { return x <= 255u; })) {
      L.w8pack.assign(((size_t)m + kEdgePad + 16 + 3) / 4, 0u);
      for (uint64_t e = 0; e < m; ++e) L.w8pack[e >> 2] |= L.in_w[e] << (8 * (e & 3));
      std::vector<uint32_t>().swap(L.in_w);
    }
  } catch (const std::bad_alloc&) {
    L = Layout();
    return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed while building the in-edge form");
  }
  // Gathers address the value array through a buffer resource with a 32-bit
  // byte range: (n + K) float64 slots must stay below 4 GiB.
  if (((uint64_t)n + L.K) * 8u >= (1ull << 32))
    return fail(DG_ERR_UNSUPPORTED, "n + hot slots = %llu exceeds the 2^29 value slots a sweep can address",
                (unsigned long long)n + L.K);
  return DG_OK;
}

uint32_t batch_workers_for(uint32_t cus, uint32_t per_cu, uint32_t batch_tiles) {
  uint32_t P = std::max(1u, std::min(cus * per_cu, batch_tiles));
  if (P > 8) P &= ~7u;
  return P;
}

uint32_t plan_workers(const Layout& L, uint32_t want_workers, uint32_t cus, uint32_t per_cu) {
  uint32_t P = want_workers ? want_workers : cus * per_cu;
  P = std::max(1u, std::min(P, L.T()));
  if (P > 8 && !want_workers) P &= ~7u;
  return P;
}

}  // namespace host
}  // namespace dg

using dg::host::fail;
using dg::host::g_last_error;

struct dg_plan {
  dg::host::Layout L;
  uint32_t P = 0;
  std::vector<uint32_t> work_t;
  std::vector<uint32_t> btile_v, btile_e0;  // tiles of the batched kernels
  std::vector<uint32_t> bwork[2];           // their default partitions: SSSP, PPR (first batched tile of each worker)
};

extern "C" {

dg_status dg_plan_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                         const uint32_t* w, const dg_graph_opts* opts, uint32_t compute_units, dg_plan** out) {
  g_last_error.clear();
  if (!out) return fail(DG_ERR_INVALID_ARGUMENT, "out is NULL");
  if (compute_units == 0) return fail(DG_ERR_INVALID_ARGUMENT, "compute_units must be >= 1");
  if (opts && opts->arrays_on_device != 0)
    return fail(DG_ERR_INVALID_ARGUMENT, "a plan is built without a device: arrays_on_device must be 0");
  dg_status st = dg::host::validate_graph(n, m, layout, ptr, idx);
  if (st != DG_OK) return st;
  dg_plan* p = new (std::nothrow) dg_plan;
  if (!p) return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
  const uint32_t workers = opts && opts->workers ? opts->workers : compute_units * dg::host::kWorkersPerCU;
  if ((st = dg::host::build_layout(n, m, layout, ptr, idx, w, opts, workers, p->L)) != DG_OK) {
    delete p;
    return st;
  }
  p->P = dg::host::plan_workers(p->L, opts ? opts->workers : 0u, compute_units, dg::host::kWorkersPerCU);
  try {
    dg::host::build_workers(p->L.tile_v, p->L.tile_e0, p->P, p->work_t);
    dg::host::build_batch_tiles(p->L.tile_v, p->L.in_ptr, dg::host::kBatchTileE, p->btile_v, p->btile_e0);
    const uint32_t Tb = (uint32_t)p->btile_v.size() - 1;
    const uint32_t per[2] = {dg::host::kBatchSsspWorkersPerCU, dg::host::kBatchPprWorkersPerCU};
    for (int a = 0; a < 2; ++a)
      dg::host::build_workers(p->btile_v, p->btile_e0, dg::host::batch_workers_for(compute_units, per[a], Tb),
                              p->bwork[a]);
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(DG_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  *out = p;
  return DG_OK;
}

dg_status dg_plan_info_get(const dg_plan* p, dg_plan_info* info) {
  if (!p || !info) return fail(DG_ERR_INVALID_ARGUMENT, "NULL argument");
  const dg::host::Layout& L = p->L;
  info->n = L.n;
  info->m = L.m;
  info->workers = p->P;
  info->tiles = L.T();
  info->max_in_degree = L.max_in_deg;
  info->dangling = L.n_dangling;
  info->hot_vertices = L.K;
  info->hot_edges = L.hot_edges;
  info->resident_vertices = L.R;
  info->resident_edges = L.res_edges;
  info->weight_bytes = !L.has_w ? 0u : (L.w8pack.empty() ? 4u : 1u);
  info->content_hash = L.hash;
  info->sweep_variant = L.variant;
  info->batch_tiles = (uint32_t)p->btile_v.size() - 1;
  info->batch_workers_sssp = (uint32_t)p->bwork[0].size() - 1;
  info->batch_workers_ppr = (uint32_t)p->bwork[1].size() - 1;
  return DG_OK;
}

dg_status dg_plan_batch_tiles(const dg_plan* p, uint32_t* btile_v, uint32_t* work_sssp, uint32_t* work_ppr) {
  if (!p) return fail(DG_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (btile_v) std::copy(p->btile_v.begin(), p->btile_v.end(), btile_v);
  if (work_sssp) std::copy(p->bwork[0].begin(), p->bwork[0].end(), work_sssp);
  if (work_ppr) std::copy(p->bwork[1].begin(), p->bwork[1].end(), work_ppr);
  return DG_OK;
}

dg_status dg_plan_arrays(const dg_plan* p, uint32_t* in_ptr, uint32_t* in_src, uint32_t* in_w, uint32_t* cpos,
                         uint32_t* tile_v, uint32_t* work_t) {
  if (!p) return fail(DG_ERR_INVALID_ARGUMENT, "plan is NULL");
  const dg::host::Layout& L = p->L;
  if (in_w && !L.has_w) return fail(DG_ERR_INVALID_ARGUMENT, "the graph has no weights");
  if (in_ptr) std::copy(L.in_ptr.begin(), L.in_ptr.end(), in_ptr);
  if (in_src) std::copy(L.in_src.begin(), L.in_src.begin() + (size_t)L.m, in_src);
  if (in_w) {
    if (L.w8pack.empty()) {
      std::copy(L.in_w.begin(), L.in_w.begin() + (size_t)L.m, in_w);
    } else {
      for (uint64_t e = 0; e < L.m; ++e) in_w[e] = (L.w8pack[e >> 2] >> (8 * (e & 3))) & 255u;
    }
  }
  if (cpos) std::copy(L.cpos.begin(), L.cpos.end(), cpos);
  if (tile_v) std::copy(L.tile_v.begin(), L.tile_v.end(), tile_v);
  if (work_t) std::copy(p->work_t.begin(), p->work_t.end(), work_t);
  return DG_OK;
}

dg_status dg_plan_destroy(dg_plan* p) {
  delete p;
  return DG_OK;
}

}  // extern "C"

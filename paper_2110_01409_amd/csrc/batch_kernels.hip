// Batched queries: many SSSP sources, or many personalised-PageRank restart
// vertices, swept together on one graph in one launch.
//
// Queries are grouped in batches of 64: the 64 lanes of a wavefront are the
// 64 queries of a batch, and values are stored vertex-major, [slot][64], so
// a gather of a source's values for the whole batch is one coalesced
// 256-byte row.  The in-edge index and weight streams are read once per
// batch instead of once per query.  Batches are the y dimension of the
// launch; a batch whose queries have all met the stopping rule exits at once.
//
// Work mapping: tiles of their own (the single-query tiles cut into runs of
// at most 4096 in-edges, a vertex with more being a run of its own), in
// contiguous blocks of a partition per algorithm (by default eight 256-thread
// workgroups per compute unit for SSSP, five for PPR), each walked in
// ascending order.  Within a tile the four wavefronts of the workgroup take
// vertices round-robin; a single-vertex tile (a hub) is split over the four
// wavefronts and combined in LDS.  For each
// vertex a wavefront reads 64 in-edges with one coalesced load, broadcasts
// each edge's source slot and weight with readlane, and keeps eight row
// gathers in flight.
//
// Commit modes are those of the single-query sweeps: synchronous (double
// buffer), asynchronous (agent-scope store per vertex), delayed (staged per
// wavefront and committed every d vertices of the worker, i.e. every
// ceil(d/4) rows of each wavefront, and at the end of the block: with
// d <= kLdsStageMaxD in LDS, beyond in a per-batch shadow array).
#include "dg_device.hpp"
#include "dg_internal.hpp"

namespace dg {
namespace {

constexpr uint32_t kQ = 64;  // queries per batch

__device__ __forceinline__ uint32_t worker_of(uint32_t b, uint32_t P) {
  if ((P & 7u) == 0) return (b & 7u) * (P >> 3) + (b >> 3);
  return b;
}

template <int M, typename T>
__device__ __forceinline__ T ld_q(const T* p) {
  if constexpr (M == kSync) return *p;
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_q(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Delayed commits staged in LDS: each wavefront keeps up to kStageRows rows
// it computed, with their slots, in its own part of the dynamic LDS and
// commits them, as coalesced 64-lane rows, once `per` are staged and at the
// end of its block.  Used instead of the global shadow when d <= kStageRows *
// waves per workgroup, so that a commit every d vertices of the worker costs
// no extra row traffic.  Each wavefront reads back only what it wrote itself,
// in order, so no barrier is needed.  Every lane stages a value (cnt stays
// the same in all lanes); a lane whose query is frozen does not store it.
// (Rows held in registers instead cost the SSSP kernel 73 VGPRs and two
// waves per SIMD: 14.3 against 12.1 ms per batch-sweep on RMAT-22.)
template <typename T>
struct LdsStage {
  T* rows;           // [kStageRows][64], this wavefront's
  uint32_t* slot;    // [kStageRows], this wavefront's
  uint32_t cnt = 0;  // the same in every lane
  __device__ __forceinline__ void flush(T* out, uint32_t lane, bool store) {
    for (uint32_t r = 0; r < cnt; ++r)
      if (store) st_q(out + (size_t)slot[r] * kQ + lane, rows[r * kQ + lane]);
    cnt = 0;
  }
  __device__ __forceinline__ void push(uint32_t p, T v, uint32_t per, T* out, uint32_t lane, bool store) {
    rows[cnt * kQ + lane] = v;
    if (lane == 0) slot[cnt] = p;
    if (++cnt >= per) flush(out, lane, store);
  }
};

// Dynamic LDS of a batched PPR sweep: the staged rows and their slots when
// a delayed sweep stages in LDS, and in every sweep each wavefront's three
// per-query partials (double) for the workgroup's fold at the end, which a
// staging wavefront writes over its own rows once it has flushed them.
template <typename T>
constexpr size_t lds_stage_bytes() {
  return (size_t)(kWG / 64) * kStageRows * (kQ * sizeof(T) + sizeof(uint32_t));
}
constexpr size_t kRedBytes = 3 * kQ * sizeof(double);  // one wavefront's partials
static_assert(kStageRows * kQ * sizeof(float) >= kRedBytes, "a wavefront's staged rows hold its partials");
template <typename T, bool STAGE>
constexpr size_t mppr_dyn_bytes() {
  return STAGE ? lds_stage_bytes<T>() : (size_t)(kWG / 64) * kRedBytes;
}

__device__ __forceinline__ uint32_t sat_add_q(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s < a ? kInf : s;
}

__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t j) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)j);
}

typedef const __attribute__((address_space(4))) uint32_t* cu32p;
__device__ __forceinline__ cu32p cst(const uint32_t* p) { return (cu32p)(p); }

// Delayed commits through the per-batch shadow array, for d beyond what a
// wavefront stages itself: the same cadence (each wavefront commits its own
// rows once `per` are staged, mid-tile, and at the end of its block), with
// the rows in the shadow.  The rows of a commit are the wavefront's vertices
// since its previous commit, walked again in the order it updated them:
// tile by tile, vertices v0 + wv, v0 + wv + 4, ... of a tile, a single-vertex
// tile being wavefront 0's.  (ft, fv) is the first of them; pend their number
// (the same in every lane).  The wavefront reads back only rows it wrote
// itself, so no barrier is needed.
struct ShadowWalk {
  uint32_t ft, fv, pend = 0;
  __device__ __forceinline__ ShadowWalk(uint32_t t0, uint32_t first_v, uint32_t wv) : ft(t0), fv(first_v + wv) {}
  // Commits the rows through vertex vl of tile tl (inclusive).
  template <typename T>
  __device__ __forceinline__ void commit(cu32p tile_v, const uint32_t* cpos, const T* shadow, T* out, uint32_t tl,
                                        uint32_t vl, uint32_t wv, uint32_t lane, bool store) {
    for (uint32_t tt = ft; tt <= tl; ++tt) {
      const uint32_t a0 = tile_v[tt], a1 = tile_v[tt + 1];
      const bool hub = a1 - a0 == 1;
      if (hub && wv != 0) continue;
      const uint32_t step = hub ? 1u : kWG / 64;
      const uint32_t end = tt == tl ? vl + 1 : a1;
      for (uint32_t v = tt == ft ? fv : (hub ? a0 : a0 + wv); v < end; v += step)
        if (store) st_q(out + (size_t)cpos[v] * kQ + lane, shadow[(size_t)v * kQ + lane]);
    }
    pend = 0;
  }
  // After the wavefront staged the row of vertex v in tile t (hub: a
  // single-vertex tile).
  template <typename T>
  __device__ __forceinline__ void staged(cu32p tile_v, const uint32_t* cpos, const T* shadow, T* out, uint32_t t,
                                         uint32_t v, bool hub, uint32_t per, uint32_t wv, uint32_t lane, bool store) {
    if (++pend < per) return;
    commit(tile_v, cpos, shadow, out, t, v, wv, lane, store);
    ft = t;
    fv = v + (hub ? 1u : kWG / 64);
  }
  // At the end of the worker's block (tiles t0 .. t1-1).
  template <typename T>
  __device__ __forceinline__ void finish(cu32p tile_v, const uint32_t* cpos, const T* shadow, T* out, uint32_t t1,
                                         uint32_t wv, uint32_t lane, bool store) {
    if (pend) commit(tile_v, cpos, shadow, out, t1 - 1, tile_v[t1] - 1, wv, lane, store);
  }
};


// min over in-edges [e0, e1) of d[src] + w, taking every `step`-th group of
// 64 edges starting at group `first`.  Lane q handles query q.
template <int M>
__device__ __forceinline__ uint32_t relax_edges(const uint32_t* __restrict__ in_src, const uint32_t* __restrict__ in_w,
                                                const uint8_t* __restrict__ in_w8, const uint32_t* d, uint32_t e0,
                                                uint32_t e1, uint32_t first, uint32_t step, uint32_t lane) {
  uint32_t acc = kInf;
  for (uint32_t e = e0 + first * 64u; e < e1; e += 64u * step) {
    const uint32_t cnt = min(64u, e1 - e);
    const uint32_t idx = lane < cnt ? in_src[e + lane] : 0u;
    const uint32_t wt = lane < cnt ? (in_w8 ? (uint32_t)in_w8[e + lane] : in_w[e + lane]) : 0u;
    uint32_t j = 0;
    for (; j + 8 <= cnt; j += 8) {
      uint32_t val[8];
#pragma unroll
      for (uint32_t q = 0; q < 8; ++q) val[q] = ld_q<M>(d + (size_t)bcast(idx, j + q) * kQ + lane);
#pragma unroll
      for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t c = sat_add_q(val[q], bcast(wt, j + q));
        acc = c < acc ? c : acc;
      }
    }
    for (; j < cnt; ++j) {
      const uint32_t c = sat_add_q(ld_q<M>(d + (size_t)bcast(idx, j) * kQ + lane), bcast(wt, j));
      acc = c < acc ? c : acc;
    }
  }
  return acc;
}

// sum over in-edges [e0, e1) of c[src] (float64), same access pattern.
template <int M, typename T>
__device__ __forceinline__ double pull_edges(const uint32_t* __restrict__ in_src, const T* c, uint32_t e0, uint32_t e1,
                                             uint32_t first, uint32_t step, uint32_t lane) {
  double acc = 0.0;
  for (uint32_t e = e0 + first * 64u; e < e1; e += 64u * step) {
    const uint32_t cnt = min(64u, e1 - e);
    const uint32_t idx = lane < cnt ? in_src[e + lane] : 0u;
    uint32_t j = 0;
    for (; j + 8 <= cnt; j += 8) {
      T val[8];
#pragma unroll
      for (uint32_t q = 0; q < 8; ++q) val[q] = ld_q<M>(c + (size_t)bcast(idx, j + q) * kQ + lane);
#pragma unroll
      for (uint32_t q = 0; q < 8; ++q) acc += (double)val[q];
    }
    for (; j < cnt; ++j) acc += (double)ld_q<M>(c + (size_t)bcast(idx, j) * kQ + lane);
  }
  return acc;
}

// ------------------------------------------------------ multi-source SSSP --

// SH: delayed commits through the shadow, compiled apart from the kernel
// that stages in LDS (as the PPR kernel).
template <int M, bool SH>
__global__ __launch_bounds__(kWG) void mbf_sweep_kernel(MbfArgs a) {
  __shared__ uint32_t s_hub[kWG / 64][kQ];
  __shared__ int s_any;
  __shared__ uint32_t s_lane[kQ];
  const uint32_t b = blockIdx.y, NB = a.NB, k = a.k;
  // batch already converged (call mode) or without running queries (serving)
  if (a.bactive ? a.bactive[b] == 0 : a.changed[k * NB + b] == 0) return;

  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint32_t w = worker_of(blockIdx.x, a.g.P);
  const size_t stride = (size_t)(a.g.n + a.g.K) * kQ;
  const uint32_t* din = a.din + b * stride;
  uint32_t* dout = a.dout + b * stride;
  uint32_t* shadow = a.shadow ? a.shadow + (size_t)b * a.g.n * kQ : nullptr;
  const cu32p tile_v = cst(a.g.tile_v);
  const cu32p in_ptr = cst(a.g.in_ptr);
  const uint32_t t0 = cst(a.g.work_t)[w], t1 = cst(a.g.work_t)[w + 1];
  if (tid == 0) s_any = 0;
  if (tid < kQ) s_lane[tid] = 0;
  __syncthreads();
  uint32_t any = 0;
  // Delayed mode without a shadow: stage in LDS, commit every per rows.
  constexpr bool lds = M == kDelayed && !SH;
  // rows per wavefront between commits (the host stages in LDS only for d <= kLdsStageMaxD)
  const uint32_t per_rows = (uint32_t)(((uint64_t)a.d + kWG / 64 - 1) / (kWG / 64));
  const uint32_t per = min(per_rows, kStageRows);
  extern __shared__ __align__(16) unsigned char s_dyn[];
  LdsStage<uint32_t> ls;
  ls.rows = reinterpret_cast<uint32_t*>(s_dyn) + (size_t)wv * kStageRows * kQ;
  ls.slot = reinterpret_cast<uint32_t*>(s_dyn + (size_t)(kWG / 64) * kStageRows * kQ * sizeof(uint32_t)) + wv * kStageRows;
  ShadowWalk sw(t0, t0 < t1 ? tile_v[t0] : 0u, wv);

  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t v0 = tile_v[t], v1 = tile_v[t + 1], nv = v1 - v0;
    if (nv == 1) {
      // Hub: the four wavefronts split its in-edges, wavefront 0 commits.
      const uint32_t e0 = in_ptr[v0], e1 = in_ptr[v1];
      s_hub[wv][lane] = relax_edges<M>(a.g.in_src, a.g.in_w, a.g.in_w8, din, e0, e1, wv, kWG / 64, lane);
      __syncthreads();
      if (wv == 0) {
        uint32_t acc = s_hub[0][lane];
        for (uint32_t i = 1; i < kWG / 64; ++i) acc = s_hub[i][lane] < acc ? s_hub[i][lane] : acc;
        const uint32_t p = a.g.cpos[v0];
        const uint32_t old = ld_q<M>(din + (size_t)p * kQ + lane);
        const uint32_t nw = acc < old ? acc : old;
        any |= nw < old;
        if constexpr (M == kSync) dout[(size_t)p * kQ + lane] = nw;
        else if constexpr (M == kAsync) st_q(dout + (size_t)p * kQ + lane, nw);
        else if constexpr (lds) ls.push(p, nw, per, dout, lane, true);
        else {
          shadow[(size_t)v0 * kQ + lane] = nw;
          sw.staged(tile_v, a.g.cpos, shadow, dout, t, v0, true, per_rows, wv, lane, true);
        }
      }
      __syncthreads();
    } else {
      for (uint32_t v = v0 + wv; v < v1; v += kWG / 64) {
        const uint32_t acc = relax_edges<M>(a.g.in_src, a.g.in_w, a.g.in_w8, din, in_ptr[v], in_ptr[v + 1], 0, 1, lane);
        const uint32_t p = a.g.cpos[v];
        const uint32_t old = ld_q<M>(din + (size_t)p * kQ + lane);
        const uint32_t nw = acc < old ? acc : old;
        any |= nw < old;
        if constexpr (M == kSync) dout[(size_t)p * kQ + lane] = nw;
        else if constexpr (M == kAsync) st_q(dout + (size_t)p * kQ + lane, nw);
        else if constexpr (lds) ls.push(p, nw, per, dout, lane, true);
        else {
          shadow[(size_t)v * kQ + lane] = nw;
          sw.staged(tile_v, a.g.cpos, shadow, dout, t, v, false, per_rows, wv, lane, true);
        }
      }
    }
    if (M == kDelayed && t + 1 == t1) {  // the end of the block
      if constexpr (lds) ls.flush(dout, lane, true);
      else sw.finish(tile_v, a.g.cpos, shadow, dout, t1, wv, lane, true);
    }
  }
  if (a.lchg) {
    // serving: which queries (lanes) changed anywhere in this sweep
    if (any) atomicOr(&s_lane[lane], 1u);
    __syncthreads();
    if (tid < kQ && s_lane[tid]) atomicOr(a.lchg + (size_t)b * kQ + tid, 1u);
    return;
  }
  if (any) s_any = 1;  // benign race: every writer stores 1
  __syncthreads();
  if (tid == 0 && s_any) {
    st_q(a.changed + (k + 1) * NB + b, 1u);
    if (a.hchanged) st_host(a.hchanged + (k + 1) * NB + b, 1u);
  }
}

__global__ __launch_bounds__(kWG) void mbf_init_kernel(uint32_t* d0, uint32_t* d1, const uint32_t* cpos,
                                                       const uint32_t* src, uint32_t nq, uint32_t n, uint32_t K,
                                                       uint32_t NB) {
  // one thread per (vertex, query) of every batch
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  const size_t per_batch = (size_t)n * kQ;
  if (i >= per_batch * NB) return;
  const uint32_t b = (uint32_t)(i / per_batch);
  const uint32_t v = (uint32_t)((i % per_batch) / kQ), q = (uint32_t)(i % kQ);
  const uint32_t qi = b * kQ + q;
  const uint32_t val = (qi < nq && src[qi] == v) ? 0u : kInf;
  const size_t off = (size_t)b * (n + K) * kQ + (size_t)cpos[v] * kQ + q;
  d0[off] = val;
  if (d1) d1[off] = val;
}

// out[q][v] = d[cpos[v]][q] for the nq queries; a 64x64 tile per block
// through LDS so both the read and the write are coalesced.
__global__ __launch_bounds__(kWG) void mbf_out_kernel(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t K,
                                                      uint32_t nq, uint32_t* out) {
  __shared__ uint32_t s[64][65];
  const uint32_t b = blockIdx.y, vb = blockIdx.x * 64;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t* db = d + (size_t)b * (n + K) * kQ;
  for (uint32_t r = wv; r < 64; r += kWG / 64) {
    const uint32_t v = vb + r;
    s[r][lane] = v < n ? db[(size_t)cpos[v] * kQ + lane] : 0u;
  }
  __syncthreads();
  for (uint32_t r = wv; r < 64; r += kWG / 64) {
    const uint32_t qi = b * kQ + r, v = vb + lane;
    if (qi < nq && v < n) out[(size_t)qi * n + v] = s[lane][r];
  }
}

// --------------------------------------------- multi personalised PageRank --
//
// Each query's scores are stored scaled: stored = true value * S, with one
// float64 factor S per query for the whole sweep.  After a sweep its total
// mass M is known and the true vector is rescaled by 1/M, which costs no pass
// over memory: S becomes S * M and the stored values are reinterpreted.  The
// fixed point has mass 1, so the rescale changes no fixed point; it removes
// the slowly decaying mass error that Gauss-Seidel-ordered (asynchronous and
// delayed) sweeps create, which synchronous sweeps do not have because they
// conserve mass exactly.

// SH: delayed commits through the shadow (d beyond what a wavefront stages
// in LDS); compiled apart from the LDS-staging kernel so that neither carries
// the other's state.
template <int M, typename T, bool SH>
__global__ __launch_bounds__(kWG) void mppr_sweep_kernel(MpprArgs a) {
  __shared__ double s_hub[kWG / 64][kQ];
  __shared__ int s_last;
  const uint32_t b = blockIdx.y, NB = a.NB, k = a.k;
  // batch already converged (call mode) or without running queries (serving)
  if (a.bactive ? a.bactive[b] == 0 : !(a.resid[k * NB + b] >= a.tol)) return;

  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint32_t P = a.g.P;
  const uint32_t w = worker_of(blockIdx.x, P);
  const size_t stride = (size_t)(a.g.n + a.g.K) * kQ;
  const T* cin = static_cast<const T*>(a.cin) + b * stride;
  T* cout = static_cast<T*>(a.cout) + b * stride;
  T* x = static_cast<T*>(a.x) + (size_t)b * a.g.n * kQ;
  T* shadow = a.shadow ? static_cast<T*>(a.shadow) + (size_t)b * a.g.n * kQ : nullptr;
  const uint32_t qi = b * kQ + lane;
  const uint32_t src = qi < a.nq ? a.src[qi] : kInf;
  // A query that met the stopping rule in an earlier sweep (and every padding
  // lane) is frozen: its lane still walks the edges with the others but
  // writes nothing, so its result is the iterate of the sweep that stopped it.
  const bool live = a.qdone[(size_t)b * kQ + lane] == 0;
  const double alpha = a.alpha;
  const size_t ring = ((size_t)(k & 1u) * NB + b) * kQ + lane;
  const double S = a.scale[ring], invS = 1.0 / S;
  const double D = a.dang[ring];
  const double restart = (1.0 - alpha) + alpha * D;
  const cu32p tile_v = cst(a.g.tile_v);
  const cu32p in_ptr = cst(a.g.in_ptr);
  const uint32_t t0 = cst(a.g.work_t)[w], t1 = cst(a.g.work_t)[w + 1];
  double r_loc = 0.0, dm_loc = 0.0, m_loc = 0.0;
  // Delayed mode without a shadow: stage in LDS, commit every per rows.
  constexpr bool lds = M == kDelayed && !SH;
  // rows per wavefront between commits (the host stages in LDS only for d <= kLdsStageMaxD)
  const uint32_t per_rows = (uint32_t)(((uint64_t)a.d + kWG / 64 - 1) / (kWG / 64));
  const uint32_t per = min(per_rows, kStageRows);
  ShadowWalk sw(t0, t0 < t1 ? tile_v[t0] : 0u, wv);
  uint32_t cur_t = t0;  // the tile being updated (for the shadow's commits)
  extern __shared__ __align__(16) unsigned char s_dyn[];
  LdsStage<T> ls;
  ls.rows = reinterpret_cast<T*>(s_dyn) + (size_t)wv * kStageRows * kQ;
  ls.slot = reinterpret_cast<uint32_t*>(s_dyn + (size_t)(kWG / 64) * kStageRows * kQ * sizeof(T)) + wv * kStageRows;
  // This wavefront's partials [3][kQ]: over its own staged rows when staging
  // (free after its last flush), else in a region of their own.
  constexpr size_t red_stride = lds ? kStageRows * kQ * sizeof(T) : kRedBytes;
  auto red = [&](uint32_t j, uint32_t wave) -> double& {
    return reinterpret_cast<double*>(s_dyn + (size_t)wave * red_stride)[j * kQ + lane];
  };

  // Called by every lane of the wavefront (frozen queries included).
  auto update = [&](uint32_t v, double acc) {
    const uint32_t p = a.g.cpos[v];
    T cn = (T)0;
    if (live) {
      const double xn = alpha * acc * invS + (v == src ? restart : 0.0);
      const double xo = (double)x[(size_t)v * kQ + lane] * invS;
      x[(size_t)v * kQ + lane] = (T)(xn * S);
      const uint32_t dg = a.g.out_deg[v];
      cn = dg ? (T)(xn * S / (double)dg) : (T)0;
      r_loc += fabs(xn - xo);
      m_loc += xn;
      if (dg == 0) dm_loc += xn;
      if constexpr (M == kSync) cout[(size_t)p * kQ + lane] = cn;
      else if constexpr (M == kAsync) st_q(cout + (size_t)p * kQ + lane, cn);
      else if constexpr (SH) shadow[(size_t)v * kQ + lane] = cn;
    }
    // outside the branch, so that the slot (written by lane 0) and the count
    // are the same for the whole wavefront; a frozen lane stores nothing
    if constexpr (lds) ls.push(p, cn, per, cout, lane, live);
    else if constexpr (SH)
      sw.staged(tile_v, a.g.cpos, shadow, cout, cur_t, v, tile_v[cur_t + 1] - tile_v[cur_t] == 1, per_rows, wv,
                lane, live);
  };

  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t v0 = tile_v[t], v1 = tile_v[t + 1], nv = v1 - v0;
    cur_t = t;
    if (nv == 1) {
      const uint32_t e0 = in_ptr[v0], e1 = in_ptr[v1];
      s_hub[wv][lane] = pull_edges<M, T>(a.g.in_src, cin, e0, e1, wv, kWG / 64, lane);
      __syncthreads();
      if (wv == 0) update(v0, s_hub[0][lane] + s_hub[1][lane] + s_hub[2][lane] + s_hub[3][lane]);
      __syncthreads();
    } else {
      for (uint32_t v = v0 + wv; v < v1; v += kWG / 64)
        update(v, pull_edges<M, T>(a.g.in_src, cin, in_ptr[v], in_ptr[v + 1], 0, 1, lane));
    }
    if (M == kDelayed && t + 1 == t1) {  // the end of the block
      if constexpr (lds) ls.flush(cout, lane, live);
      else sw.finish(tile_v, a.g.cpos, shadow, cout, t1, wv, lane, live);
    }
  }

  // Per-query partials of this worker, then the last worker of the batch
  // folds them in worker order.
  red(0, wv) = r_loc;
  red(1, wv) = dm_loc;
  red(2, wv) = m_loc;
  __syncthreads();
  double* part = a.part + ((size_t)w * NB + b) * 3 * kQ;
  if (wv == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) part[j * kQ + lane] = red(j, 0) + red(j, 1) + red(j, 2) + red(j, 3);
  }
  __threadfence();
  __syncthreads();
  // worker counter: per sweep (call mode) or a two-slot ring (serving)
  uint32_t* cnt = a.count + (size_t)(a.bactive ? (k & 1u) : k) * NB + b;
  if (tid == 0) s_last = (atomicAdd(cnt, 1u) == P - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  {
    // The batch's last worker folds the P workers' partials: wavefront wv
    // takes workers wv, wv + 4, ... in order, kFoldU at a time so that their
    // loads are in flight together (one at a time, the fold was P round trips
    // long), and wavefront 0 adds the four sums in wavefront order.  The
    // order is fixed, so the sums do not depend on which worker came last.
    constexpr uint32_t W = kWG / 64, kFoldU = 4;
    auto part_at = [&](uint32_t i, uint32_t j) {
      return __hip_atomic_load(a.part + ((size_t)i * NB + b) * 3 * kQ + j * kQ + lane, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    };
    double f[3] = {0.0, 0.0, 0.0};
    uint32_t i = wv;
    for (; i + (kFoldU - 1) * W < P; i += kFoldU * W) {
      double v[3][kFoldU];
#pragma unroll
      for (uint32_t u = 0; u < kFoldU; ++u)
#pragma unroll
        for (uint32_t j = 0; j < 3; ++j) v[j][u] = part_at(i + u * W, j);
#pragma unroll
      for (uint32_t u = 0; u < kFoldU; ++u)
#pragma unroll
        for (uint32_t j = 0; j < 3; ++j) f[j] += v[j][u];
    }
    for (; i < P; i += W)
#pragma unroll
      for (uint32_t j = 0; j < 3; ++j) f[j] += part_at(i, j);
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j) red(j, wv) = f[j];
  }
  __syncthreads();
  if (wv == 0) {
    const double r = red(0, 0) + red(0, 1) + red(0, 2) + red(0, 3);
    const double dm = red(1, 0) + red(1, 1) + red(1, 2) + red(1, 3);
    const double ms = red(2, 0) + red(2, 1) + red(2, 2) + red(2, 3);
    // A live query's mass is at least 1 - alpha > 0 (the restart term).
    const size_t next = ((size_t)((k + 1) & 1u) * NB + b) * kQ + lane;
    // The dangling mass itself, not the deficit 1 - (non-dangling mass): with
    // a one-hot restart the deficit would put a negative rank-one term on a
    // single row, and asynchronous sweeps of that operator can diverge.
    a.dang[next] = live ? dm / ms : D;
    a.scale[next] = live ? S * ms : S;
    if (live) {
      bool stop = !(r >= a.tol);
      if (!stop && a.rhist) {
        // float32 stall rule: the change of sweep k-2 is in this ring slot
        stop = r < kStallTols * a.tol && r > kStallRatio * a.rhist[ring];
        a.rhist[ring] = r;
      }
      if (stop) a.qdone[(size_t)b * kQ + lane] = k + 1;
    }
    // batch residual: the largest change among the queries still live
    double m = live ? r : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double u = __shfl_xor(m, o, 64);
      m = u > m ? u : m;
    }
    if (a.bactive) {
      // serving: clear the ring slot the next sweep counts in
      if (lane == 0) a.count[(size_t)((k + 1) & 1u) * NB + b] = 0;
    } else if (lane == 0) {
      a.resid[(k + 1) * NB + b] = m;
      if (a.hresid) st_host(a.hresid + (k + 1) * NB + b, m);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void mppr_init_kernel(T* x, T* c0, T* c1, const uint32_t* out_deg,
                                                        const uint32_t* cpos, const uint32_t* src, uint32_t nq,
                                                        uint32_t n, uint32_t K, uint32_t NB, double* dang) {
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  const size_t per_batch = (size_t)n * kQ;
  if (i >= per_batch * NB) return;
  const uint32_t b = (uint32_t)(i / per_batch);
  const uint32_t v = (uint32_t)((i % per_batch) / kQ), q = (uint32_t)(i % kQ);
  const uint32_t qi = b * kQ + q;
  const bool at_src = qi < nq && src[qi] == v;
  const uint32_t dg = out_deg[v];
  x[(size_t)b * n * kQ + (size_t)v * kQ + q] = at_src ? (T)1 : (T)0;
  const T c = (at_src && dg) ? (T)(1.0 / (double)dg) : (T)0;
  const size_t off = (size_t)b * (n + K) * kQ + (size_t)cpos[v] * kQ + q;
  c0[off] = c;
  if (c1) c1[off] = c;
  if (at_src) dang[(size_t)b * kQ + q] = dg ? 0.0 : 1.0;  // dangling mass of x0 = e_s
}

// Per-query sums of the stored scores in a fixed order, so that a row's
// normalisation does not depend on scheduling: kSumBlocks partials per batch
// (waves combined in LDS in wave order), then one fold in block order.
constexpr uint32_t kSumBlocks = 256;

template <typename T>
__global__ __launch_bounds__(kWG) void mppr_sum_kernel(const T* x, uint32_t n, double* qpart) {
  __shared__ double s[kWG / 64][kQ];
  const uint32_t b = blockIdx.y, lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const T* xb = x + (size_t)b * n * kQ;
  double acc = 0.0;
  for (uint32_t v = blockIdx.x * (kWG / 64) + wv; v < n; v += kSumBlocks * (kWG / 64)) acc += (double)xb[(size_t)v * kQ + lane];
  s[wv][lane] = acc;
  __syncthreads();
  if (wv == 0) qpart[((size_t)b * kSumBlocks + blockIdx.x) * kQ + lane] = s[0][lane] + s[1][lane] + s[2][lane] + s[3][lane];
}

__global__ __launch_bounds__(kQ) void mppr_fold_kernel(const double* qpart, double* qsum) {
  const uint32_t b = blockIdx.x, lane = threadIdx.x;
  double acc = 0.0;
  for (uint32_t i = 0; i < kSumBlocks; ++i) acc += qpart[((size_t)b * kSumBlocks + i) * kQ + lane];
  qsum[(size_t)b * kQ + lane] = acc;
}

// row q of the output = stored scores of query q / their sum (the storage
// scale cancels)
template <typename T>
__global__ __launch_bounds__(kWG) void mppr_out_kernel(const T* x, const double* qsum, uint32_t n, uint32_t nq,
                                                       double* out) {
  __shared__ double s[64][65];
  const uint32_t b = blockIdx.y, vb = blockIdx.x * 64;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const T* xb = x + (size_t)b * n * kQ;
  for (uint32_t r = wv; r < 64; r += kWG / 64) {
    const uint32_t v = vb + r;
    s[r][lane] = v < n ? (double)xb[(size_t)v * kQ + lane] : 0.0;
  }
  __syncthreads();
  for (uint32_t r = wv; r < 64; r += kWG / 64) {
    const uint32_t qi = b * kQ + r, v = vb + lane;
    if (qi < nq && v < n) out[(size_t)qi * n + v] = s[lane][r] / qsum[(size_t)b * kQ + r];
  }
}

// ------------------------------------------------ serving: lane set-up --
//
// lane_src[b * 64 + q] is the source (restart vertex) of a query admitted
// into lane q of batch b at this sweep boundary, or kInf for lanes left as
// they are; grid.y walks the list of batches that admit anything.

__global__ __launch_bounds__(kWG) void mbf_lane_init_kernel(uint32_t* d0, uint32_t* d1, const uint32_t* cpos,
                                                            uint32_t n, uint32_t K, const uint32_t* lane_src,
                                                            const uint32_t* blist) {
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= (size_t)n * kQ) return;
  const uint32_t b = blist[blockIdx.y];
  const uint32_t v = (uint32_t)(i / kQ), q = (uint32_t)(i % kQ);
  const uint32_t s = lane_src[(size_t)b * kQ + q];
  if (s == kInf) return;
  const size_t off = (size_t)b * (n + K) * kQ + (size_t)cpos[v] * kQ + q;
  const uint32_t val = s == v ? 0u : kInf;
  d0[off] = val;
  if (d1) d1[off] = val;
}

template <typename T>
__global__ __launch_bounds__(kWG) void mppr_lane_init_kernel(T* x, T* c0, T* c1, const uint32_t* out_deg,
                                                             const uint32_t* cpos, uint32_t n, uint32_t K,
                                                             const uint32_t* lane_src, const uint32_t* blist) {
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  if (i >= (size_t)n * kQ) return;
  const uint32_t b = blist[blockIdx.y];
  const uint32_t v = (uint32_t)(i / kQ), q = (uint32_t)(i % kQ);
  const uint32_t s = lane_src[(size_t)b * kQ + q];
  if (s == kInf) return;
  const bool at = s == v;
  const uint32_t dg = out_deg[v];
  x[(size_t)b * n * kQ + (size_t)v * kQ + q] = at ? (T)1 : (T)0;
  const T c = (at && dg) ? (T)(1.0 / (double)dg) : (T)0;
  const size_t off = (size_t)b * (n + K) * kQ + (size_t)cpos[v] * kQ + q;
  c0[off] = c;
  if (c1) c1[off] = c;
}

// Per-lane scalars of admitted PPR queries: restart vertex, unit scale and
// the dangling mass of x0 = e_s in both ring slots, running.
__global__ __launch_bounds__(kWG) void mppr_lane_scalars_kernel(const uint32_t* lane_src, const uint32_t* out_deg,
                                                                uint32_t NB, uint32_t* src, double* dang,
                                                                double* scale, uint32_t* qdone, double* rhist) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= NB * kQ) return;
  const uint32_t s = lane_src[i];
  if (s == kInf) return;
  src[i] = s;
  const double d0 = out_deg[s] ? 0.0 : 1.0;
  dang[i] = d0;
  dang[(size_t)NB * kQ + i] = d0;
  scale[i] = 1.0;
  scale[(size_t)NB * kQ + i] = 1.0;
  qdone[i] = 0;
  if (rhist) {
    rhist[i] = __builtin_inf();
    rhist[(size_t)NB * kQ + i] = __builtin_inf();
  }
}

// Row of one finished query: distances in vertex order.
__global__ __launch_bounds__(kWG) void mbf_lane_out_kernel(const uint32_t* d, const uint32_t* cpos, uint32_t n,
                                                           uint32_t K, uint32_t b, uint32_t q, uint32_t* out) {
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v >= n) return;
  out[v] = d[(size_t)b * (n + K) * kQ + (size_t)cpos[v] * kQ + q];
}

// Row of one finished PPR query normalised to sum 1: kSumBlocks partial sums
// in a fixed order, then every block folds them in block order and scales.
template <typename T>
__global__ __launch_bounds__(kWG) void mppr_lane_sum_kernel(const T* x, uint32_t n, uint32_t b, uint32_t q,
                                                            double* qpart) {
  __shared__ double s[kWG / 64];
  const T* xb = x + (size_t)b * n * kQ;
  double acc = 0.0;
  for (uint32_t v = blockIdx.x * kWG + threadIdx.x; v < n; v += kSumBlocks * kWG) acc += (double)xb[(size_t)v * kQ + q];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63u) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) qpart[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

template <typename T>
__global__ __launch_bounds__(kWG) void mppr_lane_out_kernel(const T* x, uint32_t n, uint32_t b, uint32_t q,
                                                            const double* qpart, double* out) {
  __shared__ double s_sum;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (uint32_t i = 0; i < kSumBlocks; ++i) t += qpart[i];
    s_sum = t;
  }
  __syncthreads();
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v >= n) return;
  out[v] = (double)x[(size_t)b * n * kQ + (size_t)v * kQ + q] / s_sum;
}

__global__ __launch_bounds__(kWG) void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kWG) void fill_f64_kernel(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * kWG + threadIdx.x;
  if (i < n) p[i] = v;
}

inline uint32_t nblocks(size_t n) { return (uint32_t)((n + kWG - 1) / kWG); }

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
  if (n) fill_u32_kernel<<<nblocks(n), kWG, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  if (n) fill_f64_kernel<<<nblocks(n), kWG, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_mbf_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, const uint32_t* src, uint32_t nq,
                           uint32_t n, uint32_t K, uint32_t NB, hipStream_t s) {
  mbf_init_kernel<<<nblocks((size_t)n * kQ * NB), kWG, 0, s>>>(d0, d1, cpos, src, nq, n, K, NB);
  return hipGetLastError();
}

hipError_t launch_mbf_sweep(int mode, const MbfArgs& a, hipStream_t s) {
  const dim3 grid(a.g.P, a.NB);
  if (mode == kSync) mbf_sweep_kernel<kSync, false><<<grid, kWG, 0, s>>>(a);
  else if (mode == kAsync) mbf_sweep_kernel<kAsync, false><<<grid, kWG, 0, s>>>(a);
  else if (a.shadow) mbf_sweep_kernel<kDelayed, true><<<grid, kWG, 0, s>>>(a);
  else mbf_sweep_kernel<kDelayed, false><<<grid, kWG, lds_stage_bytes<uint32_t>(), s>>>(a);
  return hipGetLastError();
}

hipError_t launch_mbf_out(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t K, uint32_t nq, uint32_t NB,
                          uint32_t* out, hipStream_t s) {
  mbf_out_kernel<<<dim3((n + 63) / 64, NB), kWG, 0, s>>>(d, cpos, n, K, nq, out);
  return hipGetLastError();
}

hipError_t launch_mppr_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                            const uint32_t* src, uint32_t nq, uint32_t n, uint32_t K, uint32_t NB, double* dang,
                            hipStream_t s) {
  const uint32_t nb = nblocks((size_t)n * kQ * NB);
  if (f64)
    mppr_init_kernel<double><<<nb, kWG, 0, s>>>(static_cast<double*>(x), static_cast<double*>(c0),
                                                static_cast<double*>(c1), out_deg, cpos, src, nq, n, K, NB, dang);
  else
    mppr_init_kernel<float><<<nb, kWG, 0, s>>>(static_cast<float*>(x), static_cast<float*>(c0),
                                               static_cast<float*>(c1), out_deg, cpos, src, nq, n, K, NB, dang);
  return hipGetLastError();
}

template <typename T>
static void mppr_sweep_dispatch(int mode, const MpprArgs& a, hipStream_t s) {
  const dim3 grid(a.g.P, a.NB);
  if (mode == kSync) mppr_sweep_kernel<kSync, T, false><<<grid, kWG, mppr_dyn_bytes<T, false>(), s>>>(a);
  else if (mode == kAsync) mppr_sweep_kernel<kAsync, T, false><<<grid, kWG, mppr_dyn_bytes<T, false>(), s>>>(a);
  else if (a.shadow) mppr_sweep_kernel<kDelayed, T, true><<<grid, kWG, mppr_dyn_bytes<T, false>(), s>>>(a);
  else mppr_sweep_kernel<kDelayed, T, false><<<grid, kWG, mppr_dyn_bytes<T, true>(), s>>>(a);
}

hipError_t launch_mppr_sweep(int mode, bool f64, const MpprArgs& a, hipStream_t s) {
  if (f64) mppr_sweep_dispatch<double>(mode, a, s);
  else mppr_sweep_dispatch<float>(mode, a, s);
  return hipGetLastError();
}

hipError_t launch_mppr_out(bool f64, const void* x, double* qpart, double* qsum, uint32_t n, uint32_t nq, uint32_t NB,
                           double* out, hipStream_t s) {
  const dim3 gs(kSumBlocks, NB), go((n + 63) / 64, NB);
  if (f64) mppr_sum_kernel<double><<<gs, kWG, 0, s>>>(static_cast<const double*>(x), n, qpart);
  else mppr_sum_kernel<float><<<gs, kWG, 0, s>>>(static_cast<const float*>(x), n, qpart);
  mppr_fold_kernel<<<NB, kQ, 0, s>>>(qpart, qsum);
  if (f64) mppr_out_kernel<double><<<go, kWG, 0, s>>>(static_cast<const double*>(x), qsum, n, nq, out);
  else mppr_out_kernel<float><<<go, kWG, 0, s>>>(static_cast<const float*>(x), qsum, n, nq, out);
  return hipGetLastError();
}

hipError_t launch_mbf_lane_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, uint32_t n, uint32_t K,
                                const uint32_t* lane_src, const uint32_t* blist, uint32_t nb, hipStream_t s) {
  if (nb) mbf_lane_init_kernel<<<dim3(nblocks((size_t)n * kQ), nb), kWG, 0, s>>>(d0, d1, cpos, n, K, lane_src, blist);
  return hipGetLastError();
}

hipError_t launch_mppr_lane_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                                 uint32_t n, uint32_t K, uint32_t NB, const uint32_t* lane_src, const uint32_t* blist,
                                 uint32_t nb, uint32_t* src, double* dang, double* scale, uint32_t* qdone,
                                 double* rhist, hipStream_t s) {
  if (!nb) return hipSuccess;
  const dim3 grid(nblocks((size_t)n * kQ), nb);
  if (f64)
    mppr_lane_init_kernel<double><<<grid, kWG, 0, s>>>(static_cast<double*>(x), static_cast<double*>(c0),
                                                       static_cast<double*>(c1), out_deg, cpos, n, K, lane_src, blist);
  else
    mppr_lane_init_kernel<float><<<grid, kWG, 0, s>>>(static_cast<float*>(x), static_cast<float*>(c0),
                                                      static_cast<float*>(c1), out_deg, cpos, n, K, lane_src, blist);
  mppr_lane_scalars_kernel<<<nblocks((size_t)NB * kQ), kWG, 0, s>>>(lane_src, out_deg, NB, src, dang, scale, qdone,
                                                                     rhist);
  return hipGetLastError();
}

hipError_t launch_mbf_lane_out(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t K, uint32_t b, uint32_t q,
                               uint32_t* out, hipStream_t s) {
  mbf_lane_out_kernel<<<nblocks(n), kWG, 0, s>>>(d, cpos, n, K, b, q, out);
  return hipGetLastError();
}

hipError_t launch_mppr_lane_out(bool f64, const void* x, uint32_t n, uint32_t b, uint32_t q, double* qpart,
                                double* out, hipStream_t s) {
  if (f64) {
    mppr_lane_sum_kernel<double><<<kSumBlocks, kWG, 0, s>>>(static_cast<const double*>(x), n, b, q, qpart);
    mppr_lane_out_kernel<double><<<nblocks(n), kWG, 0, s>>>(static_cast<const double*>(x), n, b, q, qpart, out);
  } else {
    mppr_lane_sum_kernel<float><<<kSumBlocks, kWG, 0, s>>>(static_cast<const float*>(x), n, b, q, qpart);
    mppr_lane_out_kernel<float><<<nblocks(n), kWG, 0, s>>>(static_cast<const float*>(x), n, b, q, qpart, out);
  }
  return hipGetLastError();
}

}  // namespace dg

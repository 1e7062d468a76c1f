// gfx950 kernels for pull-style PageRank and Bellman-Ford sweeps in the three
// commit modes of Blanco, McMillan and Low, "Delayed Asynchronous Iterative
// Graph Algorithms" (section III).
//
// Mapping (the same for both algorithms):
//   * A sweep launches P persistent workgroups ("workers").  Worker w owns a
//     contiguous range of tiles and so a contiguous vertex block (blocked
//     partitioning balanced by in-edges, section III-A) and walks it in
//     ascending vertex order.  Worker ids are spread so that each of the eight
//     XCDs (workgroups are dispatched to XCDs round-robin) owns one contiguous
//     eighth of the vertex range.
//   * A worker is one 1024-thread workgroup.  A tile holds <= 1024 vertices
//     and <= 1024 * EPT - 4 in-edges, or one vertex with more, where EPT is
//     16 (wide variants) or 8 (narrow variant), chosen per graph.  Its edges
//     are processed in chunks of 1024 * EPT slots starting at the tile's
//     first edge rounded down to a multiple of 4: thread t reduces the EPT
//     consecutive slots [EPT t, EPT t + EPT) of the chunk, fetched with
//     16-byte loads of the index stream (and one load of byte weights),
//     then EPT independent gathers.
//     Partial sums (or minima) per vertex go to LDS with ds_add_f64 /
//     ds_min_u32 once per vertex boundary crossed; a single-vertex tile uses a
//     wavefront shuffle reduction and one LDS atomic per wave instead.
//   * Published values (PageRank contributions, distances) live in slot
//     cpos[v]: v itself, or a slot in a compact region after the n regular
//     ones for the sources with the largest out-degree, so that most gathers
//     hit in L2.  The index stream already holds slots, not vertex ids.
//   * In the update phase thread i of the workgroup computes vertex i of the
//     tile and commits it according to the mode:
//       sync     plain store into the output array (double buffer);
//       async    agent-scope store into the single global array at once;
//       delayed  store into a staging buffer; the buffer is copied to the
//                global array with coalesced agent-scope stores when it holds
//                >= d values, when the next tile would overflow it, and when
//                the worker's block is done (section III-B).  The buffer is in
//                LDS for small d and a global per-vertex shadow array for large
//                d, so that big buffers do not cut occupancy.
//     Gathers in async and delayed mode are agent-scope loads so that values
//     committed by workgroups on other XCDs are seen within the same sweep
//     (global reads, section III-C); synchronous gathers are plain cached
//     loads.
//   * Each worker reduces its residual / non-dangling mass (PageRank) or
//     "changed" flag (Bellman-Ford) over its block; the last worker to finish
//     sums the per-worker partials in worker order and publishes the values the
//     next sweep reads, so termination is decided on the device.  The stopping
//     value is also stored into mapped host memory, which the host polls.
#include "dg_device.hpp"
#include "dg_internal.hpp"

namespace dg {
namespace {

__device__ __forceinline__ uint32_t worker_id(uint32_t b, uint32_t P) {
  // Workgroup b runs on XCD b % 8; give each XCD a contiguous slice of workers.
  if ((P & 7u) == 0) return (b & 7u) * (P >> 3) + (b >> 3);
  return b;
}

template <int M, typename T>
__device__ __forceinline__ T ld_shared(const T* p) {
  if constexpr (M == kSync) {
    return *p;
  } else {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t u = __shfl_xor(v, o, 64);
    v = u < v ? u : v;
  }
  return v;
}

// Workgroup barrier for LDS traffic only.  __syncthreads() also issues a
// workgroup release fence, which on this target waits for every outstanding
// global load (vmcnt(0)) and so drains the prefetches and gathers in flight.
// Tile-local hand-offs go through LDS, so waiting for LDS operations
// (lgkmcnt(0)) before the barrier is enough; global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Read-only tables indexed by workgroup-uniform values (tile and worker
// bounds, in-edge offsets at tile ends) are read through the constant
// address space so they become scalar loads, which do not sit in the
// in-order vector-load counter in front of the gathers.
typedef const __attribute__((address_space(4))) uint32_t* const_u32p;
__device__ __forceinline__ const_u32p as_const(const uint32_t* p) { return (const_u32p)(p); }

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s < a ? kInf : s;  // INF + w and overflow both saturate
}

// Largest i in [0, nv) with s_ptr[i] <= e, given s_ptr[0] <= e < s_ptr[nv]:
// the tile-local vertex that owns edge slot e.  A fixed number of halvings
// over s_ptr[min(i, nv)] (which exceeds e from nv on), without branches, so
// that the compiler can interleave its LDS reads with other work; every read
// index is <= nv <= kTileV.
static_assert((kTileV & (kTileV - 1)) == 0, "the owner search halves a power-of-two range");
__device__ __forceinline__ uint32_t owner_of(const uint32_t* s_ptr, uint32_t nv, uint32_t e) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = kTileV / 2; step > 0; step >>= 1) {
    const uint32_t c = lo + step;
    lo = s_ptr[min(c, nv)] <= e ? c : lo;
  }
  return lo;
}

// Owner walk of a thread's window: slot e has just reached `bound` =
// s_ptr[i + 1], so the owner moves to the last vertex whose first slot is e.
// The next two bounds wait in registers (b2 = s_ptr[i + 2], b3 = s_ptr[i + 3],
// read one crossing ahead), so a crossing costs no LDS round trip unless it
// skips two or more vertices without in-edges; then they are read again for
// the next crossing.  Every index read is <= nv: a step is taken only while
// e >= s_ptr[i + 1] and e < s_ptr[nv], i.e. i + 1 < nv.
__device__ __forceinline__ void next_owner(const uint32_t* s_ptr, uint32_t nv, uint32_t e, uint32_t& i,
                                           uint32_t& bound, uint32_t& b2, uint32_t& b3) {
  ++i;
  bound = b2;
  if (e >= bound) {
    ++i;
    bound = b3;
    while (e >= bound) {
      ++i;
      bound = s_ptr[i + 1];
    }
  }
  b2 = s_ptr[min(i + 2, nv)];
  b3 = s_ptr[min(i + 3, nv)];
}

// Buffer resources (raw, stride 0).  A lane whose byte offset lies outside
// [0, bytes) reads 0 and makes no memory access, which masks lanes without
// branches.  dword3 is the raw-buffer format word for this target.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
constexpr uint32_t kOut = 0xFFFFFFFFu;  // an offset that is always out of range
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// EPT consecutive 4-byte words of the in-edge stream for one thread, in
// 16-byte loads.  The window [nb, lim) is rounded up to whole 16-byte groups
// so that each load is entirely inside or outside it.
template <int EPT>
__device__ __forceinline__ void load_win(const uint32_t* stream, uint32_t nb, uint32_t lim, uint32_t tid,
                                         uint32_t (&u)[EPT]) {
  const uint32_t end = (lim + 3u) & ~3u;
  const rsrc_t r = make_rsrc(stream + nb, end > nb ? (end - nb) * 4u : 0u);
#pragma unroll
  for (int q = 0; q < EPT / 4; ++q) {
    const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, tid * (4u * EPT) + 16u * q, 0, 0);
    u[4 * q] = v.x;
    u[4 * q + 1] = v.y;
    u[4 * q + 2] = v.z;
    u[4 * q + 3] = v.w;
  }
}

// A thread's window of EPT edge weights for one chunk, from whichever stream
// the graph keeps.  One-byte weights (W8) stay packed four to a register, as
// one EPT-byte load brought them, and are unpacked where they are used; the
// widened form would hold EPT registers per window, two windows at a time.
template <int EPT, bool W8>
struct WeightWin;

template <int EPT>
struct WeightWin<EPT, true> {
  static_assert(EPT == 8 || EPT == 16, "one 8- or 16-byte load per thread");
  uint32_t q[EPT / 4] = {};
  __device__ __forceinline__ void load(const Topology& g, uint32_t nb, uint32_t lim, uint32_t tid) {
    // window [nb + EPT tid, ...) of the byte stream; nb is 4-byte aligned, as buffer loads need
    const uint32_t end = (lim + (EPT - 1)) & ~(uint32_t)(EPT - 1);
    const rsrc_t r = make_rsrc(g.in_w8 + nb, end > nb ? end - nb : 0u);
    if constexpr (EPT == 16) {
      const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, tid * 16u, 0, 0);
      q[0] = v.x;
      q[1] = v.y;
      q[2] = v.z;
      q[3] = v.w;
    } else {
      const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, tid * 8u, 0, 0);
      q[0] = v.x;
      q[1] = v.y;
    }
  }
  __device__ __forceinline__ uint32_t at(int j) const { return (q[j >> 2] >> (8 * (j & 3))) & 255u; }
};

template <int EPT>
struct WeightWin<EPT, false> {
  uint32_t w[EPT] = {};
  __device__ __forceinline__ void load(const Topology& g, uint32_t nb, uint32_t lim, uint32_t tid) {
    load_win<EPT>(g.in_w, nb, lim, tid, w);
  }
  __device__ __forceinline__ uint32_t at(int j) const { return w[j]; }
};

// Gather of a published value; out-of-range offsets read 0.  Asynchronous
// and delayed sweeps read with the agent-scope coherence bit (sc1), the
// same access an agent-scope relaxed atomic load makes.
template <int M, typename T>
__device__ __forceinline__ T gather(rsrc_t r, uint32_t off) {
  constexpr int pol = (M == kSync) ? 0 : 16;
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, pol));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, pol));
  }
}


// Resident table.  The first `res` slots of the compact region hold the
// published values of the sources with the largest out-degree; each
// workgroup keeps a copy of them in LDS, after its staging buffer, and reads
// a gather of slot n+i from entry i.  Gathers cost L2 requests, which bound
// the sweep; an LDS read costs none.  The copy is filled at the start of the
// sweep (exact for a synchronous sweep, whose input does not change during
// the sweep).  Asynchronous and delayed sweeps refresh one segment of
// kResSegBytes after every tile, so no entry is older than
// ceil(res / segment) tiles of the reader (4 at the default size): the
// segment's loads are issued after the barrier that ends a tile's gathers
// (the chunk registers are free then) and written to LDS after the barrier
// that ends the tile, before the barrier that starts the next tile's gathers.
__host__ __device__ constexpr uint32_t res_offset(uint32_t cap, uint32_t elem) {
  return (cap * (elem + 4u) + 15u) & ~15u;
}

template <int M, typename T>
struct ResTable {
  static constexpr uint32_t kPer = kResSegBytes / (kSweepWG * sizeof(T));  // values per thread per segment
  static constexpr uint32_t kSeg = kPer * kSweepWG;                         // values per segment
  T* lds;
  uint32_t res, n, next = 0;  // next: first value of the segment to refresh
  T r[kPer];
  __device__ __forceinline__ void issue(rsrc_t rc, uint32_t tid) {
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint32_t i = next + j * kSweepWG + tid;
      r[j] = gather<M, T>(rc, i < res ? (n + i) * (uint32_t)sizeof(T) : kOut);
    }
  }
  __device__ __forceinline__ void commit(uint32_t tid) {
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint32_t i = next + j * kSweepWG + tid;
      if (i < res) lds[i] = r[j];
    }
    next += kSeg;
    if (next >= res) next = 0;
  }
  // Whole table, at the start of the sweep (published by the first tile's barrier).
  __device__ __forceinline__ void fill(rsrc_t rc, uint32_t tid) {
    for (next = 0; next < res;) {
      issue(rc, tid);
      commit(tid);
      if (next == 0) break;
    }
  }
};

// ---------------------------------------------------------------- PageRank --

// LOCAL (delayed mode with the per-vertex shadow only): a gather whose source
// is one of this worker's own vertices reads the worker's staged value from
// the shadow instead of the committed array (the local-read variant of
// section III-C).  The shadow holds the newest value of every vertex of the
// block: this sweep's for vertices already updated, else the one committed at
// the end of the previous sweep.  Sources in the compact region are read from
// the committed array.
template <int M, typename T, bool LOCAL, int V>
__global__ __launch_bounds__(kSweepWG) void pr_sweep_kernel(PrArgs a) {
  constexpr int EPT = ept_of(V);
  constexpr uint32_t CH = kSweepWG * EPT;  // edge slots per chunk
  __shared__ uint32_t s_ptr[kTileV + 1];
  __shared__ double s_acc[kTileV];
  __shared__ double s_red[3 * (kSweepWG / 64)];
  __shared__ int s_last;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  T* s_stage = reinterpret_cast<T*>(s_dyn);                         // [cap] values
  uint32_t* s_spos = reinterpret_cast<uint32_t*>(s_dyn + a.cap * sizeof(T));  // [cap] slots

  const uint32_t k = a.k;
  if (!(a.st.resid[k] >= a.tol)) return;  // an earlier sweep met the stopping rule

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u, wv = tid >> 6;
  const uint32_t P = a.g.P;
  const uint32_t w = worker_id(blockIdx.x, P);
  const double inv_n = 1.0 / (double)a.g.n;
  const double alpha = a.alpha;
  // Mass spread uniformly over all vertices: one minus the mass the
  // non-dangling vertices held after the previous sweep.  With total mass 1
  // this is exactly the dangling mass; when an asynchronous sweep leaves the
  // total off 1 it also returns the deficit, so the total-mass error mode
  // decays at once instead of at rate alpha.  The fixed point is unchanged.
  double base = (1.0 - alpha) * inv_n + alpha * a.st.dang[k] * inv_n;
  if (a.wseg) {  // graph sets: the graph's own deficit over its own vertices
    const uint32_t gi = a.wgraph[w];
    base = (1.0 - alpha) * inv_n + alpha * a.gdang[(k & 1u) * a.G + gi] / (double)(a.voff[gi + 1] - a.voff[gi]);
  }
  // Personalised PageRank: no uniform term; the restart vertex gets the
  // teleport and the dangling mass; values are stored at scale S.  For
  // global PageRank S = 1 and the extra term never applies, so the update
  // below is exactly the global one.
  const uint32_t psrc = a.psrc;
  double S = 1.0, extra = 0.0;
  if (psrc != kInf) {
    S = a.st.scale[k];
    extra = (1.0 - alpha) + alpha * a.st.dang[k];
    base = 0.0;
  }
  const double invS = 1.0 / S;
  const T* cin = static_cast<const T*>(a.cin);
  T* cout = static_cast<T*>(a.cout);
  T* x = static_cast<T*>(a.x);
  T* shadow = static_cast<T*>(a.shadow);
  const rsrc_t rc = make_rsrc(cin, (a.g.n + a.g.K) * (uint32_t)sizeof(T));
  ResTable<M, T> rt;
  rt.lds = reinterpret_cast<T*>(s_dyn + res_offset(M == kDelayed ? a.cap : 0u, sizeof(T)));
  rt.res = a.res;
  rt.n = a.g.n;
  // Graph sets: a worker of a graph that already met tol has nothing to do.
  const bool frozen = a.wseg && a.gsweeps[a.wgraph[w]] != 0;
  if (rt.res && !frozen) rt.fill(rc, tid);

  double r_loc = 0.0, nd_loc = 0.0, m_loc = 0.0;
  const const_u32p tile_v = as_const(a.g.tile_v);
  const uint32_t t0 = as_const(a.g.work_t)[w], t1 = frozen ? t0 : as_const(a.g.work_t)[w + 1];
  const uint32_t n = a.g.n;
  uint32_t staged = 0;
  const uint32_t bv0 = tile_v[t0], bv1 = tile_v[t1];  // this worker's vertex block

  // Offsets of the first tile; later tiles' offsets are prefetched into
  // registers while the previous tile's gathers are in flight.
  uint32_t v0 = tile_v[t0];
  // Indices of the next chunk to gather.  They are always loaded one chunk
  // ahead (software pipelining): while a chunk's gathers are in flight the
  // following chunk's indices, of this tile or of the worker's next tile,
  // are already on their way.
  uint32_t u[EPT];
  // Per-vertex inputs of a tile's update phase (old score, out-degree, slot)
  // and the next tile's offsets are loaded during the previous tile's last
  // chunk, next to the index prefetch, with branch-free clamped loads.
  T xo_n = static_cast<T>(0);
  uint32_t dg_n = 0, p_n = 0, nxt = 0, nxt_end = 0;
  if (t0 < t1) {
    const uint32_t nv0 = tile_v[t0 + 1] - v0;
    if (tid <= nv0) s_ptr[tid] = a.g.in_ptr[v0 + tid];
    if (tid == 0 && nv0 == kTileV) s_ptr[kTileV] = a.g.in_ptr[v0 + kTileV];
    const uint32_t b0 = as_const(a.g.in_ptr)[v0] & ~3u;
    load_win<EPT>(a.g.in_src, b0, as_const(a.g.in_ptr)[tile_v[t0 + 1]], tid, u);
    const uint32_t vi = min(v0 + tid, n - 1);
    xo_n = x[vi];
    dg_n = a.g.out_deg[vi];
    p_n = a.g.cpos[vi];
  }
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t v1 = tile_v[t + 1], nv = v1 - v0;
    const bool more = t + 1 < t1;
    const uint32_t nvn = more ? tile_v[t + 2] - v1 : 0u;
    const T xo = xo_n;
    const uint32_t dg = dg_n, p = p_n;
    const uint32_t ee_next = as_const(a.g.in_ptr)[v1 + nvn];  // last edge of the next tile
    // Loads for the next tile; issued right after the index prefetch of
    // this tile's last chunk (or here when the tile has no edges).
    auto prefetch_next = [&]() {
      const uint32_t vi = min(v1 + tid, n - 1);
      xo_n = x[vi];
      dg_n = a.g.out_deg[vi];
      p_n = a.g.cpos[vi];
      nxt = a.g.in_ptr[min(v1 + tid, n)];
      nxt_end = ee_next;
    };
    // Delayed mode: this tile ends with a commit of the staged values.
    const bool flush = M == kDelayed && (!more || staged + nv >= a.d || (!shadow && staged + nv + nvn > a.cap));
    // Refresh a segment of the resident table for the next tile.
    const bool refresh = M != kSync && rt.res && more;
    if (tid < nv) s_acc[tid] = 0.0;
    lds_barrier();
    const uint32_t eb = s_ptr[0], ee = s_ptr[nv];
    for (uint32_t cb = eb & ~3u; cb < ee; cb += CH) {
      const uint32_t e0 = cb + tid * EPT;
      const bool active = (e0 < ee) && (e0 + EPT > eb);
      // Branch-free: slots outside the tile, and slots in the resident table,
      // read 0 without a memory access.  A table slot's value comes from LDS
      // into the same register: in the wide variant right after its gather is
      // issued (the LDS read then waits for the loads before it, which paces
      // the wave's gathers), else once all of the chunk's gathers are in
      // flight (see SweepVariant).
      T raw[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const bool ok = (e0 + j >= eb) & (e0 + j < ee);
        const uint32_t ri = u[j] - n;  // resident index (wraps for regular slots)
        const bool inres = ok & (ri < rt.res);
        if constexpr (LOCAL) {
          const bool loc = ok & (u[j] >= bv0) & (u[j] < bv1);
          raw[j] = gather<M, T>(rc, (ok & !loc & !inres) ? u[j] * (uint32_t)sizeof(T) : kOut);
          if (loc) raw[j] = shadow[u[j]];
        } else {
          raw[j] = gather<M, T>(rc, (ok & !inres) ? u[j] * (uint32_t)sizeof(T) : kOut);
        }
        if constexpr (!all_in_flight(V)) {
          if (inres) raw[j] = rt.lds[ri];
        }
      }
      if constexpr (all_in_flight(V)) {
        if (rt.res) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) {
            const uint32_t ri = u[j] - n;
            const bool inres = (e0 + j >= eb) & (e0 + j < ee) & (ri < rt.res);
            const T r = rt.lds[inres ? ri : 0u];
            raw[j] = inres ? r : raw[j];
          }
        }
      }
      // The owner of the window's first slot, searched while the gathers are
      // in flight.
      const uint32_t es = e0 > eb ? e0 : eb;
      const uint32_t i0 = (nv > 1 && active) ? owner_of(s_ptr, nv, es) : 0u;
      // Prefetch the next chunk's indices: the next chunk of this tile, else
      // the first chunk of the next tile (its window starts at this tile's
      // last edge rounded down), else nothing.
      const bool last = cb + CH >= ee;
      const uint32_t nb = !last ? cb + CH : (more ? (ee & ~3u) : cb);
      const uint32_t lim = !last ? ee : (more ? ee_next : cb);
      load_win<EPT>(a.g.in_src, nb, lim, tid, u);
      if (last) prefetch_next();
      double val[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) val[j] = (double)raw[j];
      if (nv == 1) {
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) q += val[j];
        q = wave_sum(q);
        if (lane == 0) atomicAdd(&s_acc[0], q);
      } else if (active) {
        const uint32_t en = (e0 + EPT < ee) ? e0 + EPT : ee;
        uint32_t i = i0;
        uint32_t bound = s_ptr[i + 1], b2 = s_ptr[min(i + 2, nv)], b3 = s_ptr[min(i + 3, nv)];
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const uint32_t e = e0 + j;
          if (e >= es && e < en) {
            if (e >= bound) {
              atomicAdd(&s_acc[i], part);
              part = 0.0;
              next_owner(s_ptr, nv, e, i, bound, b2, b3);
            }
            part += val[j];
          }
        }
        atomicAdd(&s_acc[i], part);
      }
    }
    if (eb >= ee) {
      // A tile without in-edges ran no chunk: fetch the next tile's window here.
      if (more) load_win<EPT>(a.g.in_src, ee & ~3u, ee_next, tid, u);
      prefetch_next();
    }
    lds_barrier();
    if (refresh) rt.issue(rc, tid);
    if (tid < nv) {
      const uint32_t v = v0 + tid;
      const double xn = base + alpha * s_acc[tid] * invS + (v == psrc ? extra : 0.0);
      x[v] = static_cast<T>(xn * S);
      const T cn = dg ? static_cast<T>(xn * S / (double)dg) : static_cast<T>(0);
      // Change of the score: new value before rounding to storage minus the
      // stored old value (in float64 both are the same value).
      r_loc += fabs(xn - (double)xo * invS);
      if (dg != 0) nd_loc += xn;
      m_loc += xn;
      if constexpr (M == kSync) {
        cout[p] = cn;
      } else if constexpr (M == kAsync) {
        st_agent(cout + p, cn);
      } else if (shadow) {
        shadow[v] = cn;
      } else {
        s_stage[staged + tid] = cn;
        s_spos[staged + tid] = p;
      }
    }
    if constexpr (M == kDelayed) {
      staged += nv;
      if (flush) {
        if (shadow) __syncthreads(); else lds_barrier();
        if (shadow) {
          const uint32_t f0 = v1 - staged;
          for (uint32_t i = tid; i < staged; i += kSweepWG) st_agent(cout + a.g.cpos[f0 + i], shadow[f0 + i]);
        } else {
          for (uint32_t i = tid; i < staged; i += kSweepWG) st_agent(cout + s_spos[i], s_stage[i]);
        }
        staged = 0;
      }
    }
    // Local reads of the next tile must see this tile's shadow stores, which
    // needs the full barrier (it waits for outstanding global stores).
    if constexpr (LOCAL) __syncthreads(); else lds_barrier();
    if (refresh) rt.commit(tid);  // every wave is past this tile's gathers
    if (more) {
      if (tid < nvn) s_ptr[tid] = nxt;
      if (tid == 0) s_ptr[nvn] = nxt_end;
    }
    v0 = v1;
  }

  // Worker partials, then the last worker folds them in worker order.
  r_loc = wave_sum(r_loc);
  nd_loc = wave_sum(nd_loc);
  m_loc = wave_sum(m_loc);
  constexpr uint32_t NW = kSweepWG / 64;  // wavefronts per workgroup
  if (lane == 0) {
    s_red[wv] = r_loc;
    s_red[NW + wv] = nd_loc;
    s_red[2 * NW + wv] = m_loc;
  }
  __syncthreads();
  if (tid == 0) {
    double r_w = 0.0, nd_w = 0.0, m_w = 0.0;  // in wavefront order
    for (uint32_t i = 0; i < NW; ++i) {
      r_w += s_red[i];
      nd_w += s_red[NW + i];
      m_w += s_red[2 * NW + i];
    }
    a.st.part[w] = r_w;
    if (!frozen) {
      a.st.part[P + w] = nd_w;
      a.st.part[2 * P + w] = m_w;
    }
    __threadfence();
    const uint32_t prev = atomicAdd(&a.st.count[k], 1u);
    s_last = (prev == P - 1);
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    auto part = [&](uint32_t i) {
      return __hip_atomic_load(a.st.part + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    double r = 0.0, dd = 0.0, mm = 0.0;
    if (!a.wseg) {
      for (uint32_t i = tid; i < P; i += kSweepWG) r += part(i);
      if (psrc != kInf)
        for (uint32_t i = tid; i < P; i += kSweepWG) mm += part(2 * P + i);
    } else {
      // Graph sets: each graph's change relative to its own mass (its L1
      // change once normalised); the sweep's value is the largest of them.
      for (uint32_t gi = tid; gi < a.G; gi += kSweepWG) {
        double rg = 0.0, ng = 0.0, mg = 0.0;
        const uint32_t i1 = a.wseg[gi + 1];
        for (uint32_t i = a.wseg[gi]; i < i1; i += 8) {
          // eight loads in flight, then the sums in worker order
          double vr[8], vn[8], vm[8];
#pragma unroll
          for (uint32_t j = 0; j < 8; ++j) {
            vr[j] = i + j < i1 ? part(i + j) : 0.0;
            vn[j] = i + j < i1 ? part(P + i + j) : 0.0;
            vm[j] = i + j < i1 ? part(2 * P + i + j) : 0.0;
          }
#pragma unroll
          for (uint32_t j = 0; j < 8; ++j) {
            rg += vr[j];
            ng += vn[j];
            mg += vm[j];
          }
        }
        const double q = rg / mg;
        r = q > r ? q : r;
        if (q < a.tol && a.gsweeps[gi] == 0) a.gsweeps[gi] = k + 1;
        a.gdang[((k + 1) & 1u) * a.G + gi] = (double)(a.voff[gi + 1] - a.voff[gi]) * inv_n - ng;
      }
    }
    for (uint32_t i = tid; i < P; i += kSweepWG) dd += part(P + i);
    if (!a.wseg) {
      r = wave_sum(r);
    } else {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(r, o, 64);
        r = t > r ? t : r;
      }
    }
    dd = wave_sum(dd);
    mm = wave_sum(mm);
    if (lane == 0) {
      s_red[wv] = r;
      s_red[NW + wv] = dd;
      s_red[2 * NW + wv] = mm;
    }
    __syncthreads();
    if (tid == 0) {
      double r_all = 0.0, r_max = 0.0, d_all = 0.0, m_all = 0.0;
      for (uint32_t i = 0; i < NW; ++i) {
        r_all += s_red[i];
        r_max = fmax(r_max, s_red[i]);
        d_all += s_red[NW + i];
        m_all += s_red[2 * NW + i];
      }
      double r_k = !a.wseg ? r_all : r_max;
      // Float32 personalised PageRank: a change below kStallTols x tol that
      // no longer shrinks over two sweeps is the rounding floor; it is
      // recorded negated, which stops the call like a change below tol.
      if constexpr (sizeof(T) == 4) {
        if (psrc != kInf && r_k >= a.tol && r_k < kStallTols * a.tol && r_k > kStallRatio * a.st.resid[k - 1 + (k == 0)])
          r_k = -r_k;
      }
      a.st.resid[k + 1] = r_k;
      if (psrc == kInf) {
        a.st.dang[k + 1] = 1.0 - d_all;
      } else {
        // the dangling mass itself (not the deficit), then the rescale to
        // mass 1: the new iterate's true values are its stored ones / (S m)
        a.st.dang[k + 1] = (m_all - d_all) / m_all;
        a.st.scale[k + 1] = S * m_all;
      }
      if (a.st.hresid) st_host(a.st.hresid + k + 1, r_k);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void pr_init_kernel(T* x, T* c0, T* c1, const uint32_t* out_deg,
                                                      const uint32_t* cpos, uint32_t n, SweepState st, uint32_t S,
                                                      double d0, uint32_t psrc) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  const double x0 = psrc == kInf ? 1.0 / (double)n : (i == psrc ? 1.0 : 0.0);
  if (i < n) {
    const uint32_t dg = out_deg[i];
    const T c = dg ? static_cast<T>(x0 / (double)dg) : static_cast<T>(0);
    const uint32_t p = cpos[i];
    x[i] = static_cast<T>(x0);
    c0[p] = c;
    if (c1) c1[p] = c;
  }
  if (i <= S) {
    st.resid[i] = (i == 0) ? __builtin_inf() : 0.0;
    st.dang[i] = (i == 0) ? d0 : 0.0;
    st.count[i] = 0;
    st.changed[i] = (i == 0) ? 1u : 0u;
    if (st.scale) st.scale[i] = 1.0;
  }
}

// ------------------------------------------------------------ Bellman-Ford --

// LOCAL: as for pr_sweep_kernel, reads of this worker's own vertices come
// from its shadow (delayed mode with the per-vertex shadow only).
// W8: the graph keeps its weights as bytes (in_w8), else as 4-byte words.
template <int M, bool LOCAL, int V, bool W8>
__global__ __launch_bounds__(kSweepWG) void bf_sweep_kernel(BfArgs a) {
  constexpr int EPT = ept_of(V);
  constexpr uint32_t CH = kSweepWG * EPT;  // edge slots per chunk
  __shared__ uint32_t s_ptr[kTileV + 1];
  __shared__ uint32_t s_acc[kTileV];
  extern __shared__ __align__(16) unsigned char s_dyn[];
  uint32_t* s_stage = reinterpret_cast<uint32_t*>(s_dyn);       // [cap] values
  uint32_t* s_spos = s_stage + a.cap;                           // [cap] slots

  const uint32_t k = a.k;
  if (a.st.changed[k] == 0) return;  // an earlier sweep made no update

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t w = worker_id(blockIdx.x, a.g.P);
  const uint32_t* din = a.din;
  uint32_t* dout = a.dout;
  const rsrc_t rd = make_rsrc(din, (a.g.n + a.g.K) * 4u);
  const const_u32p tile_v = as_const(a.g.tile_v);
  // Graph sets: a worker of a graph that already settled has nothing to do.
  const bool frozen = a.wseg && a.gsweeps[a.wgraph[w]] != 0;
  const uint32_t t0 = as_const(a.g.work_t)[w], t1 = frozen ? t0 : as_const(a.g.work_t)[w + 1];
  const uint32_t n = a.g.n;
  uint32_t staged = 0;
  int any = 0;
  ResTable<M, uint32_t> rt;
  rt.lds = reinterpret_cast<uint32_t*>(s_dyn + res_offset(M == kDelayed ? a.cap : 0u, 4u));
  rt.res = a.res;
  rt.n = n;
  if (rt.res && !frozen) rt.fill(rd, tid);
  const uint32_t bv0 = tile_v[t0], bv1 = tile_v[t1];  // this worker's vertex block

  uint32_t v0 = tile_v[t0];
  uint32_t u[EPT];  // next chunk's indices and weights, loaded one chunk ahead
  WeightWin<EPT, W8> wt;
  uint32_t p_n = 0, nxt = 0, nxt_end = 0;
  if (t0 < t1) {
    const uint32_t nv0 = tile_v[t0 + 1] - v0;
    if (tid <= nv0) s_ptr[tid] = a.g.in_ptr[v0 + tid];
    if (tid == 0 && nv0 == kTileV) s_ptr[kTileV] = a.g.in_ptr[v0 + kTileV];
    const uint32_t b0 = as_const(a.g.in_ptr)[v0] & ~3u;
    const uint32_t l0 = as_const(a.g.in_ptr)[tile_v[t0 + 1]];
    load_win<EPT>(a.g.in_src, b0, l0, tid, u);
    wt.load(a.g, b0, l0, tid);
    p_n = a.g.cpos[min(v0 + tid, n - 1)];
  }
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t v1 = tile_v[t + 1], nv = v1 - v0;
    const bool more = t + 1 < t1;
    const uint32_t nvn = more ? tile_v[t + 2] - v1 : 0u;
    const uint32_t p = p_n;
    const uint32_t ee_next = as_const(a.g.in_ptr)[v1 + nvn];
    auto prefetch_next = [&]() {
      p_n = a.g.cpos[min(v1 + tid, n - 1)];
      nxt = a.g.in_ptr[min(v1 + tid, n)];
      nxt_end = ee_next;
    };
    const bool flush = M == kDelayed && (!more || staged + nv >= a.d || (!a.shadow && staged + nv + nvn > a.cap));
    const bool refresh = M != kSync && rt.res && more;
    if (tid < nv) s_acc[tid] = kInf;
    lds_barrier();
    const uint32_t eb = s_ptr[0], ee = s_ptr[nv];
    for (uint32_t cb = eb & ~3u; cb < ee; cb += CH) {
      const uint32_t e0 = cb + tid * EPT;
      const bool active = (e0 < ee) && (e0 + EPT > eb);
      bool ok[EPT];
      uint32_t du[EPT];
      const WeightWin<EPT, W8> wc = wt;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        ok[j] = (e0 + j >= eb) & (e0 + j < ee);
        const uint32_t ri = u[j] - n;
        const bool inres = ok[j] & (ri < rt.res);
        if constexpr (LOCAL) {
          const bool loc = ok[j] & (u[j] >= bv0) & (u[j] < bv1);
          du[j] = gather<M, uint32_t>(rd, (ok[j] & !loc & !inres) ? u[j] * 4u : kOut);
          if (loc) du[j] = a.shadow[u[j]];
        } else {
          du[j] = gather<M, uint32_t>(rd, (ok[j] & !inres) ? u[j] * 4u : kOut);
        }
        if constexpr (!all_in_flight(V)) {
          if (inres) du[j] = rt.lds[ri];
        }
      }
      if constexpr (all_in_flight(V)) {
        if (rt.res) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) {
            const uint32_t ri = u[j] - n;
            const bool inres = ok[j] & (ri < rt.res);
            const uint32_t r = rt.lds[inres ? ri : 0u];
            du[j] = inres ? r : du[j];
          }
        }
      }
      // The owner of the window's first slot, searched while the gathers are
      // in flight.
      const uint32_t es = e0 > eb ? e0 : eb;
      const uint32_t i0 = (nv > 1 && active) ? owner_of(s_ptr, nv, es) : 0u;
      const bool last = cb + CH >= ee;
      const uint32_t nb = !last ? cb + CH : (more ? (ee & ~3u) : cb);
      const uint32_t lim = !last ? ee : (more ? ee_next : cb);
      load_win<EPT>(a.g.in_src, nb, lim, tid, u);
      wt.load(a.g, nb, lim, tid);
      if (last) prefetch_next();
      uint32_t cand[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) cand[j] = ok[j] ? sat_add(du[j], wc.at(j)) : kInf;
      if (nv == 1) {
        uint32_t q = kInf;
#pragma unroll
        for (int j = 0; j < EPT; ++j) q = cand[j] < q ? cand[j] : q;
        q = wave_min(q);
        if (lane == 0 && q != kInf) atomicMin(&s_acc[0], q);
      } else if (active) {
        const uint32_t en = (e0 + EPT < ee) ? e0 + EPT : ee;
        uint32_t i = i0;
        uint32_t bound = s_ptr[i + 1], b2 = s_ptr[min(i + 2, nv)], b3 = s_ptr[min(i + 3, nv)];
        uint32_t part = kInf;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const uint32_t e = e0 + j;
          if (e >= es && e < en) {
            if (e >= bound) {
              if (part != kInf) atomicMin(&s_acc[i], part);
              part = kInf;
              next_owner(s_ptr, nv, e, i, bound, b2, b3);
            }
            part = cand[j] < part ? cand[j] : part;
          }
        }
        if (part != kInf) atomicMin(&s_acc[i], part);
      }
    }
    if (eb >= ee) {
      if (more) {
        load_win<EPT>(a.g.in_src, ee & ~3u, ee_next, tid, u);
        wt.load(a.g, ee & ~3u, ee_next, tid);
      }
      prefetch_next();
    }
    lds_barrier();
    if (refresh) rt.issue(rd, tid);
    if (tid < nv) {
      const uint32_t old = ld_shared<M>(din + p);
      const uint32_t best = s_acc[tid];
      const uint32_t nw = best < old ? best : old;
      any |= (nw < old);
      if constexpr (M == kSync) {
        dout[p] = nw;
      } else if constexpr (M == kAsync) {
        st_agent(dout + p, nw);
      } else if (a.shadow) {
        a.shadow[v0 + tid] = nw;
      } else {
        s_stage[staged + tid] = nw;
        s_spos[staged + tid] = p;
      }
    }
    if constexpr (M == kDelayed) {
      staged += nv;
      if (flush) {
        if (a.shadow) __syncthreads(); else lds_barrier();
        if (a.shadow) {
          const uint32_t f0 = v1 - staged;
          for (uint32_t i = tid; i < staged; i += kSweepWG) st_agent(dout + a.g.cpos[f0 + i], a.shadow[f0 + i]);
        } else {
          for (uint32_t i = tid; i < staged; i += kSweepWG) st_agent(dout + s_spos[i], s_stage[i]);
        }
        staged = 0;
      }
    }
    if constexpr (LOCAL) __syncthreads(); else lds_barrier();
    if (refresh) rt.commit(tid);
    if (more) {
      if (tid < nvn) s_ptr[tid] = nxt;
      if (tid == 0) s_ptr[nvn] = nxt_end;
    }
    v0 = v1;
  }
  const int anyb = __syncthreads_or(any);
  if (!a.wseg) {
    if (anyb && tid == 0) {
      st_agent(a.st.changed + k + 1, 1u);
      if (a.st.hchanged) st_host(a.st.hchanged + k + 1, 1u);
    }
    return;
  }
  // Graph sets: per-worker change flags; the last worker folds them per
  // graph, records the graphs that settled, and flags the sweep if any
  // graph changed.
  __shared__ int s_last;
  if (tid == 0) {
    a.st.part[w] = anyb ? 1.0 : 0.0;
    __threadfence();
    s_last = atomicAdd(&a.st.count[k], 1u) == a.g.P - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  int ch_any = 0;
  for (uint32_t gi = tid; gi < a.G; gi += kSweepWG) {
    int ch = 0;
    const uint32_t i1 = a.wseg[gi + 1];
    for (uint32_t i = a.wseg[gi]; i < i1; i += 8) {
      double v[8];  // eight loads in flight
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j)
        v[j] = i + j < i1 ? __hip_atomic_load(a.st.part + i + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) ch |= v[j] != 0.0;
    }
    if (!ch && a.gsweeps[gi] == 0) a.gsweeps[gi] = k + 1;
    ch_any |= ch;
  }
  if (__syncthreads_or(ch_any) && tid == 0) {
    st_agent(a.st.changed + k + 1, 1u);
    if (a.st.hchanged) st_host(a.st.hchanged + k + 1, 1u);
  }
}

__global__ __launch_bounds__(kWG) void bf_init_kernel(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, uint32_t n,
                                                      uint32_t src, SweepState st, uint32_t S) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) {
    const uint32_t v = (i == src) ? 0u : kInf;
    const uint32_t p = cpos[i];
    d0[p] = v;
    if (d1) d1[p] = v;
  }
  if (i <= S) {
    st.resid[i] = 0.0;
    st.dang[i] = 0.0;
    st.count[i] = 0;
    st.changed[i] = (i == 0) ? 1u : 0u;
  }
}

__global__ __launch_bounds__(kWG) void bf_gather_kernel(const uint32_t* d, const uint32_t* cpos, uint32_t n,
                                                        uint32_t* out) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) out[i] = d[cpos[i]];
}

// ----------------------------------------------------------- normalisation --

template <typename T>
__global__ __launch_bounds__(kWG) void sum_blocks_kernel(const T* x, uint32_t n, double* part) {
  __shared__ double s[kWG / 64];
  double acc = 0.0;
  for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) acc += (double)x[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63u) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(kWG) void sum_partials_kernel(double* part, uint32_t nb) {
  __shared__ double s[kWG / 64];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < nb; i += kWG) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63u) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[nb] = s[0] + s[1] + s[2] + s[3];
}

template <typename T>
__global__ __launch_bounds__(kWG) void scale_kernel(const T* x, uint32_t n, const double* total, double* out) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i < n) out[i] = (double)x[i] / *total;
}

// Error certificate of a score vector y (float64, vertex order, sum 1): the
// inputs of one synchronous float64 sweep, which then evaluates T(y) and
// reports ||T(y) - y||_1 as its residual.  x[v] = y[v] (the sweep's old
// score), c[cpos[v]] = y[v] / outdeg(v) (0 for a dangling v), and part[b] =
// the dangling mass in block b's grid-stride share (summed in fixed order).
__global__ __launch_bounds__(kWG) void bound_init_kernel(const double* y, double* x, double* c,
                                                         const uint32_t* out_deg, const uint32_t* cpos, uint32_t n,
                                                         double* part) {
  __shared__ double s[kWG / 64];
  double acc = 0.0;
  for (uint32_t v = blockIdx.x * kWG + threadIdx.x; v < n; v += gridDim.x * kWG) {
    const double yv = y[v];
    const uint32_t dg = out_deg[v];
    x[v] = yv;
    c[cpos[v]] = dg ? yv / (double)dg : 0.0;
    if (dg == 0) acc += yv;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63u) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Sweep state of the certificate sweep (sweep 0 of a fresh row): it runs
// (resid[0] = inf), spreads the dangling mass *dang (= D(y)), and starts its
// worker count at 0.
__global__ void bound_state_kernel(SweepState st, const double* dang) {
  if (threadIdx.x == 0) {
    st.resid[0] = __builtin_inf();
    st.resid[1] = 0.0;
    st.dang[0] = *dang;
    st.count[0] = 0;
    st.count[1] = 0;
    if (st.scale) st.scale[0] = 1.0;
  }
}

// out[v] = c[cpos[v]]: committed values in vertex order (the local-read
// variant starts its shadow from them).
template <typename T>
__global__ __launch_bounds__(kWG) void by_vertex_kernel(const T* c, const uint32_t* cpos, uint32_t n, T* out) {
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v < n) out[v] = c[cpos[v]];
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kWG - 1) / kWG); }

template <int M, typename T>
size_t pr_dyn_lds(const PrArgs& a) {
  return (size_t)res_offset(M == kDelayed ? a.cap : 0u, sizeof(T)) + (size_t)a.res * sizeof(T);
}

}  // namespace

hipError_t launch_pr_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                          uint32_t n, SweepState st, uint32_t S, double d0, uint32_t psrc, hipStream_t s) {
  const uint32_t nb = blocks_for((uint64_t)(n > S + 1 ? n : S + 1));
  if (f64) {
    pr_init_kernel<double><<<nb, kWG, 0, s>>>(static_cast<double*>(x), static_cast<double*>(c0),
                                              static_cast<double*>(c1), out_deg, cpos, n, st, S, d0, psrc);
  } else {
    pr_init_kernel<float><<<nb, kWG, 0, s>>>(static_cast<float*>(x), static_cast<float*>(c0),
                                             static_cast<float*>(c1), out_deg, cpos, n, st, S, d0, psrc);
  }
  return hipGetLastError();
}

// The sweep kernels take more dynamic LDS than the default 64 KB limit; the
// attribute is set once per kernel instance.
template <auto Kernel>
static void allow_dyn_lds() {
  static const bool done = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(Kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kSweepDynLds);
    return true;
  }();
  (void)done;
}

template <int M, typename T, bool LOCAL, int V>
static void pr_sweep_go(const PrArgs& a, hipStream_t s) {
  allow_dyn_lds<pr_sweep_kernel<M, T, LOCAL, V>>();
  pr_sweep_kernel<M, T, LOCAL, V><<<a.g.P, kSweepWG, pr_dyn_lds<M, T>(a), s>>>(a);
}

template <int M, typename T, bool LOCAL>
static void pr_sweep_variant(const PrArgs& a, hipStream_t s) {
  if (a.g.variant == kNarrow) pr_sweep_go<M, T, LOCAL, kNarrow>(a, s);
  else if (a.g.variant == kWideInFlight) pr_sweep_go<M, T, LOCAL, kWideInFlight>(a, s);
  else pr_sweep_go<M, T, LOCAL, kWide>(a, s);
}

hipError_t launch_pr_sweep(int mode, bool f64, const PrArgs& a, hipStream_t s) {
  if (f64) {
    if (mode == kSync) pr_sweep_variant<kSync, double, false>(a, s);
    else if (mode == kAsync) pr_sweep_variant<kAsync, double, false>(a, s);
    else if (mode == kDelayedLocal) pr_sweep_variant<kDelayed, double, true>(a, s);
    else pr_sweep_variant<kDelayed, double, false>(a, s);
  } else {
    if (mode == kSync) pr_sweep_variant<kSync, float, false>(a, s);
    else if (mode == kAsync) pr_sweep_variant<kAsync, float, false>(a, s);
    else if (mode == kDelayedLocal) pr_sweep_variant<kDelayed, float, true>(a, s);
    else pr_sweep_variant<kDelayed, float, false>(a, s);
  }
  return hipGetLastError();
}

hipError_t launch_bound_setup(const double* y, double* x, double* c, const uint32_t* out_deg, const uint32_t* cpos,
                              uint32_t n, SweepState st, double* scratch, hipStream_t s) {
  bound_init_kernel<<<kNormBlocks, kWG, 0, s>>>(y, x, c, out_deg, cpos, n, scratch);
  sum_partials_kernel<<<1, kWG, 0, s>>>(scratch, kNormBlocks);
  bound_state_kernel<<<1, 64, 0, s>>>(st, scratch + kNormBlocks);
  return hipGetLastError();
}

hipError_t launch_by_vertex(bool f64, const void* c, const uint32_t* cpos, uint32_t n, void* out, hipStream_t s) {
  if (f64)
    by_vertex_kernel<double><<<blocks_for(n), kWG, 0, s>>>(static_cast<const double*>(c), cpos, n,
                                                          static_cast<double*>(out));
  else
    by_vertex_kernel<float><<<blocks_for(n), kWG, 0, s>>>(static_cast<const float*>(c), cpos, n,
                                                         static_cast<float*>(out));
  return hipGetLastError();
}

hipError_t launch_bf_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, uint32_t n, uint32_t src,
                          SweepState st, uint32_t S, hipStream_t s) {
  const uint32_t nb = blocks_for((uint64_t)(n > S + 1 ? n : S + 1));
  bf_init_kernel<<<nb, kWG, 0, s>>>(d0, d1, cpos, n, src, st, S);
  return hipGetLastError();
}

hipError_t launch_bf_gather(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t* out, hipStream_t s) {
  bf_gather_kernel<<<blocks_for(n), kWG, 0, s>>>(d, cpos, n, out);
  return hipGetLastError();
}

template <int M, bool LOCAL, int V>
static void bf_sweep_go(const BfArgs& a, size_t lds, hipStream_t s) {
  if (a.g.in_w8) {
    allow_dyn_lds<bf_sweep_kernel<M, LOCAL, V, true>>();
    bf_sweep_kernel<M, LOCAL, V, true><<<a.g.P, kSweepWG, lds, s>>>(a);
  } else {
    allow_dyn_lds<bf_sweep_kernel<M, LOCAL, V, false>>();
    bf_sweep_kernel<M, LOCAL, V, false><<<a.g.P, kSweepWG, lds, s>>>(a);
  }
}

template <int M, bool LOCAL>
static void bf_sweep_variant(const BfArgs& a, size_t lds, hipStream_t s) {
  if (a.g.variant == kNarrow) bf_sweep_go<M, LOCAL, kNarrow>(a, lds, s);
  else if (a.g.variant == kWideInFlight) bf_sweep_go<M, LOCAL, kWideInFlight>(a, lds, s);
  else bf_sweep_go<M, LOCAL, kWide>(a, lds, s);
}

hipError_t launch_bf_sweep(int mode, const BfArgs& a, hipStream_t s) {
  const size_t lds = (size_t)res_offset(mode == kDelayed || mode == kDelayedLocal ? a.cap : 0u, 4u) +
                     (size_t)a.res * sizeof(uint32_t);
  if (mode == kSync) bf_sweep_variant<kSync, false>(a, lds, s);
  else if (mode == kAsync) bf_sweep_variant<kAsync, false>(a, lds, s);
  else if (mode == kDelayedLocal) bf_sweep_variant<kDelayed, true>(a, lds, s);
  else bf_sweep_variant<kDelayed, false>(a, lds, s);
  return hipGetLastError();
}

hipError_t launch_normalize(bool f64, const void* x, uint32_t n, double* out, double* scratch, hipStream_t s) {
  const uint32_t nb = kNormBlocks;
  if (f64) {
    sum_blocks_kernel<double><<<nb, kWG, 0, s>>>(static_cast<const double*>(x), n, scratch);
  } else {
    sum_blocks_kernel<float><<<nb, kWG, 0, s>>>(static_cast<const float*>(x), n, scratch);
  }
  sum_partials_kernel<<<1, kWG, 0, s>>>(scratch, nb);
  if (f64) {
    scale_kernel<double><<<blocks_for(n), kWG, 0, s>>>(static_cast<const double*>(x), n, scratch + nb, out);
  } else {
    scale_kernel<float><<<blocks_for(n), kWG, 0, s>>>(static_cast<const float*>(x), n, scratch + nb, out);
  }
  return hipGetLastError();
}

}  // namespace dg

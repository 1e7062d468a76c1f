// Sets of graphs swept together (many small or uneven graphs on one GPU).
//
// The graphs are laid out as one union graph: vertex ids of graph i start at
// g_voff[i], and tiles (<= 256 vertices, <= 2044 in-edges, or one vertex with
// more) never span two graphs.  One launch of P persistent workgroups runs a
// sweep over every graph still running: each workgroup takes the next tile
// from a global work list (an atomic cursor per sweep), so a graph that has
// converged costs one flag test per tile and the work of the graphs still
// running spreads over the whole GPU.
//
// Within a tile the mapping is the one of the single-graph sweeps: chunks of
// 2048 in-edge slots, eight consecutive slots per thread, a segmented
// reduction into LDS, one thread per vertex in the update phase.  Commit
// modes are those of the paper (section III): synchronous (double buffer),
// asynchronous (agent-scope store at once), delayed (per-vertex shadow copy,
// committed once the workgroup has staged >= d vertices, or 64 tiles, and at
// the end of its sweep).
//
// Each tile leaves its partial reductions in memory; a fold kernel with one
// workgroup per graph then reduces them in tile order (the same result every
// run), applies each graph's stopping rule, and advances the sweep index kept
// on the device.  Because no launch argument changes from sweep to sweep, a
// chunk of sweeps can be captured once into a HIP graph and replayed.
#include "dg_internal.hpp"

namespace dg {
namespace {

constexpr uint32_t kRing = 64;  // tiles a delayed-mode workgroup stages at most

template <int M, typename T>
__device__ __forceinline__ T ld_pub(const T* p) {
  if constexpr (M == kSync) return *p;
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_pub(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wmin(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t u = __shfl_xor(v, o, 64);
    v = u < v ? u : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t sadd(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s < a ? kInf : s;
}

// Largest i in [0, nv) with s_ptr[i] <= e (the tile-local owner of edge e).
__device__ __forceinline__ uint32_t owner(const uint32_t* s_ptr, uint32_t nv, uint32_t e) {
  uint32_t lo = 0, hi = nv;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s_ptr[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// Graph of union vertex v: largest i with g_voff[i] <= v.
__device__ __forceinline__ uint32_t graph_of(const uint32_t* g_voff, uint32_t G, uint32_t v) {
  uint32_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (g_voff[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// Next tile of the work list for the whole workgroup.
__device__ __forceinline__ uint32_t grab(uint32_t* cursor, uint32_t* s_t) {
  if (threadIdx.x == 0) *s_t = atomicAdd(cursor, 1u);
  __syncthreads();
  const uint32_t t = *s_t;
  __syncthreads();
  return t;
}

// Loads the tile's in-edge offsets into LDS (nv + 1 <= 257 entries).
__device__ __forceinline__ void load_ptr(const uint32_t* in_ptr, uint32_t v0, uint32_t nv, uint32_t* s_ptr) {
  const uint32_t tid = threadIdx.x;
  if (tid <= nv) s_ptr[tid] = in_ptr[v0 + tid];
  if (tid == 0 && nv == (uint32_t)kTileV) s_ptr[kTileV] = in_ptr[v0 + kTileV];
}

// ---------------------------------------------------------------- PageRank --

template <int M, typename T>
__global__ __launch_bounds__(kWG) void set_pr_sweep_kernel(SetPrArgs a) {
  __shared__ uint32_t s_ptr[kTileV + 1];
  __shared__ double s_acc[kTileV];
  __shared__ double s_red[2][kWG / 64];
  __shared__ uint32_t s_t;
  __shared__ uint32_t s_ring[kRing];
  const uint32_t k = *a.c.cur;
  if (k >= a.c.S || a.c.live[k] == 0) return;

  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const T* cin = static_cast<const T*>((M == kSync && (k & 1u)) ? a.c1 : a.c0);
  T* cout = static_cast<T*>(M == kSync ? ((k & 1u) ? a.c0 : a.c1) : a.c0);
  T* x = static_cast<T*>(a.x);
  T* shadow = static_cast<T*>(a.shadow);
  const double alpha = a.alpha;
  const SetTopo& g = a.g;
  uint32_t nring = 0, staged = 0;

  for (;;) {
    const uint32_t t = grab(a.c.next + k, &s_t);
    if (t >= g.T) break;
    const uint32_t gi = g.tile_g[t];
    if (a.c.gdone[gi] != 0) continue;
    const uint32_t v0 = g.tile_v[t], nv = g.tile_v[t + 1] - v0;
    const double inv_n = 1.0 / (double)(g.g_voff[gi + 1] - g.g_voff[gi]);
    // teleport plus the spread mass (1 - non-dangling mass of the previous
    // sweep, the same deficit form as the single-graph sweeps)
    const double base = ((1.0 - alpha) + alpha * a.gdang[(size_t)(k & 1u) * g.G + gi]) * inv_n;
    load_ptr(g.in_ptr, v0, nv, s_ptr);
    if (tid < nv) s_acc[tid] = 0.0;
    __syncthreads();
    const uint32_t eb = s_ptr[0], ee = s_ptr[nv];
    for (uint32_t cb = eb; cb < ee; cb += kChunk) {
      const uint32_t e0 = cb + tid * kEPT;
      double val[kEPT];
#pragma unroll
      for (int j = 0; j < kEPT; ++j) {
        const uint32_t e = e0 + j;
        const uint32_t ec = e < ee ? e : ee - 1;  // clamped: all eight gathers issue together
        const double raw = (double)ld_pub<M>(cin + g.in_src[ec]);
        val[j] = e < ee ? raw : 0.0;
      }
      if (nv == 1) {
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < kEPT; ++j) q += val[j];
        q = wsum(q);
        if (lane == 0) atomicAdd(&s_acc[0], q);
      } else if (e0 < ee) {
        uint32_t i = owner(s_ptr, nv, e0);
        uint32_t bound = s_ptr[i + 1];
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < kEPT; ++j) {
          const uint32_t e = e0 + j;
          if (e < ee) {
            if (e >= bound) {
              atomicAdd(&s_acc[i], part);
              part = 0.0;
              do { ++i; bound = s_ptr[i + 1]; } while (e >= bound);
            }
            part += val[j];
          }
        }
        atomicAdd(&s_acc[i], part);
      }
    }
    __syncthreads();
    double r = 0.0, nd = 0.0;
    if (tid < nv) {
      const uint32_t v = v0 + tid;
      const double xn = base + alpha * s_acc[tid];
      const double xo = (double)x[v];
      x[v] = static_cast<T>(xn);
      const uint32_t dg = g.out_deg[v];
      const T cn = dg ? static_cast<T>(xn / (double)dg) : static_cast<T>(0);
      r = fabs(xn - xo);
      if (dg != 0) nd = xn;
      if constexpr (M == kSync) cout[v] = cn;
      else if constexpr (M == kAsync) st_pub(cout + v, cn);
      else shadow[v] = cn;
    }
    r = wsum(r);
    nd = wsum(nd);
    if (lane == 0) {
      s_red[0][wv] = r;
      s_red[1][wv] = nd;
    }
    __syncthreads();
    if (tid == 0) {
      a.tpart[2 * (size_t)t] = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
      a.tpart[2 * (size_t)t + 1] = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
    }
    if constexpr (M == kDelayed) {
      if (tid == 0) s_ring[nring] = t;
      ++nring;
      staged += nv;
      if (staged >= a.d || nring == kRing) {
        __syncthreads();
        for (uint32_t i = 0; i < nring; ++i) {
          const uint32_t f0 = g.tile_v[s_ring[i]], f1 = g.tile_v[s_ring[i] + 1];
          for (uint32_t v = f0 + tid; v < f1; v += kWG) st_pub(cout + v, shadow[v]);
        }
        nring = 0;
        staged = 0;
      }
    }
  }
  if constexpr (M == kDelayed) {
    if (nring) {
      __syncthreads();
      for (uint32_t i = 0; i < nring; ++i) {
        const uint32_t f0 = g.tile_v[s_ring[i]], f1 = g.tile_v[s_ring[i] + 1];
        for (uint32_t v = f0 + tid; v < f1; v += kWG) st_pub(cout + v, shadow[v]);
      }
    }
  }
}

// Closes sweep k for the block's graph and, in the last block, for the set.
__device__ __forceinline__ void close_sweep(const SetCtl& c, uint32_t k) {
  if (threadIdx.x != 0) return;
  __threadfence();
  const uint32_t prev = atomicAdd(c.fcount + k, 1u);
  if (prev == gridDim.x - 1) {
    __threadfence();
    const uint32_t live = __hip_atomic_load(c.live + k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(c.host_live + k + 1, live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    *c.cur = k + 1;
  }
}

__global__ __launch_bounds__(kWG) void set_pr_fold_kernel(SetPrArgs a) {
  __shared__ double s_r[kWG / 64], s_n[kWG / 64];
  const uint32_t gi = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint32_t k = *a.c.cur;
  if (k >= a.c.S) return;
  if (a.c.live[k] != 0 && a.c.gdone[gi] == 0) {
    const uint32_t t0 = a.g.g_toff[gi], t1 = a.g.g_toff[gi + 1];
    double r = 0.0, nd = 0.0;
    for (uint32_t t = t0 + tid; t < t1; t += kWG) {
      r += a.tpart[2 * (size_t)t];
      nd += a.tpart[2 * (size_t)t + 1];
    }
    r = wsum(r);
    nd = wsum(nd);
    if (lane == 0) {
      s_r[wv] = r;
      s_n[wv] = nd;
    }
    __syncthreads();
    if (tid == 0) {
      r = s_r[0] + s_r[1] + s_r[2] + s_r[3];
      nd = s_n[0] + s_n[1] + s_n[2] + s_n[3];
      a.gdang[(size_t)((k + 1) & 1u) * a.g.G + gi] = 1.0 - nd;
      a.gres[gi] = r;
      if (!(r >= a.tol)) a.c.gdone[gi] = k + 1;
      else atomicAdd(a.c.live + k + 1, 1u);
    }
  }
  close_sweep(a.c, k);
}

template <typename T>
__global__ __launch_bounds__(kWG) void set_pr_init_kernel(SetPrArgs a, const double* dang0) {
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v < a.g.G) a.gdang[v] = dang0[v];
  if (v >= a.g.N) return;
  const uint32_t gi = graph_of(a.g.g_voff, a.g.G, v);
  const double x0 = 1.0 / (double)(a.g.g_voff[gi + 1] - a.g.g_voff[gi]);
  const uint32_t dg = a.g.out_deg[v];
  static_cast<T*>(a.x)[v] = static_cast<T>(x0);
  const T c = dg ? static_cast<T>(x0 / (double)dg) : static_cast<T>(0);
  static_cast<T*>(a.c0)[v] = c;
  if (a.c1) static_cast<T*>(a.c1)[v] = c;
}

// One block per graph: sum of its scores in a fixed order, then x / sum.
template <typename T>
__global__ __launch_bounds__(kWG) void set_pr_out_kernel(SetPrArgs a, double* out) {
  __shared__ double s[kWG / 64];
  const uint32_t gi = blockIdx.x, tid = threadIdx.x;
  const uint32_t v0 = a.g.g_voff[gi], v1 = a.g.g_voff[gi + 1];
  const T* x = static_cast<const T*>(a.x);
  double acc = 0.0;
  for (uint32_t v = v0 + tid; v < v1; v += kWG) acc += (double)x[v];
  acc = wsum(acc);
  if ((tid & 63u) == 0) s[tid >> 6] = acc;
  __syncthreads();
  const double sum = s[0] + s[1] + s[2] + s[3];
  for (uint32_t v = v0 + tid; v < v1; v += kWG) out[v] = (double)x[v] / sum;
}

// ------------------------------------------------------------ Bellman-Ford --

template <int M>
__global__ __launch_bounds__(kWG) void set_bf_sweep_kernel(SetBfArgs a) {
  __shared__ uint32_t s_ptr[kTileV + 1];
  __shared__ uint32_t s_min[kTileV];
  __shared__ uint32_t s_t;
  __shared__ uint32_t s_ring[kRing];
  __shared__ uint32_t s_chg;
  const uint32_t k = *a.c.cur;
  if (k >= a.c.S || a.c.live[k] == 0) return;

  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t* din = (M == kSync && (k & 1u)) ? a.c1 : a.c0;
  uint32_t* dout = M == kSync ? ((k & 1u) ? a.c0 : a.c1) : a.c0;
  const SetTopo& g = a.g;
  uint32_t nring = 0, staged = 0;

  for (;;) {
    const uint32_t t = grab(a.c.next + k, &s_t);
    if (t >= g.T) break;
    const uint32_t gi = g.tile_g[t];
    if (a.c.gdone[gi] != 0) continue;
    const uint32_t v0 = g.tile_v[t], nv = g.tile_v[t + 1] - v0;
    load_ptr(g.in_ptr, v0, nv, s_ptr);
    if (tid < nv) s_min[tid] = kInf;
    if (tid == 0) s_chg = 0;
    __syncthreads();
    const uint32_t eb = s_ptr[0], ee = s_ptr[nv];
    for (uint32_t cb = eb; cb < ee; cb += kChunk) {
      const uint32_t e0 = cb + tid * kEPT;
      uint32_t val[kEPT];
#pragma unroll
      for (int j = 0; j < kEPT; ++j) {
        const uint32_t e = e0 + j;
        const uint32_t ec = e < ee ? e : ee - 1;
        const uint32_t c = sadd(ld_pub<M>(din + g.in_src[ec]), g.in_w[ec]);
        val[j] = e < ee ? c : kInf;
      }
      if (nv == 1) {
        uint32_t q = kInf;
#pragma unroll
        for (int j = 0; j < kEPT; ++j) q = val[j] < q ? val[j] : q;
        q = wmin(q);
        if (lane == 0) atomicMin(&s_min[0], q);
      } else if (e0 < ee) {
        uint32_t i = owner(s_ptr, nv, e0);
        uint32_t bound = s_ptr[i + 1];
        uint32_t part = kInf;
#pragma unroll
        for (int j = 0; j < kEPT; ++j) {
          const uint32_t e = e0 + j;
          if (e < ee) {
            if (e >= bound) {
              atomicMin(&s_min[i], part);
              part = kInf;
              do { ++i; bound = s_ptr[i + 1]; } while (e >= bound);
            }
            part = val[j] < part ? val[j] : part;
          }
        }
        atomicMin(&s_min[i], part);
      }
    }
    __syncthreads();
    if (tid < nv) {
      const uint32_t v = v0 + tid;
      const uint32_t old = din[v];  // only this tile's workgroup writes v in this sweep
      const uint32_t nw = s_min[tid] < old ? s_min[tid] : old;
      if (nw < old) s_chg = 1u;
      if constexpr (M == kSync) dout[v] = nw;
      else if constexpr (M == kAsync) st_pub(dout + v, nw);
      else a.shadow[v] = nw;
    }
    __syncthreads();
    if (tid == 0) a.tchg[t] = s_chg;
    if constexpr (M == kDelayed) {
      if (tid == 0) s_ring[nring] = t;
      ++nring;
      staged += nv;
      if (staged >= a.d || nring == kRing) {
        __syncthreads();
        for (uint32_t i = 0; i < nring; ++i) {
          const uint32_t f0 = g.tile_v[s_ring[i]], f1 = g.tile_v[s_ring[i] + 1];
          for (uint32_t v = f0 + tid; v < f1; v += kWG) st_pub(dout + v, a.shadow[v]);
        }
        nring = 0;
        staged = 0;
      }
    }
  }
  if constexpr (M == kDelayed) {
    if (nring) {
      __syncthreads();
      for (uint32_t i = 0; i < nring; ++i) {
        const uint32_t f0 = g.tile_v[s_ring[i]], f1 = g.tile_v[s_ring[i] + 1];
        for (uint32_t v = f0 + tid; v < f1; v += kWG) st_pub(dout + v, a.shadow[v]);
      }
    }
  }
}

__global__ __launch_bounds__(kWG) void set_bf_fold_kernel(SetBfArgs a) {
  const uint32_t gi = blockIdx.x, tid = threadIdx.x;
  const uint32_t k = *a.c.cur;
  if (k >= a.c.S) return;
  const bool run = a.c.live[k] != 0 && a.c.gdone[gi] == 0;  // uniform over the block
  if (run) {
    const uint32_t t0 = a.g.g_toff[gi], t1 = a.g.g_toff[gi + 1];
    int any = 0;
    for (uint32_t t = t0 + tid; t < t1; t += kWG) any |= a.tchg[t] != 0;
    any = __syncthreads_or(any);
    if (tid == 0) {
      if (!any) a.c.gdone[gi] = k + 1;
      else atomicAdd(a.c.live + k + 1, 1u);
    }
  }
  close_sweep(a.c, k);
}

__global__ __launch_bounds__(kWG) void set_bf_init_kernel(SetBfArgs a, const uint32_t* src) {
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v >= a.g.N) return;
  const uint32_t gi = graph_of(a.g.g_voff, a.g.G, v);
  const uint32_t d0 = src[gi] == v ? 0u : kInf;
  a.c0[v] = d0;
  if (a.c1) a.c1[v] = d0;
}

// One block per graph copies its distances from the buffer its last sweep wrote.
__global__ __launch_bounds__(kWG) void set_bf_out_kernel(SetBfArgs a, int sync, uint32_t last_k, uint32_t* out) {
  const uint32_t gi = blockIdx.x;
  const uint32_t v0 = a.g.g_voff[gi], v1 = a.g.g_voff[gi + 1];
  const uint32_t done = a.c.gdone[gi];
  const uint32_t kl = done ? done - 1 : last_k;
  const uint32_t* d = sync ? ((kl & 1u) ? a.c0 : a.c1) : a.c0;
  for (uint32_t v = v0 + threadIdx.x; v < v1; v += kWG) out[v] = d[v];
}

// Resets the control state of a call.
__global__ __launch_bounds__(kWG) void set_ctl_reset_kernel(SetCtl c, uint32_t G) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i == 0) *c.cur = 0;
  if (i <= c.S) {
    c.next[i] = 0;
    c.fcount[i] = 0;
    c.live[i] = i == 0 ? G : 0u;
  }
  if (i < G) c.gdone[i] = 0;
}

inline uint32_t blocks(uint32_t n) { return (n + kWG - 1) / kWG; }

hipError_t reset(const SetCtl& c, uint32_t G, hipStream_t s) {
  const uint32_t n = (c.S + 1 > G ? c.S + 1 : G);
  set_ctl_reset_kernel<<<blocks(n), kWG, 0, s>>>(c, G);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_set_pr_init(bool f64, const SetPrArgs& a, const double* dang0, hipStream_t s) {
  hipError_t e = reset(a.c, a.g.G, s);
  if (e != hipSuccess) return e;
  const uint32_t n = a.g.N > a.g.G ? a.g.N : a.g.G;
  if (f64) set_pr_init_kernel<double><<<blocks(n), kWG, 0, s>>>(a, dang0);
  else set_pr_init_kernel<float><<<blocks(n), kWG, 0, s>>>(a, dang0);
  return hipGetLastError();
}

template <typename T>
static void set_pr_go(int mode, const SetPrArgs& a, hipStream_t s) {
  if (mode == kSync) set_pr_sweep_kernel<kSync, T><<<a.g.P, kWG, 0, s>>>(a);
  else if (mode == kAsync) set_pr_sweep_kernel<kAsync, T><<<a.g.P, kWG, 0, s>>>(a);
  else set_pr_sweep_kernel<kDelayed, T><<<a.g.P, kWG, 0, s>>>(a);
}

hipError_t launch_set_pr_sweep(int mode, bool f64, const SetPrArgs& a, hipStream_t s) {
  if (f64) set_pr_go<double>(mode, a, s);
  else set_pr_go<float>(mode, a, s);
  set_pr_fold_kernel<<<a.g.G, kWG, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_set_pr_out(bool f64, const SetPrArgs& a, double* out, hipStream_t s) {
  if (f64) set_pr_out_kernel<double><<<a.g.G, kWG, 0, s>>>(a, out);
  else set_pr_out_kernel<float><<<a.g.G, kWG, 0, s>>>(a, out);
  return hipGetLastError();
}

hipError_t launch_set_bf_init(const SetBfArgs& a, const uint32_t* src, hipStream_t s) {
  hipError_t e = reset(a.c, a.g.G, s);
  if (e != hipSuccess) return e;
  set_bf_init_kernel<<<blocks(a.g.N), kWG, 0, s>>>(a, src);
  return hipGetLastError();
}

hipError_t launch_set_bf_sweep(int mode, const SetBfArgs& a, hipStream_t s) {
  if (mode == kSync) set_bf_sweep_kernel<kSync><<<a.g.P, kWG, 0, s>>>(a);
  else if (mode == kAsync) set_bf_sweep_kernel<kAsync><<<a.g.P, kWG, 0, s>>>(a);
  else set_bf_sweep_kernel<kDelayed><<<a.g.P, kWG, 0, s>>>(a);
  set_bf_fold_kernel<<<a.g.G, kWG, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_set_bf_out(int mode, const SetBfArgs& a, uint32_t last_k, uint32_t* out, hipStream_t s) {
  set_bf_out_kernel<<<a.g.G, kWG, 0, s>>>(a, mode == kSync ? 1 : 0, last_k, out);
  return hipGetLastError();
}

}  // namespace dg

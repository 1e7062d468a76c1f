// Topology instrumentation: the access matrix of one sweep (section IV, the
// effects of graph topology).  Every in-edge u -> v of the pull sweep is a
// read, by the worker that owns v, of a value that the worker owning u
// writes.  Workers are coarsened into B groups of consecutive workers (B = 8
// makes each group one XCD's share); the result is the B x B matrix of read
// counts (row: reading group, column: owning group) plus the reads whose
// source the reading worker writes itself.
#include "dg_internal.hpp"

namespace dg {
namespace {

// worker of each vertex: block w fills its own vertex range
__global__ __launch_bounds__(kWG) void vertex_worker_kernel(Topology g, uint32_t* vw) {
  const uint32_t w = blockIdx.x;
  const uint32_t v0 = g.tile_v[g.work_t[w]], v1 = g.tile_v[g.work_t[w + 1]];
  for (uint32_t v = v0 + threadIdx.x; v < v1; v += kWG) vw[v] = w;
}

// vertex of each slot of the compact region
__global__ __launch_bounds__(kWG) void hot_inverse_kernel(Topology g, uint32_t* inv) {
  const uint32_t v = blockIdx.x * kWG + threadIdx.x;
  if (v >= g.n) return;
  const uint32_t p = g.cpos[v];
  if (p >= g.n) inv[p - g.n] = v;
}

// Grid-stride over destination vertices; a B x B histogram per workgroup in
// LDS, added to the global matrix once.
__global__ __launch_bounds__(kWG) void access_kernel(Topology g, const uint32_t* vw, const uint32_t* inv,
                                                     uint32_t B, unsigned long long* counts,
                                                     unsigned long long* self) {
  extern __shared__ uint32_t s_h[];  // [B*B]
  __shared__ unsigned long long s_self;
  for (uint32_t i = threadIdx.x; i < B * B; i += kWG) s_h[i] = 0;
  if (threadIdx.x == 0) s_self = 0;
  __syncthreads();
  const uint32_t P = g.P;
  unsigned long long mine = 0;
  for (uint32_t v = blockIdx.x * kWG + threadIdx.x; v < g.n; v += gridDim.x * kWG) {
    const uint32_t rw = vw[v];
    const uint32_t rg = (uint32_t)((unsigned long long)rw * B / P);
    for (uint32_t e = g.in_ptr[v]; e < g.in_ptr[v + 1]; ++e) {
      const uint32_t slot = g.in_src[e];
      const uint32_t u = slot < g.n ? slot : inv[slot - g.n];
      const uint32_t ow = vw[u];
      mine += ow == rw;
      atomicAdd(&s_h[rg * B + (uint32_t)((unsigned long long)ow * B / P)], 1u);
    }
  }
  atomicAdd(&s_self, mine);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < B * B; i += kWG)
    if (s_h[i]) atomicAdd(counts + i, (unsigned long long)s_h[i]);
  if (threadIdx.x == 0) atomicAdd(self, s_self);
}

}  // namespace

hipError_t launch_access_matrix(const Topology& g, uint32_t* vw, uint32_t* inv, uint32_t B,
                                unsigned long long* counts, unsigned long long* self, hipStream_t s) {
  vertex_worker_kernel<<<g.P, kWG, 0, s>>>(g, vw);
  if (g.K) hot_inverse_kernel<<<(g.n + kWG - 1) / kWG, kWG, 0, s>>>(g, inv);
  const uint32_t blocks = 1024;
  access_kernel<<<blocks, kWG, (size_t)B * B * 4, s>>>(g, vw, inv, B, counts, self);
  return hipGetLastError();
}

}  // namespace dg

// Kernels of graph sets.  A set is stored as one union graph (graph i's
// vertices are the range [voff[i], voff[i+1]) and no edge crosses two
// graphs) and swept by the single-graph kernels; these two kernels start
// every graph's Bellman-Ford from its own source and give every graph's
// PageRank its own normalisation.
#include "dg_internal.hpp"

namespace dg {
namespace {

__global__ __launch_bounds__(kWG) void bf_more_sources_kernel(uint32_t* d0, uint32_t* d1, const uint32_t* cpos,
                                                              const uint32_t* src, uint32_t k) {
  const uint32_t i = blockIdx.x * kWG + threadIdx.x;
  if (i >= k) return;
  const uint32_t p = cpos[src[i]];
  d0[p] = 0;
  if (d1) d1[p] = 0;
}

// One block per graph: the sum of its scores in a fixed order (threads
// strided, then wavefront and workgroup reductions in lane and wave order),
// then the scores divided by it.
__global__ __launch_bounds__(kWG) void segment_normalize_kernel(double* x, const uint32_t* voff) {
  __shared__ double s[kWG / 64];
  const uint32_t g = blockIdx.x, tid = threadIdx.x;
  const uint32_t v0 = voff[g], v1 = voff[g + 1];
  double acc = 0.0;
  for (uint32_t v = v0 + tid; v < v1; v += kWG) acc += x[v];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((tid & 63u) == 0) s[tid >> 6] = acc;
  __syncthreads();
  const double sum = s[0] + s[1] + s[2] + s[3];
  for (uint32_t v = v0 + tid; v < v1; v += kWG) x[v] /= sum;
}

}  // namespace

hipError_t launch_bf_more_sources(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, const uint32_t* src, uint32_t k,
                                  hipStream_t s) {
  if (k) bf_more_sources_kernel<<<(k + kWG - 1) / kWG, kWG, 0, s>>>(d0, d1, cpos, src, k);
  return hipGetLastError();
}

hipError_t launch_segment_normalize(double* x, const uint32_t* voff, uint32_t G, hipStream_t s) {
  if (G) segment_normalize_kernel<<<G, kWG, 0, s>>>(x, voff);
  return hipGetLastError();
}

}  // namespace dg

// Gather-rate probe: the rate at which one MI355X serves random 4-byte loads
// from a table of a given size, the access that bounds a single query's pull
// sweep (one scattered read of a published value per in-edge).  Two forms:
//   hashed    each thread computes its table indices (no index traffic);
//   streamed  the indices come from a coalesced stream in device memory, one
//             4-byte index per gather, as in a sweep's in-edge stream.
// Indices are uniform over the table, from the 32-bit integer mixer
// "lowbias32" (Wellons, 2018) applied to the gather's global number.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dg.h"
#include "dg_host.hpp"

namespace dg {
namespace {

constexpr int kProbeWG = 256;
constexpr int kProbeUnroll = 16;  // gathers a thread keeps in flight

__device__ __host__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Gather j of thread t is number j * T + t (T threads), so the index stream
// is read with consecutive threads at consecutive words.
template <bool STREAM>
__global__ __launch_bounds__(kProbeWG) void probe_gather_kernel(const uint32_t* __restrict__ table, uint32_t mask,
                                                                const uint32_t* __restrict__ idx, uint32_t per_thread,
                                                                uint32_t* __restrict__ out) {
  const uint32_t t = blockIdx.x * kProbeWG + threadIdx.x;
  const uint32_t T = gridDim.x * kProbeWG;
  uint32_t acc = 0;
  for (uint32_t j = 0; j < per_thread; j += kProbeUnroll) {
    uint32_t v[kProbeUnroll];
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) {
      const uint32_t g = (j + q) * T + t;
      const uint32_t i = STREAM ? idx[g] : (mix32(g) & mask);
      v[q] = table[i];
    }
#pragma unroll
    for (int q = 0; q < kProbeUnroll; ++q) acc += v[q];
  }
  out[t] = acc;
}

__global__ __launch_bounds__(kProbeWG) void probe_fill_kernel(uint32_t* idx, uint64_t count, uint32_t mask,
                                                              uint32_t* table, uint64_t entries) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeWG;
  for (uint64_t i = blockIdx.x * kProbeWG + threadIdx.x; i < count; i += stride) idx[i] = mix32((uint32_t)i) & mask;
  for (uint64_t i = blockIdx.x * kProbeWG + threadIdx.x; i < entries; i += stride) table[i] = (uint32_t)i;
}

}  // namespace
}  // namespace dg

using dg::host::fail;

extern "C" dg_status dg_probe_gather(uint64_t table_bytes, int streamed, uint32_t per_thread, uint32_t workgroups,
                                     double* out_seconds, void* hip_stream) {
  using namespace dg;
  host::g_last_error.clear();
  if (table_bytes < 4096 || table_bytes > (1ull << 32) || (table_bytes & (table_bytes - 1)))
    return fail(DG_ERR_INVALID_ARGUMENT, "table_bytes must be a power of two in [4 KiB, 4 GiB]");
  if (streamed != 0 && streamed != 1) return fail(DG_ERR_INVALID_ARGUMENT, "streamed must be 0 or 1");
  if (per_thread == 0 || per_thread % kProbeUnroll || per_thread > 4096)
    return fail(DG_ERR_INVALID_ARGUMENT, "per_thread must be a multiple of %d in [%d, 4096]", kProbeUnroll,
                kProbeUnroll);
  if (workgroups == 0 || workgroups > 65536) return fail(DG_ERR_INVALID_ARGUMENT, "workgroups must be in [1, 65536]");
  if (!out_seconds) return fail(DG_ERR_INVALID_ARGUMENT, "out_seconds is NULL");
  const uint64_t threads = (uint64_t)workgroups * kProbeWG;
  const uint64_t gathers = threads * per_thread;
  if (gathers >= (1ull << 32)) return fail(DG_ERR_INVALID_ARGUMENT, "more than 2^32 gathers per launch");
  const uint64_t entries = table_bytes / 4;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  uint32_t *table = nullptr, *idx = nullptr, *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dg_status st = DG_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    if (table) (void)hipFree(table);
    if (idx) (void)hipFree(idx);
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = hipMalloc(&table, table_bytes);
  if (e == hipSuccess && streamed) e = hipMalloc(&idx, gathers * 4);
  if (e == hipSuccess) e = hipMalloc(&out, threads * 4);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    probe_fill_kernel<<<1024, kProbeWG, 0, s>>>(idx, streamed ? gathers : 0, (uint32_t)(entries - 1), table, entries);
    e = hipGetLastError();
  }
  // One warm-up launch, then the best of three timed ones.
  double best = 1e300;
  for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
    e = hipEventRecord(e0, s);
    if (e != hipSuccess) break;
    if (streamed)
      probe_gather_kernel<true><<<workgroups, kProbeWG, 0, s>>>(table, (uint32_t)(entries - 1), idx, per_thread, out);
    else
      probe_gather_kernel<false><<<workgroups, kProbeWG, 0, s>>>(table, (uint32_t)(entries - 1), idx, per_thread, out);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && rep > 0) best = ms * 1e-3 < best ? ms * 1e-3 : best;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    st = fail(e == hipErrorOutOfMemory ? DG_ERR_OUT_OF_MEMORY : DG_ERR_DEVICE, "gather probe failed: %s",
              hipGetErrorString(e));
  } else {
    *out_seconds = best;
  }
  cleanup();
  return st;
}

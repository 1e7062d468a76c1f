// Host-side helpers shared by the translation units of the C ABI
// (dg_api.cpp: single graphs and batched queries; dg_set.cpp: graph sets).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dg {
namespace host {

// Message of the last error on the calling thread (dg_last_error).
extern thread_local std::string g_last_error;

// Records a printf-style message and returns s.
dg_status fail(dg_status s, const char* fmt, ...);

// Allocation hooks installed by dg_set_allocator (both null: hipMalloc/hipFree).
void current_allocator(dg_alloc_fn& alloc, dg_free_fn& free_fn, void*& ctx);

// Tiles of consecutive vertices: at most kTileV vertices and max_e in-edges,
// except that a vertex with more in-edges is a tile of its own; a tile also
// ends before every vertex listed in seg_v (the graphs of a set).
void build_tiles(const std::vector<uint32_t>& in_ptr, uint32_t n, std::vector<uint32_t>& tile_v,
                 const std::vector<uint32_t>* seg_v, uint32_t max_e);

// In-edges per tile of the batched kernels.  Their workers gather a 256-byte
// row per edge, so a single-query tile (up to 16380 in-edges) is a coarse
// unit for them: a graph with a thousand tiles could not give eight
// 256-thread workgroups to each compute unit.
constexpr uint32_t kBatchTileE = 4096;

// Tiles of the batched kernels: each tile of tile_v split greedily into runs
// of consecutive vertices with at most max_e in-edges, a vertex with more
// being a run of its own; a single-vertex tile stays whole.  Runs never
// cross a tile boundary (nor, therefore, a graph of a set).  btile_e0[t] is
// the first in-edge of run t.
void build_batch_tiles(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& in_ptr, uint32_t max_e,
                       std::vector<uint32_t>& btile_v, std::vector<uint32_t>& btile_e0);

}  // namespace host
}  // namespace dg

#define DG_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipGetLastError();                                                                \
      return ::dg::host::fail(e_ == hipErrorOutOfMemory ? DG_ERR_OUT_OF_MEMORY : DG_ERR_DEVICE, \
                              "%s failed: %s", #call, hipGetErrorString(e_));                 \
    }                                                                                         \
  } while (0)

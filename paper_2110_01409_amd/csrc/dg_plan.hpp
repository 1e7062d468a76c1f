// Host-only construction of a graph's device layout: the in-edge form, the
// compact region and its resident table, the tiles and the worker
// partition.  dg_graph_create uploads exactly what build_layout and
// build_partition produce; dg_plan_* expose the same result without a
// device.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "dg.h"

namespace dg {
namespace host {

struct Layout {
  uint32_t n = 0;
  uint64_t m = 0;
  bool has_w = false;
  uint32_t K = 0;             // compact-region slots
  uint32_t R = 0;             // leading compact-region slots in the resident table
  uint64_t hot_edges = 0;     // in-edges whose source is in the compact region
  uint64_t res_edges = 0;     // in-edges whose source is in the resident table
  uint32_t max_in_deg = 0, n_dangling = 0;
  uint64_t hash = 0;          // content hash of the in-edge form (FNV-1a)
  std::vector<uint32_t> in_ptr;   // [n+1]
  std::vector<uint32_t> in_src;   // [m + kEdgePad] slot of each in-edge's source
  std::vector<uint32_t> in_w;     // [m + kEdgePad] uint32 weights, empty when packed or unweighted
  std::vector<uint32_t> w8pack;   // bytes of the weights packed four to a word, when all are <= 255
  std::vector<uint32_t> out_deg;  // [n]
  std::vector<uint32_t> cpos;     // [n] slot of each vertex's published value
  std::vector<uint32_t> tile_v;   // [T+1] first vertex of each tile
  std::vector<uint32_t> tile_e0;  // [T+1] first in-edge of each tile
  uint32_t variant = 0;           // SweepVariant of the single-query sweeps
  uint32_t T() const { return (uint32_t)tile_v.size() - 1; }
};

// Checks the arrays of dg_graph_create (the checks its documentation lists).
dg_status validate_graph(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx);

// Builds everything but the worker partition from validated arrays.
// `workers` is the partition's worker count, which the automatic sweep
// variant is chosen for.
// Returns DG_ERR_OUT_OF_MEMORY on host allocation failure and
// DG_ERR_UNSUPPORTED when n plus the compact region exceeds the slots a
// sweep can address.
// seg_v (optional, [G+1]): first vertices of the graphs of a set; no tile
// crosses one of them.
dg_status build_layout(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                       const uint32_t* w, const dg_graph_opts* opts, uint32_t workers, Layout& L,
                       const std::vector<uint32_t>* seg_v = nullptr);

// Worker count for a device of `cus` compute units: want_workers if set,
// else per_cu per compute unit rounded down to a multiple of 8; never more
// than the tiles.
uint32_t plan_workers(const Layout& L, uint32_t want_workers, uint32_t cus, uint32_t per_cu);

// Default workers of a batched partition: per_cu per compute unit, rounded
// down to a multiple of 8, at most one per batched tile, at least one.
uint32_t batch_workers_for(uint32_t cus, uint32_t per_cu, uint32_t batch_tiles);

// Contiguous tile ranges of P workers balanced by 256 + in-edges + 4 x
// vertices per tile; work_t[P+1].
void build_workers(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& tile_e0, uint32_t P,
                   std::vector<uint32_t>& work_t);

// The same for a set: P >= G workers, each graph gets at least one and
// otherwise workers in proportion to its cost, and its tiles are split
// among them as above.  Returns wseg[G+1], the first worker of each graph.
void build_workers_seg(const std::vector<uint32_t>& tile_v, const std::vector<uint32_t>& tile_e0,
                       const std::vector<uint32_t>& seg_v, uint32_t P, std::vector<uint32_t>& work_t,
                       std::vector<uint32_t>& wseg);

}  // namespace host
}  // namespace dg

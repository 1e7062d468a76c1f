// The resident graph object behind dg_graph*, shared by the host translation
// units (dg_api.cpp: single graphs, batched queries, tuning; dg_server.cpp:
// the serving loop).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "dg.h"
#include "dg_internal.hpp"

namespace dg {
namespace host {

// Sweeps the host keeps queued beyond the one whose result it waits for: at
// most kMaxLookahead, and enough to cover about kHostReactUs of the host's
// reaction time at the call's measured sweep time.  Each queued sweep first
// tests on the device whether an earlier one met the stopping rule.
constexpr uint32_t kMaxLookahead = 8;
constexpr double kHostReactUs = 150.0;
// Per-sweep completion events, reused round-robin (more than the lookahead).
constexpr uint32_t kEventRing = 16;
constexpr uint32_t kMaxSweeps = 1000000;
// Default persistent workgroups per compute unit of the single-query sweeps:
// one 1024-thread workgroup, whose LDS holds the resident table.
constexpr uint32_t kWorkersPerCU = 1;
// The same for the batched kernels (256 threads, no table), one partition
// per algorithm: on RMAT-22 the SSSP kernel runs 5-8% faster per batch-sweep
// with eight than with five, the PPR kernel 2-5% slower.
constexpr uint32_t kBatchSsspWorkersPerCU = 8;
constexpr uint32_t kBatchPprWorkersPerCU = 5;
// Which batched partition: SSSP (dg_sssp_batch, the server's SSSP pools) or
// personalised PageRank (dg_ppr_batch, the server's PPR pools).
enum BatchAlgo : int { kBatchSssp = 0, kBatchPpr = 1 };
// A partition of the batched tiles (dg_graph::btile_v) into batched workers
// (the grid's x dimension).
struct BatchPart {
  uint32_t P = 0;                  // workers
  uint32_t max_block_v = 1;        // most vertices any worker owns
  uint32_t* work_t = nullptr;      // device [P + 1]: first batched tile of each worker
  std::vector<uint32_t> work_t_h;  // host copy
};
// The same for the union graph of a set: smaller blocks, several sweep
// workgroups per compute unit in turn, so that the last graphs to converge
// (the others' workers exit at once) still spread over the whole GPU.
// Three to five measured best on a 64-graph set.
constexpr uint32_t kSetWorkersPerCU = 5;
// Automatic sweep variant: narrow below kNarrowBelow wide tiles per worker,
// wide with all gathers in flight up to kInFlightUpTo, wide beyond.
// Measured per float32 PageRank sweep on R-MAT with 256 workers: narrow
// wins up to scale 18 (27.5 against 34.8 us at scale 16, synchronous),
// all-in-flight at scale 20 (80 against 96 us), the paced wide variant at
// scale 22 (4680 tiles).
constexpr uint64_t kNarrowBelow = 2;
constexpr uint64_t kInFlightUpTo = 8;
// Captured launches (dg_graph_set_capture): at most kMaxCaptureChunk sweeps
// per recorded chunk, and at most kMaxCapturedChunks chunks recorded per call
// shape; a call that runs longer launches its later sweeps one by one.
constexpr uint32_t kMaxCaptureChunk = 64;
constexpr uint32_t kMaxCapturedChunks = 256;

}  // namespace host
}  // namespace dg

struct dg_graph {
  uint32_t n = 0;
  uint64_t m = 0;
  bool has_w = false;
  uint32_t P = 0, T = 0, cus = 0, max_in_deg = 0, n_dangling = 0;
  uint32_t variant = 0;  // SweepVariant of the single-query sweeps
  uint32_t variant0 = 0; // the variant chosen at creation
  uint32_t K = 0;          // sources stored in the compact region
  uint32_t max_block_v = 1;  // most vertices any worker owns
  // Tiles of the batched kernels (the tiles split by build_batch_tiles), and
  // their partitions into batched workers, one per algorithm (indexed by
  // BatchAlgo).
  std::vector<uint32_t> btile_v_h, btile_e0_h;  // host: first vertex / first in-edge of each batched tile
  uint32_t* btile_v = nullptr;                  // device copy of btile_v_h
  dg::host::BatchPart bp[2];
  std::vector<uint32_t> tile_v_h, tile_e0_h;  // host copies: first vertex / first in-edge of each tile
  std::vector<uint32_t> work_t_h;             // host copy of work_t: first tile of each worker
  std::vector<uint32_t> in_ptr_h;             // host copy of in_ptr (re-tiling by dg_graph_set_mapping)
  uint32_t res_limit = 0xFFFFFFFFu;           // resident-table entries the sweeps may use (<= R)
  uint64_t hash = 0;                         // content hash of the in-edge form (tuning cache key)
  // Graph sets: the union of G graphs, with worker blocks aligned to graph
  // boundaries (graph i's workers are wseg[i] .. wseg[i+1]-1); G = 0 otherwise.
  uint32_t G = 0;
  std::vector<uint32_t> seg_v;  // [G+1] first vertex of each graph (host)
  std::vector<uint32_t> wseg_h; // [G+1] first worker of each graph (host)
  uint32_t* wseg = nullptr;     // device copy of wseg_h
  std::vector<uint32_t> wgraph_h;  // [P] graph of each worker (host)
  uint32_t* wgraph = nullptr;      // device copy of wgraph_h
  uint32_t* gsweeps = nullptr;  // [G] first sweep that took each graph below tol
  uint32_t* segv_d = nullptr;   // device copy of seg_v
  double* gdang = nullptr;      // [2][G] per-graph dangling deficits (PrArgs::gdang)
  std::vector<double> gdang0;   // [G] each graph's dangling share of the union before sweep 0
  uint64_t hot_edges = 0;  // in-edges whose source is in the compact region
  uint32_t R = 0;          // leading compact-region slots kept in the sweeps' LDS table
  uint64_t res_edges = 0;  // in-edges whose source is one of them
  size_t lds_per_block = 65536;
  // allocator captured at creation
  dg_alloc_fn alloc = nullptr;
  dg_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  hipStream_t create_stream = nullptr;
  std::vector<void*> owned;
  uint64_t graph_bytes = 0;
  // resident graph
  uint32_t *in_ptr = nullptr, *in_src = nullptr, *in_w = nullptr, *out_deg = nullptr, *cpos = nullptr;
  uint8_t* in_w8 = nullptr;  // weights as bytes when all are <= 255 (then in_w is null)
  uint32_t *tile_v = nullptr, *work_t = nullptr;
  // workspace (grown on demand)
  void* vals[3] = {nullptr, nullptr, nullptr};  // 8(n+K) bytes each
  double* norm = nullptr;                        // kNormBlocks + 1
  uint32_t ws_sweeps = 0;
  double *resid = nullptr, *dang = nullptr, *part = nullptr;
  double* scale = nullptr;  // [S+1] storage scales of personalised PageRank sweeps
  uint32_t *count = nullptr, *changed = nullptr;
  void* host_poll = nullptr;      // mapped pinned [S+1] doubles: the sweeps' stopping values
  void* host_poll_dev = nullptr;  // its device address
  uint32_t lookahead = 4;         // sweeps queued ahead, from the last call's sweep time
  hipEvent_t ev_start = nullptr;
  hipEvent_t ev_sweep[dg::host::kEventRing] = {};
  bool events = false;
  // Captured launches: 0 = every sweep launched on its own; else chunks of
  // `capture` consecutive sweeps, each recorded once into a HIP graph (on
  // cap_stream, which holds no other work) and replayed on the call's stream.
  // cap_exec[j] holds sweeps j*capture .. j*capture+capture-1 of calls whose
  // launch arguments (pointers, sizes, mode, limits) are the bytes cap_key.
  uint32_t capture = 0;
  hipStream_t cap_stream = nullptr;
  std::vector<unsigned char> cap_key;
  std::vector<hipGraphExec_t> cap_exec;
};

namespace dg {
namespace host {

// Destroys the graph's recorded chunks (their key no longer matches, or the
// capture length or the mapping changed).
void drop_captures(dg_graph* g);
// Device allocations through the graph's allocator hooks (tracked, freed with
// the graph).
void* dev_alloc(dg_graph* g, size_t bytes, hipStream_t s);
void dev_free(dg_graph* g, void* p);
// Device arrays of the resident graph as passed to the single-query sweep
// kernels (P workers), and to the batched kernels (the partition `which`).
Topology topo(const dg_graph* g);
Topology topo_batch(const dg_graph* g, int which);
// dg_graph_create for the union graph of a set: seg_v[G+1] are the first
// vertices of the G graphs.  Tiles never cross a graph boundary and every
// graph gets its own worker blocks (at least one).
dg_status graph_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                       const uint32_t* w, const dg_graph_opts* opts, const std::vector<uint32_t>* seg_v,
                       void* hip_stream, dg_graph** out);
// Staging of a delayed single-query sweep for commit interval d with elem-byte
// values and res resident-table entries: LDS capacity cap (0 = the global
// per-vertex shadow, shadow = true) and the effective interval d_eff.
void staging(const dg_graph* g, uint32_t d, size_t elem, uint32_t res, uint32_t& cap, uint32_t& d_eff,
             bool& shadow);
// Commits per sweep of a delayed single-query sweep with that staging.
uint32_t commits_per_sweep(const dg_graph* g, uint32_t d, uint32_t cap, bool shadow);
// PageRank (psrc = 0xFFFFFFFF, as dg_pagerank) or personalised PageRank with
// restart vertex psrc (as dg_ppr).
dg_status pr_run(dg_graph* g, uint32_t psrc, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                 uint32_t max_sweeps, double* out_scores, int out_on_device, dg_stats* stats, void* hip_stream);
// Bellman-Ford from src and, when n_more > 0, also from the n_more sources in
// the device array more_src (distance to the nearest source); otherwise as
// dg_sssp.
dg_status sssp_run(dg_graph* g, uint32_t src, const uint32_t* more_src, uint32_t n_more, dg_mode mode, uint32_t d,
                   uint32_t max_sweeps, uint32_t* out_dist, int out_on_device, dg_stats* stats, void* hip_stream);

}  // namespace host
}  // namespace dg

// Internal interface between the host driver (dg_api.cpp) and the gfx950
// sweep kernels (sweep_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dg {

// Workgroup of the streaming, batched, set and instrumentation kernels: 4 wave64s.
constexpr int kWG = 256;
// Workgroup of the single-query sweep kernels: 16 wave64s, one workgroup per
// compute unit, so that one LDS copy of the hottest sources (the resident
// table) can take most of the unit's 160 KB.
constexpr int kSweepWG = 1024;
// Consecutive in-edges one thread reduces per chunk in the wide sweep
// variants (four 16-byte index loads); the narrow variant takes half.
constexpr int kEPT = 16;
constexpr int kEPTNarrow = 8;

// Sweep kernel variants, chosen per graph when it is created (the values
// are those of dg_graph_opts.sweep_variant):
//   kWide          16 in-edges per thread; a resident-table slot is read
//                  from LDS right after its gather is issued, which makes the
//                  wave wait for its outstanding loads and so paces its
//                  gathers.  Fastest on graphs with many tiles per worker,
//                  where the gathers of all workers saturate the memory path.
//   kWideInFlight  16 per thread; all of a chunk's gathers are issued before
//                  the table is read.  Fastest at a few tiles per worker.
//   kNarrow        8 per thread (tiles of at most kTileENarrow in-edges),
//                  all gathers in flight: more, shorter tiles for graphs too
//                  small to give every worker two wide tiles, whose sweeps
//                  are bound by a tile's latency.
enum SweepVariant : uint32_t { kWide = 1, kWideInFlight = 2, kNarrow = 3 };
__host__ __device__ constexpr int ept_of(int v) { return v == kNarrow ? kEPTNarrow : kEPT; }
__host__ __device__ constexpr bool all_in_flight(int v) { return v != kWide; }
// Edge slots a sweep workgroup covers per chunk.
constexpr int kChunk = kSweepWG * kEPT;
// At most this many vertices per tile: one vertex per thread in the update phase.
constexpr int kTileV = kSweepWG;
// Edge budget of a multi-vertex tile.  A chunk starts at the tile's first
// edge rounded down to a multiple of 4 (16-byte aligned vector loads), so a
// tile of at most kChunk-4 edges always fits one chunk.  A single vertex with
// more in-edges gets a tile of its own that spans several chunks.
constexpr int kTileE = kChunk - 4;
constexpr int kTileENarrow = kSweepWG * kEPTNarrow - 4;
// Zero padding after in_src / in_w so that the last chunk's vector loads stay
// inside the allocation.
constexpr uint32_t kEdgePad = kChunk + 16;

constexpr uint32_t kInf = 0xFFFFFFFFu;

// LDS of a sweep workgroup: the whole compute unit's 160 KB.
constexpr uint32_t kLdsBudget = 160 * 1024;
// Resident table: LDS copy of the first slots of the compact region (the
// sources with the largest out-degree), read instead of gathering them.
constexpr uint32_t kResBytes = 128 * 1024;
// Bytes of the table refreshed at once (8 registers per thread).
constexpr uint32_t kResSegBytes = kSweepWG * 8 * 4;
// Dynamic LDS a sweep kernel may request (the rest of 160 KB after its
// static LDS, which stays under 14 KB).
constexpr uint32_t kSweepDynLds = 146 * 1024;

// Commit modes; kDelayedLocal is delayed commits with local reads of a
// worker's own staged values (single-query sweeps only).
enum Mode : int { kSync = 0, kAsync = 1, kDelayed = 2, kDelayedLocal = 3 };

// Graph arrays resident in HBM (all device pointers).
struct Topology {
  const uint32_t* in_ptr;   // [n+1] in-edge offsets (CSC over destinations)
  const uint32_t* in_src;   // [m + kEdgePad] slot (cpos) of each in-edge's source
  const uint32_t* in_w;     // [m + kEdgePad] weight of each in-edge, when stored as uint32 (else null)
  const uint8_t* in_w8;     // [m + kEdgePad + 16] the same as bytes, when every weight is <= 255 (else null)
  const uint32_t* out_deg;  // [n] out-degree
  const uint32_t* cpos;     // [n] slot of each vertex's published value: v, or
                            // n + rank for the K sources of the compact region
  const uint32_t* tile_v;   // [T+1] first vertex of each tile
  const uint32_t* work_t;   // [P+1] first tile of each worker
  uint32_t n;
  uint32_t K;               // slots of the compact region after the n regular ones
  uint32_t P;               // workers = workgroups launched per sweep
  uint32_t variant;         // SweepVariant of the single-query sweeps
};

// Per-call convergence state, indexed by sweep.  Sweep k reads entry k and
// writes entry k+1, so a queued sweep can test on the device whether an
// earlier one already met the stopping rule.
struct SweepState {
  double* resid;      // [S+1] resid[k+1] = L1 change of sweep k; resid[0] = +inf
  double* dang;       // [S+1] mass sweep k spreads uniformly: 1 - non-dangling mass after sweep k-1
  uint32_t* count;    // [S+1] workers finished in sweep k
  uint32_t* changed;  // [S+1] changed[k+1] != 0 iff sweep k decreased a distance
  double* part;       // [3P] per-worker partial sums (residual, non-dangling mass, total mass)
  // Personalised PageRank only (PrArgs::psrc set): scale[k] is the storage
  // scale of sweep k's values (stored = true value * scale[k]); null otherwise.
  double* scale = nullptr;
  // Mapped host mirrors of resid and changed (device addresses of pinned
  // host memory the host polls; same row indices), or null.
  double* hresid = nullptr;
  uint32_t* hchanged = nullptr;
};

struct PrArgs {
  Topology g;
  SweepState st;
  void* x;          // [n] scores, written only by their owner
  const void* cin;  // [n] contributions read by the sweep
  void* cout;       // [n] contributions written (== cin unless synchronous)
  double alpha;
  double tol;
  void* shadow;     // [n] global staging buffer indexed by vertex, or null to stage in LDS
  uint32_t k;       // sweep index
  uint32_t d;       // commit interval in vertices (delayed mode)
  uint32_t cap;     // LDS staging capacity in vertices (delayed mode, LDS staging)
  // Graph sets (the union of G graphs, worker blocks aligned to graph
  // boundaries): graph i's workers are wseg[i] .. wseg[i+1]-1.  The stopping
  // value of a sweep is then the largest per-graph L1 change divided by that
  // graph's mass, and gsweeps[i] records the first sweep that took graph i
  // below tol (0 until then).  wseg is null for a single graph.
  // A worker whose graph has already met tol skips its block and keeps its
  // mass partials of the sweep that converged (its values stay as they were).
  const uint32_t* wseg;
  const uint32_t* wgraph;  // [P] graph of each worker
  uint32_t G;
  uint32_t* gsweeps;
  // Graph sets: each graph keeps its own mass (its share n_i/n of the
  // union's): its dangling deficit gdang[(k & 1) G + i] = n_i/n minus its
  // non-dangling mass after sweep k-1 is spread over its own n_i vertices,
  // so every graph iterates as it would alone (scaled by n_i/n).
  // voff[G+1] are the graphs' first vertices.
  const uint32_t* voff;
  double* gdang;  // [2][G]
  // Slots n .. n+res-1 are read from the workgroup's LDS table (0 = none).
  // The table is filled at the start of the sweep; an asynchronous sweep
  // refreshes one segment of it after every tile, a delayed sweep after
  // every tile that ends with a commit.
  uint32_t res;
  // Personalised PageRank with restart vertex psrc (kInf: global PageRank).
  // Teleport and dangling mass go to psrc; st.dang[k] is the dangling mass
  // (true scale) of the previous iterate, and values are stored scaled by
  // st.scale[k], which the sweep's last worker multiplies by the iterate's
  // mass (a rescale to mass 1 without a pass over memory).  Not for sets.
  uint32_t psrc = 0xFFFFFFFFu;
};

struct BfArgs {
  Topology g;
  SweepState st;
  const uint32_t* din;  // [n] distances read by the sweep
  uint32_t* dout;       // [n] distances written (== din unless synchronous)
  uint32_t* shadow;     // [n] global staging buffer indexed by vertex, or null to stage in LDS
  uint32_t k;
  uint32_t d;
  uint32_t cap;
  uint32_t res;  // as PrArgs::res
  // Graph sets, as in PrArgs: gsweeps[i] records the first sweep in which
  // graph i changed no distance (its distances are final then: no edge
  // crosses two graphs), and its workers skip their blocks from then on.
  const uint32_t* wseg;
  const uint32_t* wgraph;
  uint32_t G;
  uint32_t* gsweeps;
};

// Float32 personalised PageRank stops at its rounding floor: a query whose
// L1 change is below kStallTols x tol and no smaller than kStallRatio times
// its change two sweeps earlier stops as if it had met tol.  In exact
// arithmetic the change of a synchronous sweep contracts by at least
// damping^2 over two sweeps, so a change that stops shrinking is rounding
// noise (a float32 vector can settle into a period-2 cycle above tol).
constexpr double kStallTols = 2.0;
constexpr double kStallRatio = 0.9;

// Batched queries: rows a wavefront stages in LDS in delayed mode, and the
// largest commit interval staged that way (four wavefronts per workgroup);
// larger intervals stage in a global shadow array.
constexpr uint32_t kStageRows = 16;
constexpr uint32_t kLdsStageMaxD = kStageRows * (kWG / 64);

// Batched queries (64 per batch, vertex-major [slot][64] values).
struct MbfArgs {
  Topology g;
  const uint32_t* din;  // [NB][n+K][64] distances read
  uint32_t* dout;       // [NB][n+K][64] distances written (== din unless synchronous)
  uint32_t* shadow;     // [NB][n][64] delayed-mode staging, else null
  uint32_t* changed;    // [(S+1)][NB] changed[(k+1)NB+b] != 0 iff sweep k changed batch b (call mode)
  uint32_t* lchg;       // serving: [NB][64] set to nonzero for every query that changed in the sweep, else null
  const uint32_t* bactive;  // serving: [NB] nonzero for batches with running queries, else null
  uint32_t* hchanged = nullptr;  // mapped host mirror of changed (call mode), or null
  uint32_t k, d, NB;
};

struct MpprArgs {
  Topology g;
  const void* cin;      // [NB][n+K][64] contributions read (float or double)
  void* cout;           // [NB][n+K][64] contributions written
  void* x;              // [NB][n][64] scores
  void* shadow;         // [NB][n][64] delayed-mode staging, else null
  const uint32_t* src;  // [nq] restart vertex of each query
  double* resid;        // [(S+1)][NB] largest per-query L1 change of sweep k-1; entry 0 = +inf
  double* dang;         // [2][NB][64] dangling mass (true scale) returned to the restart vertex, by sweep parity
  double* scale;        // [2][NB][64] storage scale of each query's values, by sweep parity
  uint32_t* qdone;      // [NB][64] 0 while a query runs, else the sweep count that stopped it
  double* rhist;        // [2][NB][64] float32 only: each query's change of sweep k-2 (slot k & 1), for
                        // the stall rule; null = no stall rule
  const uint32_t* bactive;  // serving: [NB] nonzero for batches with running queries (count is then a
                            // [2][NB] ring and resid is unused), else null
  uint32_t* count;      // [(S+1)][NB] workers finished
  double* part;         // [P][NB][3][64] per-worker partials (change, dangling mass, total mass)
  double* hresid = nullptr;  // mapped host mirror of resid (call mode), or null
  double alpha, tol;
  uint32_t nq, k, d, NB;
};

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_mbf_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, const uint32_t* src, uint32_t nq,
                           uint32_t n, uint32_t K, uint32_t NB, hipStream_t s);
hipError_t launch_mbf_sweep(int mode, const MbfArgs& a, hipStream_t s);
hipError_t launch_mbf_out(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t K, uint32_t nq, uint32_t NB,
                          uint32_t* out, hipStream_t s);
hipError_t launch_mppr_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                            const uint32_t* src, uint32_t nq, uint32_t n, uint32_t K, uint32_t NB, double* dang,
                            hipStream_t s);
hipError_t launch_mppr_sweep(int mode, bool f64, const MpprArgs& a, hipStream_t s);
// qpart: [NB][256][64] float64 scratch; qsum: [NB][64]
hipError_t launch_mppr_out(bool f64, const void* x, double* qpart, double* qsum, uint32_t n, uint32_t nq, uint32_t NB,
                           double* out, hipStream_t s);

// Launchers (enqueue only; return the launch status).
// x = 1/n (psrc = kInf) or the one-hot vector of psrc; c = x / outdeg in
// slot order (both buffers when c1 is set); state rows 0..S: resid[0] = inf,
// dang[0] = d0, scale = 1 (when st.scale is set), counters 0.
hipError_t launch_pr_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                          uint32_t n, SweepState st, uint32_t S, double d0, uint32_t psrc, hipStream_t s);
hipError_t launch_pr_sweep(int mode, bool f64, const PrArgs& a, hipStream_t s);
hipError_t launch_bf_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, uint32_t n, uint32_t src,
                          SweepState st, uint32_t S, hipStream_t s);
// out[v] = d[cpos[v]]: distances back in vertex order.
hipError_t launch_bf_gather(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t* out, hipStream_t s);
hipError_t launch_bf_sweep(int mode, const BfArgs& a, hipStream_t s);
// out[v] = c[cpos[v]] for v < n (float or double): values in vertex order.
hipError_t launch_by_vertex(bool f64, const void* c, const uint32_t* cpos, uint32_t n, void* out, hipStream_t s);
// out[v] = x[v] / sum(x), sum in float64 with a fixed reduction order.
hipError_t launch_normalize(bool f64, const void* x, uint32_t n, double* out, double* scratch, hipStream_t s);
constexpr uint32_t kNormBlocks = 512;  // scratch needs kNormBlocks + 1 doubles
// Inputs of a synchronous float64 sweep that evaluates T(y) for the float64
// scores y (vertex order): x = y, c[cpos[v]] = y[v] / outdeg(v), and sweep
// state row 0 set to run once spreading the dangling mass of y.  The sweep's
// residual resid[1] is then ||T(y) - y||_1.  scratch: kNormBlocks + 1 doubles.
hipError_t launch_bound_setup(const double* y, double* x, double* c, const uint32_t* out_deg, const uint32_t* cpos,
                              uint32_t n, SweepState st, double* scratch, hipStream_t s);

// Sets of graphs stored as one union graph (disjoint vertex ranges).
// Distances 0 at k more sources (device array src of vertex ids), in both
// buffers when d1 is not null.
hipError_t launch_bf_more_sources(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, const uint32_t* src, uint32_t k,
                                  hipStream_t s);
// x[voff[g] .. voff[g+1]) /= its sum, for each of the G graphs (fixed order).
hipError_t launch_segment_normalize(double* x, const uint32_t* voff, uint32_t G, hipStream_t s);

// Access matrix of one pull sweep: counts[r * B + c] += reads by worker group r
// of values written by group c; *self += reads of a value the reader writes.
// vw: [n] scratch (worker of each vertex), inv: [K] scratch (vertex of each hot slot).
hipError_t launch_access_matrix(const Topology& g, uint32_t* vw, uint32_t* inv, uint32_t B,
                                unsigned long long* counts, unsigned long long* self, hipStream_t s);

// Serving (continuous batching): lanes admitted at a sweep boundary, rows of
// finished lanes.  lane_src: [NB][64] source per admitted lane, kInf elsewhere;
// blist: the nb batches that admit anything.
hipError_t launch_mbf_lane_init(uint32_t* d0, uint32_t* d1, const uint32_t* cpos, uint32_t n, uint32_t K,
                                const uint32_t* lane_src, const uint32_t* blist, uint32_t nb, hipStream_t s);
hipError_t launch_mppr_lane_init(bool f64, void* x, void* c0, void* c1, const uint32_t* out_deg, const uint32_t* cpos,
                                 uint32_t n, uint32_t K, uint32_t NB, const uint32_t* lane_src, const uint32_t* blist,
                                 uint32_t nb, uint32_t* src, double* dang, double* scale, uint32_t* qdone,
                                 double* rhist, hipStream_t s);
hipError_t launch_mbf_lane_out(const uint32_t* d, const uint32_t* cpos, uint32_t n, uint32_t K, uint32_t b, uint32_t q,
                               uint32_t* out, hipStream_t s);
// qpart: [256] float64 scratch
hipError_t launch_mppr_lane_out(bool f64, const void* x, uint32_t n, uint32_t b, uint32_t q, double* qpart,
                                double* out, hipStream_t s);

}  // namespace dg

/*
 * dg.h - C ABI of the delayed asynchronous graph sweep library (MI355X, gfx950).
 *
 * The library runs the per-iteration vertex-update sweep of two iterative
 * graph algorithms from Blanco, McMillan and Low, "Delayed Asynchronous
 * Iterative Graph Algorithms" (HPEC 2021):
 *
 *   - pull-style PageRank (section IV-A, dense updates: every vertex is
 *     recomputed from its in-neighbours every sweep);
 *   - pull-style Bellman-Ford single-source shortest paths with 32-bit
 *     unsigned path lengths (section IV-D);
 *
 * each in three commit modes (section III and figure 1):
 *
 *   DG_SYNC     outputs go to a separate array that becomes the input of the
 *               next sweep (Jacobi; one barrier per sweep, the kernel edge);
 *   DG_ASYNC    every new value is written to the single global array as
 *               soon as it is computed (delta = 0);
 *   DG_DELAYED  new values are staged in a workgroup-local buffer (LDS) and
 *               copied to the global array every d vertices of the worker's
 *               block and when the block is done (the paper's hybrid, delta=d).
 *
 *   DG_DELAYED_LOCAL  DG_DELAYED, and a worker reads the values of its own
 *               vertices from its staging buffer (newest, maybe not yet
 *               committed) instead of the global array: the local-read
 *               variant of section III-C, here as an ablation.  Staging is
 *               the per-vertex shadow array; sources in the compact region
 *               of high-out-degree vertices are read from the global array.
 *               dg_pagerank and dg_sssp only.
 *
 * Other reads come from the global array (the global-read variant of section
 * III-C).  Work is split into contiguous vertex blocks, one per persistent
 * workgroup ("worker"), balanced by in-edges (section III-A).
 *
 * Conventions for every function:
 *   - every function returns a dg_status; nothing throws or aborts across the
 *     ABI; on error dg_last_error() returns a message for the calling thread;
 *   - argument validation happens on the host before any HIP call, and on a
 *     validation error no output is touched;
 *   - `hip_stream` is a hipStream_t (NULL = the legacy default stream); all
 *     device work of a call is enqueued on it and the call returns after the
 *     result is complete (the stream is synchronised);
 *   - one graph handle may be used by one call at a time; distinct handles may
 *     run concurrently on distinct streams.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_ERR_INVALID_ARGUMENT = 1, /* malformed input; nothing was changed        */
  DG_ERR_OUT_OF_MEMORY = 2,    /* a device or host allocation failed         */
  DG_ERR_DEVICE = 3,           /* a HIP call failed (no device, fault, ...)  */
  DG_ERR_NOT_CONVERGED = 4,    /* max_sweeps reached; outputs and stats hold
                                  the last iterate                            */
  DG_ERR_UNSUPPORTED = 5       /* valid request the library cannot run       */
} dg_status;

/* Commit mode of a sweep (section III). */
typedef enum { DG_SYNC = 0, DG_ASYNC = 1, DG_DELAYED = 2, DG_DELAYED_LOCAL = 3 } dg_mode;

/* Layout of the adjacency handed to dg_graph_create.
 * DG_CSR: ptr is indexed by source vertex, idx holds destinations (out-edges).
 * DG_CSC: ptr is indexed by destination vertex, idx holds sources (in-edges). */
typedef enum { DG_CSR = 0, DG_CSC = 1 } dg_layout;

/* Storage precision of PageRank scores.  Sums over in-edges, the residual,
 * the dangling mass and the final normalisation are float64 in both. */
typedef enum { DG_F32 = 0, DG_F64 = 1 } dg_dtype;

/* Commit interval meaning "the worker's whole block": flush only when the
 * worker's block is done (or the staging buffer is full). */
#define DG_D_WHOLE 0xFFFFFFFFu

/* Distance of a vertex the source cannot reach. */
#define DG_INF_DIST 0xFFFFFFFFu

typedef struct dg_graph dg_graph;

/* Per-call statistics.  Every field is written by the call except
 * `request`, which the caller sets (zero-initialise the struct otherwise).
 *
 * Commit granularity.  A worker computes the vertices of one tile (up to
 * 1024 consecutive vertices) at once, after all of the tile's gathers, so a
 * commit can only fall between tiles: in DG_DELAYED a worker commits at the
 * end of the first tile that brings its staged count to >= d (and at the end
 * of its block).  Any d up to the tile size therefore commits after every
 * tile; `commit_interval` reports the interval that took effect. */
#define DG_STATS_ERR_BOUND 1u
typedef struct {
  uint32_t sweeps;          /* sweeps run, including the confirming one     */
  uint32_t workers;         /* persistent workgroups (contiguous blocks)    */
  uint32_t tile_vertices;   /* mean vertices per tile: n / tiles, rounded
                               (batched calls: per batched tile)            */
  uint32_t commit_interval; /* delayed modes: mean vertices per commit of a
                               worker's staged values, n / commits, rounded
                               (>= d up to the end of a block); 0 otherwise */
  double residual;          /* PageRank: L1 change of the last sweep        */
  double seconds;           /* time to convergence: first sweep launch to
                               the end of the sweep that met the stopping
                               rule, measured with events on the stream     */
  uint64_t edges_traversed; /* m * sweeps                                   */
  double err_bound;         /* dg_pagerank and dg_ppr, when `request` holds
                               DG_STATS_ERR_BOUND: ||T(x) - x||_1 / (1 -
                               damping) for the returned scores x and the
                               call's map T, computed on the device in
                               float64 after the sweeps (one more pull
                               sweep, not part of `seconds`).  T is an L1
                               contraction with factor damping, so this
                               bounds the L1 distance of x to the exact
                               fixed point; it overstates it by at most
                               (1 + damping) / (1 - damping).  0 otherwise. */
  uint32_t request;         /* in: DG_STATS_ERR_BOUND, or 0                 */
  uint32_t commits;         /* delayed modes: commits per sweep, over all
                               workers; 0 otherwise                         */
} dg_stats;

/* Static facts about an uploaded graph. */
typedef struct {
  uint32_t n;          /* vertices                                         */
  uint64_t m;          /* edges                                            */
  uint32_t workers;    /* persistent workgroups used by the sweeps         */
  uint32_t tiles;      /* tiles over all workers                           */
  uint32_t max_in_degree;
  uint32_t dangling;   /* vertices with out-degree 0                       */
  uint32_t has_weights;
  uint32_t compute_units;
  uint32_t hot_vertices; /* sources stored in the compact region            */
  uint64_t hot_edges;    /* in-edges whose source is in the compact region  */
  uint32_t resident_vertices; /* leading compact-region sources in the LDS table */
  uint64_t resident_edges;    /* in-edges whose source is in the table          */
  uint32_t weight_bytes;      /* bytes per stored weight: 1 when every weight is
                                 <= 255, 4 otherwise, 0 without weights        */
  uint64_t device_bytes; /* device memory held by the graph (not workspace) */
  uint32_t sweep_variant; /* DG_SWEEP_WIDE, _WIDE_INFLIGHT or _NARROW          */
  uint32_t batch_tiles;   /* tiles of the batched calls: each tile split into
                             runs of at most 4096 in-edges (a vertex with more
                             is a run of its own), at most one batched worker
                             per run                                        */
} dg_graph_info;

/* Device memory hooks.  alloc(bytes, stream, ctx) returns device memory or
 * NULL; free(ptr, stream, ctx) releases it.  Passing NULL for both restores
 * hipMalloc/hipFree.  The hooks apply to allocations made after the call; a
 * graph frees its memory with the hooks that allocated it, so they must stay
 * valid until every graph created under them is destroyed. */
typedef void* (*dg_alloc_fn)(size_t bytes, void* hip_stream, void* ctx);
typedef void (*dg_free_fn)(void* ptr, void* hip_stream, void* ctx);
dg_status dg_set_allocator(dg_alloc_fn alloc, dg_free_fn free_fn, void* ctx);

/* Options of dg_graph_create (pass NULL for the defaults).
 *   workers       persistent workgroups that own the contiguous vertex blocks
 *                 of the single-query sweeps; 0 = automatic (one 1024-thread
 *                 workgroup per compute unit, at most one per tile).  The
 *                 batched calls use tiles and partitions of their own: the
 *                 tiles cut into runs of at most 4096 in-edges
 *                 (dg_graph_info.batch_tiles), split per algorithm over
 *                 256-thread workgroups, eight per compute unit for SSSP
 *                 (dg_sssp_batch, the server's SSSP pools) and five for
 *                 personalised PageRank (dg_ppr_batch, its PPR pools), at
 *                 most one per run.
 *   hot_vertices  at most this many sources with the largest out-degree (and
 *                 above-average out-degree) get their published value stored
 *                 in a compact region after the n regular slots, so gathers
 *                 from them hit in L2; ownership, blocks and commit points are
 *                 unchanged, only the storage address moves.
 *                 DG_HOT_AUTO = 524288, 0 = no compact region
 *   resident_vertices
 *                 at most this many of the compact region's sources, those
 *                 with the largest out-degree, are also read from a copy in
 *                 each workgroup's LDS (the resident table) instead of being
 *                 gathered; at most 32768 (a float64 sweep uses the first
 *                 16384).  DG_RESIDENT_AUTO = 32768 if those cover at least
 *                 1/16 of the in-edges, else 0; 0 = no table.  A read of a
 *                 resident source returns, in
 *                   DG_SYNC     the value of the previous sweep, exactly as a
 *                               gather would;
 *                   DG_ASYNC, DG_DELAYED, DG_DELAYED_LOCAL
 *                               a value read from the global array at most
 *                               four tiles of the reader earlier (the table
 *                               is refreshed a quarter at a time after each
 *                               tile), instead of at the moment of the read.
 *                 Results converge to the same fixed point / distances.
 *   sweep_variant how the single-query sweep kernels spread a tile's in-edges
 *                 over a workgroup's threads (all compute the same values):
 *                   DG_SWEEP_WIDE       16 in-edges per thread, tiles of at
 *                                       most 16380 in-edges; the gathers of a
 *                                       wave are paced by its resident-table
 *                                       reads (best with many tiles per worker)
 *                   DG_SWEEP_WIDE_INFLIGHT
 *                                       the same tiles, all of a thread's
 *                                       gathers in flight at once
 *                   DG_SWEEP_NARROW     8 per thread, tiles of at most 8188
 *                                       in-edges, all gathers in flight (best
 *                                       for small graphs)
 *                 DG_SWEEP_AUTO (0): NARROW if the wide tiles number fewer
 *                 than 2 per default worker, else WIDE_INFLIGHT up to 8 per
 *                 default worker, else WIDE.  The choice is reported in
 *                 dg_graph_info.sweep_variant. */
#define DG_HOT_AUTO 0xFFFFFFFFu
#define DG_RESIDENT_AUTO 0xFFFFFFFFu
#define DG_SWEEP_AUTO 0u
#define DG_SWEEP_WIDE 1u
#define DG_SWEEP_WIDE_INFLIGHT 2u
#define DG_SWEEP_NARROW 3u
typedef struct {
  uint32_t workers;
  uint32_t hot_vertices;
  uint32_t resident_vertices;
  uint32_t sweep_variant;
  uint32_t arrays_on_device; /* 1: ptr, idx and w of dg_graph_create are
                                device memory (see there); 0: host memory */
} dg_graph_opts;

/* Upload a graph and build its in-edge form (pull sweeps need in-neighbours,
 * section III-A).
 *   n          vertices, 1 <= n; n plus the compact-region slots must stay
 *              below 2^29 (DG_ERR_UNSUPPORTED otherwise)
 *   m          edges, m < 2^32 - 4096
 *   layout     DG_CSR or DG_CSC (see dg_layout)
 *   ptr        array of n+1 uint64 offsets: ptr[0] = 0, non-decreasing,
 *              ptr[n] = m
 *   idx        array of m uint32 vertex ids, each < n
 *   w          array of m uint32 edge weights, or NULL (PageRank only).
 *              Path lengths saturate at DG_INF_DIST.  When every weight is
 *              <= 255 the device keeps them as bytes (dg_graph_info.
 *              weight_bytes), which shortens the sweeps' weight stream.
 *   opts       creation options, or NULL for the defaults
 * The three arrays are host memory, or device memory of the current device
 * when opts->arrays_on_device is 1 (then they are read on hip_stream after
 * the work already queued on it; the in-edge form, tiles and partition are
 * built on the host from a copy, so the call moves the arrays over PCIe
 * once each way).  Device arrays are validated after that copy, with the
 * same rules; a pointer that is not device memory is INVALID_ARGUMENT.
 * Duplicate edges are kept (PageRank counts multiplicity, SSSP takes the
 * minimum) and self-loops count in the out-degree.  The arrays are copied:
 * the caller keeps ownership and may free them when the call returns.  On
 * success *out owns device memory until dg_graph_destroy.
 * Errors: INVALID_ARGUMENT (malformed arrays, NULL pointers,
 * arrays_on_device not 0 or 1), OUT_OF_MEMORY, DEVICE. */
dg_status dg_graph_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr,
                          const uint32_t* idx, const uint32_t* w, const dg_graph_opts* opts,
                          void* hip_stream, dg_graph** out);

/* Release a graph and its workspace.  NULL is a no-op. */
dg_status dg_graph_destroy(dg_graph* g);

/* Fill *info with static facts about g. */
dg_status dg_graph_info_get(const dg_graph* g, dg_graph_info* info);

/* Layout plans: the host-side part of dg_graph_create, without a device.
 * dg_plan_create validates the arrays exactly as dg_graph_create does and
 * builds what it would upload for a device of `compute_units` compute units
 * (>= 1): the in-edge form with source slots (section III-A: pull sweeps read
 * in-neighbours), the compact region and its resident table, the tiles, and
 * the blocked worker partition balanced by in-edges (section III-A).  For
 * inspecting a layout before uploading it, and for testing it on machines
 * without a GPU.  Arguments and errors as dg_graph_create, except DEVICE,
 * which cannot occur, and opts->arrays_on_device, which must be 0 (a plan is
 * built without a device); *out is owned by the caller until dg_plan_destroy. */
typedef struct dg_plan dg_plan;
typedef struct {
  uint32_t n;
  uint64_t m;
  uint32_t workers;           /* worker blocks                                  */
  uint32_t tiles;
  uint32_t max_in_degree;
  uint32_t dangling;
  uint32_t hot_vertices;      /* K: sources in the compact region               */
  uint64_t hot_edges;
  uint32_t resident_vertices; /* R: leading compact-region slots in the table   */
  uint64_t resident_edges;
  uint32_t weight_bytes;      /* 1, 4, or 0 without weights                     */
  uint64_t content_hash;      /* hash of the in-edge form (the tuning cache key) */
  uint32_t sweep_variant;     /* DG_SWEEP_WIDE, _WIDE_INFLIGHT or _NARROW        */
  uint32_t batch_tiles;       /* tiles of the batched calls (as dg_graph_info)  */
  uint32_t batch_workers_sssp; /* default batched partitions on compute_units:  */
  uint32_t batch_workers_ppr;  /* SSSP and personalised PageRank workers        */
} dg_plan_info;
dg_status dg_plan_create(uint32_t n, uint64_t m, dg_layout layout, const uint64_t* ptr, const uint32_t* idx,
                         const uint32_t* w, const dg_graph_opts* opts, uint32_t compute_units, dg_plan** out);
dg_status dg_plan_info_get(const dg_plan* p, dg_plan_info* info);
/* Copies the plan into caller arrays; any pointer may be NULL to skip it.
 *   in_ptr [n+1]    in-edge offsets
 *   in_src [m]      slot of each in-edge's source: the vertex itself, or
 *                   n + rank for the K compact-region sources (the first R
 *                   of them are the resident table)
 *   in_w   [m]      the weight of each in-edge, widened to uint32
 *                   (INVALID_ARGUMENT if the graph has none)
 *   cpos   [n]      slot of each vertex's published value
 *   tile_v [tiles+1]  first vertex of each tile
 *   work_t [workers+1] first tile of each worker */
dg_status dg_plan_arrays(const dg_plan* p, uint32_t* in_ptr, uint32_t* in_src, uint32_t* in_w, uint32_t* cpos,
                         uint32_t* tile_v, uint32_t* work_t);
/* Copies the batched calls' layout into caller arrays (host memory); any
 * array pointer may be NULL to skip it.
 *   btile_v   [batch_tiles+1]        first vertex of each tile of the batched calls
 *   work_sssp [batch_workers_sssp+1] first batched tile of each worker of the
 *   work_ppr  [batch_workers_ppr+1]  default SSSP and PPR partitions */
dg_status dg_plan_batch_tiles(const dg_plan* p, uint32_t* btile_v, uint32_t* work_sssp, uint32_t* work_ppr);
dg_status dg_plan_destroy(dg_plan* p);

/* PageRank by repeated pull sweeps (sections III and IV-A).
 *   damping     0 <= damping < 1 (0.85 is the customary value)
 *   tol         stop after the first sweep whose L1 score change is < tol
 *               (the paper's stopping rule with a threshold); tol >= 0, finite;
 *               tol = 0 runs exactly max_sweeps sweeps
 *   mode, d     commit mode; d >= 1 is the commit interval in vertices for
 *               DG_DELAYED (DG_D_WHOLE = whole block) and ignored otherwise
 *   dtype       score storage precision
 *   max_sweeps  1 <= max_sweeps <= 1000000
 *   out_scores  n float64 scores normalised to sum 1; device memory when
 *               out_on_device != 0, else host memory
 *   stats       may be NULL
 * Scores start at 1/n.  The mass of dangling vertices (out-degree 0) is spread
 * evenly over all vertices; a sweep spreads 1 minus the mass the non-dangling
 * vertices held after the previous sweep, which equals the dangling mass when
 * the scores sum to 1 (always, in synchronous mode) and also returns any mass
 * an asynchronous sweep lost or gained.  The residual of a sweep is the sum
 * over vertices of |new score - previous stored score|, the new score taken
 * in float64 before rounding to the storage precision.
 * Returns NOT_CONVERGED (with out_scores and stats filled) when max_sweeps
 * sweeps ran without meeting the stopping rule. */
dg_status dg_pagerank(dg_graph* g, double damping, double tol, dg_mode mode, uint32_t d,
                      dg_dtype dtype, uint32_t max_sweeps, double* out_scores,
                      int out_on_device, dg_stats* stats, void* hip_stream);

/* Personalised PageRank of one restart vertex by repeated pull sweeps: the
 * single-query form of dg_ppr_batch, on the sweep kernels of dg_pagerank
 * (same partition, commit modes, staging and resident table).  It computes
 *   x = (1 - damping) e_s + damping (A x + D(x) e_s),  s = src,
 * where D(x) is the mass on dangling vertices: teleport and dangling mass
 * both return to the restart vertex (the reading used for batched queries).
 * Scores start at e_s.  After every sweep the vector is rescaled to mass 1
 * (a per-sweep float64 factor; stored values are never touched): the fixed
 * point has mass 1, and the rescale removes the mass error that
 * asynchronous and delayed commits leave.  The stopping rule, tol, dtype,
 * d, max_sweeps and outputs are those of dg_pagerank (scores normalised to
 * sum 1; stats.err_bound, when requested, is the certificate of this map).
 * The stopping rule bounds a synchronous iterate's L1 error by
 * damping / (1 - damping) x tol (5.7 tol at 0.85), so an error of 1e-6 needs
 * tol <= 1.5e-7, which float32 storage reaches on R-MAT, banded and
 * dangling-heavy graphs (measured).  Where float32 rounding keeps the change
 * above tol (mass on a few vertices can settle into a period-2 cycle near
 * 2e-7), DG_F32 also stops at the first sweep whose change is below 2 tol and
 * more than 0.9 times the change two sweeps earlier (exact synchronous
 * changes shrink by damping^2 over two sweeps); stats.residual then holds
 * that change, >= tol.
 *   src   restart vertex, < n
 * Not for the union graph of a set (DG_ERR_UNSUPPORTED). */
dg_status dg_ppr(dg_graph* g, uint32_t src, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                 uint32_t max_sweeps, double* out_scores, int out_on_device, dg_stats* stats, void* hip_stream);

/* Error certificate of any score vector x (n float64 values, normalised to
 * sum 1 by the caller): ||T(x) - x||_1 / (1 - damping) for the PageRank map T
 * of dg_pagerank (restart = DG_NO_RESTART) or the personalised map of dg_ppr
 * with that restart vertex, computed on the device in float64 by one
 * synchronous sweep.  T is an L1 contraction with factor damping, so the
 * value bounds the L1 distance of x to the exact fixed point, and is at most
 * (1 + damping) / (1 - damping) times that distance.  For the results of
 * dg_ppr_batch and the server, which report no bound themselves.
 *   scores       device memory when scores_on_device != 0, else host memory
 *   out_bound    host double
 * Uses the graph's workspace: not concurrently with another call on g. */
#define DG_NO_RESTART 0xFFFFFFFFu
dg_status dg_error_bound(dg_graph* g, double damping, uint32_t restart, const double* scores, int scores_on_device,
                         double* out_bound, void* hip_stream);

/* Bellman-Ford single-source shortest paths by repeated pull relaxation
 * sweeps (sections III and IV-D): d'(v) = min(d(v), min over in-edges
 * (u,v) of d(u) + w(u,v)), stored every sweep, stopping after the first
 * sweep in which no distance decreased.
 *   src         source vertex, < n
 *   mode, d     as for dg_pagerank
 *   max_sweeps  1 <= max_sweeps <= 1000000
 *   out_dist    n uint32 distances, DG_INF_DIST for unreachable vertices;
 *               device memory when out_on_device != 0, else host memory
 * Requires a graph created with weights.  Distances are exact whenever the
 * longest shortest path is below 2^32 - 1. */
dg_status dg_sssp(dg_graph* g, uint32_t src, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                  uint32_t* out_dist, int out_on_device, dg_stats* stats, void* hip_stream);

/* Batched queries (forms beyond the paper's single query: many sources swept
 * together on one graph).  Queries are grouped 64 to a batch and every
 * batch of a call runs in the same sweep launches; values are stored
 * vertex-major so one gather serves the 64 queries of a batch.  Each batch
 * stops when all its queries met the stopping rule; the call returns when
 * every batch has.  Commit modes are those of the single-query calls.  A
 * batched worker's four wavefronts take its vertices in turn, one at a time
 * (not a tile at once), so DG_DELAYED commits every d vertices of the worker
 * within a tile too: each wavefront commits its own staged rows every
 * ceil(d/4) of its vertices, and at the end of the block.
 *   sources     host array of k vertex ids (< n); k >= 1
 *   max_sweeps  1 <= max_sweeps <= 100000
 *   stats       sweeps = sweeps until every batch converged;
 *               edges_traversed = m * sum over queries of their batch's sweeps;
 *               workers = the batched partition's workers; in DG_DELAYED,
 *               commits = commits per sweep of one batch, over every
 *               wavefront of every worker, and commit_interval = n / commits
 *
 * dg_sssp_batch: Bellman-Ford from each source (as dg_sssp).
 *   out_dist    k rows of n uint32: row q holds the distances from sources[q]
 *
 * dg_ppr_batch: personalised PageRank with a one-hot restart vector per
 * query: x = (1 - damping) e_s + damping (A x + D(x) e_s), where D(x) is the
 * mass on dangling vertices, i.e. teleport and dangling mass both return to
 * the restart vertex s = sources[q].  Scores are stored in float32 or
 * float64 (dtype) with float64 sums, residuals and normalisation.  After
 * every sweep each query's vector is rescaled to mass 1 (a per-query factor,
 * no extra pass over memory): the fixed point has mass 1, and the rescale
 * removes the mass error that Gauss-Seidel-ordered sweeps accumulate.  Each
 * query stops at the first sweep whose L1 change for that query is < tol and
 * its row is the iterate of that sweep (later sweeps of its batch leave it
 * untouched), so a row does not depend on the other queries of the call in
 * synchronous mode.  Float32 storage has a noise floor: the L1 change of a
 * sweep cannot settle much below the rounding of a vector of mass 1 (about
 * 1e-7).  The stopping rule bounds a synchronous row's L1 error by
 * damping / (1 - damping) x tol, so 1e-6 needs tol <= 1.5e-7, which float32
 * rows reach on R-MAT, banded and dangling-heavy graphs (measured).  A
 * float32 query also stops at its rounding floor, by the rule of dg_ppr: a
 * change below 2 tol that is more than 0.9 times its change two sweeps
 * earlier.
 *   damping     0 <= damping < 1
 *   dtype       DG_F32 or DG_F64
 *   out_scores  k rows of n float64, each normalised to sum 1 */
dg_status dg_sssp_batch(dg_graph* g, const uint32_t* sources, uint32_t k, dg_mode mode, uint32_t d,
                        uint32_t max_sweeps, uint32_t* out_dist, int out_on_device, dg_stats* stats,
                        void* hip_stream);
dg_status dg_ppr_batch(dg_graph* g, const uint32_t* sources, uint32_t k, double damping, double tol,
                       dg_mode mode, uint32_t d, dg_dtype dtype, uint32_t max_sweeps, double* out_scores,
                       int out_on_device, dg_stats* stats, void* hip_stream);

/* The static blocked partition (section III-A) of a graph: worker w owns
 * vertices [out_first_vertex[w], out_first_vertex[w+1]).
 *   out_first_vertex  host array of workers + 1 entries (dg_graph_info) */
dg_status dg_graph_partition(const dg_graph* g, uint32_t* out_first_vertex, void* hip_stream);

/* Re-partitions the single-query sweeps of a resident graph over `workers`
 * workers (0 = the default, one per compute unit rounded down to a multiple
 * of 8), without re-uploading it.  The blocked partition is rebuilt as at
 * creation (section III-A); more workers than compute units run in turn.
 * Must not overlap a sweep call on the same graph. */
dg_status dg_graph_repartition(dg_graph* g, uint32_t workers, void* hip_stream);

/* Changes how the single-query sweeps map a resident graph onto the GPU,
 * without re-uploading it (a form beyond the paper, for the autotuner):
 *   sweep_variant      DG_SWEEP_WIDE, _WIDE_INFLIGHT or _NARROW, or
 *                      DG_SWEEP_AUTO for the variant chosen at creation; a
 *                      switch to or from DG_SWEEP_NARROW rebuilds the tiles
 *                      (its tile cap differs), the batched calls' runs cut
 *                      from them, and every partition over either
 *   resident_vertices  at most this many resident-table entries are read
 *                      from LDS (<= dg_graph_info.resident_vertices; 0 = no
 *                      table; DG_RESIDENT_AUTO = all of them)
 *   workers            as dg_graph_repartition (0 = the default)
 * Results do not change beyond the reordering of floating-point sums and the
 * timing-dependent commits of the asynchronous modes.  Not for the union
 * graph of a set.  Must not overlap a sweep call on the same graph. */
dg_status dg_graph_set_mapping(dg_graph* g, uint32_t sweep_variant, uint32_t resident_vertices, uint32_t workers,
                               void* hip_stream);

/* Captured launches (a form beyond the paper, which runs one sweep after
 * another on the CPU; here for graphs whose sweeps are short enough that
 * launching them costs time).  chunk_sweeps = 0 (the default) launches every
 * sweep on its own; 1..64 records chunks of that many consecutive sweeps into
 * HIP graphs and replays them with one launch each.  It applies to every
 * later dg_pagerank, dg_ppr, dg_sssp, dg_sssp_batch and dg_ppr_batch call on
 * the graph (and to dg_set_* through dg_set_set_capture).
 *  - Chunk j (sweeps j*chunk_sweeps ..) is recorded the first time a call of
 *    the same shape reaches it and kept for later calls of that shape: same
 *    entry point, mode, d, dtype, tol, damping, max_sweeps, restart vertex
 *    and the same device buffers (the graph's own workspace, reused by the
 *    single-query calls; the batched calls allocate theirs per call and are
 *    recorded again when an address differs).  At most 256 chunks are kept
 *    per shape; a call beyond them launches its later sweeps one by one.
 *    A call of another shape replaces the recorded chunks.
 *  - Results are those of the eager launches: the replayed kernels and
 *    arguments are the same (bit for bit in synchronous mode).  Sweeps after
 *    the converging one in its chunk exit at once on the device; stats.seconds
 *    runs to the end of that chunk.
 *  - The recorded graphs hold device memory until the shape changes, the
 *    setting changes, dg_graph_set_mapping / dg_graph_repartition is called,
 *    or the graph is destroyed.
 * Errors: DG_ERR_INVALID_ARGUMENT for a NULL graph or chunk_sweeps > 64;
 * recording failures surface as DG_ERR_DEVICE from the sweep call.  Must not
 * overlap a sweep call on the same graph. */
dg_status dg_graph_set_capture(dg_graph* g, uint32_t chunk_sweeps);

/* Autotuner (a form beyond the paper, which leaves the choice of delta to
 * future work and shows that it depends on topology, thread count and update
 * density: sections IV and V).  Chooses, for one algorithm on one graph:
 *   1. the commit mode and interval: a full run of every candidate (sync,
 *      async, delayed with d in {16, 64, 256, 1024, 4096, whole}) at the
 *      current mapping gives its sweep count;
 *   2. the partition size: for 1, 2, 3 and 4 sweep workgroups per compute
 *      unit (rounded down to a multiple of 8), a 6-sweep probe of every
 *      candidate gives its time per sweep (best of two); the least predicted
 *      time to convergence (sweeps x time per sweep) wins;
 *   3. the mapping, for that mode, d and partition: every sweep variant
 *      (wide, wide with all gathers in flight, narrow) with the whole
 *      resident table, half of it and none, each run to convergence three
 *      times; the least median time wins;
 *   4. the launch: one launch per sweep against chunks of 16 captured sweeps
 *      (dg_graph_set_capture), three runs each; the lesser median wins and
 *      the graph keeps that setting (stages 1-3 and the default run with one
 *      launch per sweep).
 * The choice and the default (the mapping and partition chosen at creation,
 * delayed d = 64) are each run to convergence three times: their median,
 * fastest and slowest times are reported.  The graph is left with the chosen
 * partition and mapping (with DG_TUNE_KEEP_WORKERS neither changes and only
 * stage 1 runs, at the current partition).  Results are cached in-process by
 * the graph's 64-bit content hash, the algorithm, dtype, tol and source; a
 * cached entry is applied and returned at once (from_cache = 1) unless
 * DG_TUNE_NO_CACHE.
 *   algo   DG_ALGO_PAGERANK (damping 0.85, tol > 0, dtype) or DG_ALGO_SSSP
 *          (source src; tol and dtype ignored) */
typedef enum { DG_ALGO_PAGERANK = 0, DG_ALGO_SSSP = 1 } dg_algo;
#define DG_TUNE_NO_CACHE 1u
#define DG_TUNE_KEEP_WORKERS 2u
typedef struct {
  uint32_t workers;          /* chosen partition size (now the graph's) */
  dg_mode mode;              /* chosen commit mode */
  uint32_t d;                /* chosen commit interval (delayed) */
  uint32_t sweeps;           /* sweeps of the last measuring run */
  double seconds;            /* median time to convergence of the choice */
  double predicted_seconds;  /* the sweep-count x sweep-time model's estimate */
  uint32_t candidates;       /* configurations evaluated */
  uint32_t from_cache;
  uint64_t graph_hash;       /* content hash of the graph */
  uint32_t sweep_variant;    /* chosen sweep variant (now the graph's) */
  uint32_t resident_vertices; /* chosen resident-table limit, or DG_RESIDENT_AUTO */
  uint32_t repeats;          /* timed runs of the choice and of the default */
  uint32_t capture_chunk;    /* chosen captured-launch chunk (dg_graph_set_capture), 0 = one launch per sweep */
  double seconds_min, seconds_max;                 /* fastest and slowest run of the choice */
  double default_seconds;                          /* median of the default */
  double default_seconds_min, default_seconds_max; /* fastest and slowest run of the default */
} dg_tuning;
dg_status dg_tune(dg_graph* g, dg_algo algo, dg_dtype dtype, double tol, uint32_t src, uint32_t flags,
                  dg_tuning* out, void* hip_stream);

/* Autotuner of the batched calls (dg_sssp_batch, or dg_ppr_batch for
 * DG_ALGO_PAGERANK with damping 0.85, tol and dtype): on the given sample of
 * k (1..1024) sources, every commit mode and interval (sync, async, delayed
 * d in {16, 64, 256, whole}) for 3, 5 and 8 batched workgroups per compute
 * unit, each run three times; the least median time wins, and the graph's
 * batched partition for that algorithm (SSSP: dg_sssp_batch and the server's
 * SSSP pools; PageRank: dg_ppr_batch and its PPR pools) is left at the
 * chosen size.  The default is delayed d = 64 with 8 (SSSP) or 5 (PageRank)
 * workgroups per compute unit.  A live server's PPR pools resize their
 * per-worker partials at their next sweep.  Fills dg_tuning as dg_tune
 * (predicted_seconds = the measured median; sweep_variant and
 * resident_vertices are unchanged); nothing is cached.  flags must be 0. */
dg_status dg_tune_batch(dg_graph* g, dg_algo algo, dg_dtype dtype, double tol, const uint32_t* sources, uint32_t k,
                        uint32_t flags, dg_tuning* out, void* hip_stream);

/* Re-partitions the batched calls of one algorithm (DG_ALGO_SSSP:
 * dg_sssp_batch and the server's SSSP pools; DG_ALGO_PAGERANK: dg_ppr_batch
 * and its PPR pools) over `workers` 256-thread workgroups per batch (0 = the
 * default: 8 per compute unit for SSSP, 5 for PageRank, rounded down to a
 * multiple of 8), at most one per batched tile (dg_graph_info.batch_tiles),
 * as dg_tune_batch leaves it after tuning.  A live server's PPR pools resize
 * their per-worker partials at their next sweep.  Must not overlap a sweep
 * call on the same graph. */
dg_status dg_graph_repartition_batch(dg_graph* g, dg_algo algo, uint32_t workers, void* hip_stream);

/* The in-process cache of tuning results: cleared, written to and merged
 * from a text file (one result per line, comments start with '#'). */
dg_status dg_tune_cache_clear(void);
dg_status dg_tune_cache_save(const char* path);
dg_status dg_tune_cache_load(const char* path);

/* Topology instrumentation (section IV, effects of graph topology, Fig. 5):
 * the access matrix of one pull sweep under the graph's static blocked
 * partition.  Each in-edge u -> v is a read, by the worker owning v, of the
 * value the worker owning u writes; workers are coarsened into `groups`
 * groups of consecutive workers (8 groups = one per XCD), giving a coarsened
 * adjacency matrix.  The paper finds that delaying commits pays little when
 * reads cluster on the diagonal (a worker mostly reads what it writes itself)
 * and pays when they are spread.
 *   groups      1 <= groups <= min(64, workers)
 *   out_counts  host array of groups*groups (row: reading group, column:
 *               owning group), or NULL
 *   stats       totals and shares, or NULL (not both NULL) */
typedef struct {
  uint64_t reads;           /* in-edges: the gathers of one sweep */
  uint64_t same_worker;     /* reads of a value the reading worker writes itself */
  uint64_t diagonal;        /* reads within the reading group (matrix diagonal) */
  uint32_t groups;
  uint32_t workers;
  double self_share;        /* same_worker / reads */
  double diagonal_share;    /* diagonal / reads */
  double uniform_diagonal;  /* diagonal share expected if reads ignored the reader:
                               sum over groups of row share x column share */
} dg_access_stats;
dg_status dg_access_matrix(dg_graph* g, uint32_t groups, uint64_t* out_counts, dg_access_stats* stats,
                           void* hip_stream);

/* Commit-mode predictor (sections IV-C and V: when reads cluster, so that a
 * worker mostly reads values written within its own part of the machine,
 * buffering its commits only delays what it reads itself; when reads are
 * spread, delaying commits cuts the contention on shared lines).  From the
 * access matrix with one group per XCD (8 groups, or one per worker when
 * there are fewer), without running a sweep:
 *   lift = diagonal_share / uniform_diagonal
 *   lift >= DG_PREDICT_CLUSTER_LIFT: DG_ASYNC (commits unbuffered);
 *   otherwise: DG_DELAYED with d = 64 (one commit per tile, the finest
 *   interval the sweeps have).
 * The same choice serves PageRank and SSSP.  Costs one access-matrix pass
 * (about one sweep).  Errors as dg_access_matrix. */
#define DG_PREDICT_CLUSTER_LIFT 2.0
typedef struct {
  dg_mode mode;            /* predicted commit mode */
  uint32_t d;              /* commit interval for DG_DELAYED, else 0 */
  uint32_t groups;         /* groups of the access matrix used */
  uint32_t reserved;
  double diagonal_share;   /* as dg_access_stats */
  double uniform_diagonal;
  double lift;             /* diagonal_share / uniform_diagonal */
  double self_share;
} dg_prediction;
dg_status dg_predict_mode(dg_graph* g, dg_prediction* out, void* hip_stream);

/* Graph sets (a form beyond the paper's single graph: many graphs, of uneven
 * sizes, resident together and swept in one launch per sweep).  The graphs
 * are stored as one union graph (graph i's vertices follow those of graphs
 * 0..i-1; no edge crosses two graphs) and swept by the single-graph kernels
 * in the commit modes of section III, so one launch serves every graph and
 * the blocked partition balances the union's edges over the GPU.
 *  - SSSP: every graph's Bellman-Ford starts from its own source; each
 *    graph's distances are exactly those of dg_sssp on it.
 *  - PageRank: the union's PageRank restricted to one graph and renormalised
 *    to sum 1 equals that graph's own (each graph's dangling mass is spread
 *    over its own vertices, so the graph keeps the mass it starts with and
 *    iterates as it would alone).  Each graph stops on its own L1 change
 *    (see dg_set_pagerank).
 * A graph that met its stopping rule is no longer swept, while the others
 * go on; out_sweeps reports each graph's own sweep count. */
typedef struct dg_set dg_set;

typedef struct {
  uint32_t n;           /* vertices, >= 1 */
  uint64_t m;           /* edges */
  const uint64_t* ptr;  /* host, n+1 out-edge offsets (CSR), ptr[0] = 0, ptr[n] = m */
  const uint32_t* idx;  /* host, m destinations < n */
  const uint32_t* w;    /* host, m weights, or NULL (all graphs of a set alike) */
} dg_graph_desc;

typedef struct {
  uint32_t workers;  /* workgroups per sweep; 0 = 5 per compute unit.  Every
                        graph gets at least one worker of its own (so a set
                        of more graphs than this uses one per graph), the
                        rest go to graphs by their sweep cost (in-edges plus
                        per-vertex and per-tile terms). */
} dg_set_opts;

typedef struct {
  uint32_t graphs;
  uint64_t n;        /* vertices over all graphs */
  uint64_t m;        /* edges over all graphs */
  uint32_t tiles;
  uint32_t workers;
  uint32_t has_weights;
  uint64_t device_bytes;
} dg_set_info;


/* Builds and uploads a set of `count` graphs (host CSR arrays; copied, not
 * retained) as one union graph whose tiles and worker blocks never cross a
 * graph boundary.  Limits: total vertices < 2^31, total edges < 2^32 - 2^12. */
dg_status dg_set_create(uint32_t count, const dg_graph_desc* graphs, const dg_set_opts* opts, void* hip_stream,
                        dg_set** out);
dg_status dg_set_destroy(dg_set* s);
dg_status dg_set_info_get(const dg_set* s, dg_set_info* info);
/* dg_graph_set_capture for the set's union graph: later dg_set_pagerank and
 * dg_set_sssp calls run as recorded chunks of chunk_sweeps sweeps (0 = one
 * launch per sweep).  Errors as dg_graph_set_capture, or a NULL set. */
dg_status dg_set_set_capture(dg_set* s, uint32_t chunk_sweeps);
/* Rebuilds the set's worker blocks for `workers` sweep workgroups (0 = the
 * default, five per compute unit rounded down to a multiple of 8; at least one
 * per graph, the rest in proportion to each graph's cost), without
 * re-uploading.  Must not overlap a sweep call on the set. */
dg_status dg_set_repartition(dg_set* s, uint32_t workers, void* hip_stream);
/* Autotuner for a set (as dg_tune, for the whole set): every commit mode and
 * interval (sync, async, delayed d in {16, 64, 256, 1024, whole}) at every
 * partition (the current one and 2, 3, 5 and 8 workgroups per compute unit),
 * each run to convergence after a warm-up run, three times; the least median
 * time wins and the set keeps its partition.  The current partition with
 * delayed d = 64 is among the candidates and is reported as the default, so
 * the choice is never slower than it in the same measurement.
 *   algo     DG_ALGO_PAGERANK (damping 0.85, tol > 0 per graph, dtype; float32
 *            needs tol >= 1e-7) or DG_ALGO_SSSP (sources: one local source
 *            per graph, as dg_set_sssp)
 *   flags    0
 * Fills dg_tuning as dg_tune (predicted_seconds = seconds; from_cache = 0;
 * sweep_variant and resident_vertices are the union graph's own).  Not cached. */
dg_status dg_set_tune(dg_set* s, dg_algo algo, dg_dtype dtype, double tol, const uint32_t* sources, uint32_t flags,
                      dg_tuning* out, void* hip_stream);

/* PageRank of every graph of the set (as dg_pagerank, per graph).  All
 * graphs are swept together; each graph's dangling mass is spread over its
 * own vertices only, so a graph iterates as it would alone (synchronous
 * sweeps give each graph's own Jacobi iterates).  Every graph's own L1
 * change of normalised scores is measured each sweep, and the set stops at
 * the first sweep after which every graph has met tol (the single-graph
 * rule, graph by graph); graphs that met it earlier are no longer swept.
 *   flags       0 (reserved)
 *   dtype       DG_F32 only for tol >= 1e-7 (the float32 rounding floor) or
 *               tol = 0, else DG_ERR_UNSUPPORTED: use DG_F64
 *   out_scores  n float64 over the union (graph i's vertices at its offset,
 *               the sum of the n of graphs before it), each graph normalised
 *               to sum 1; device memory when out_on_device != 0
 *   out_sweeps  host array of `graphs` entries or NULL: for each graph the
 *               first sweep after which its change was below tol (0 = none
 *               within max_sweeps)
 *   stats       as dg_pagerank's on the union: sweeps, device seconds of the
 *               sweeps, edges_traversed = total edges x sweeps */
dg_status dg_set_pagerank(dg_set* s, double damping, double tol, dg_mode mode, uint32_t d, dg_dtype dtype,
                          uint32_t max_sweeps, uint32_t flags, double* out_scores, int out_on_device,
                          uint32_t* out_sweeps, dg_stats* stats, void* hip_stream);

/* Bellman-Ford of every graph from its own source (as dg_sssp, per graph).
 * All graphs are swept together; a graph whose sweep changed no distance is
 * final (no edge crosses two graphs) and is not swept again.
 *   sources     host array of `graphs` vertex ids, local to each graph
 *   flags       0 (reserved)
 *   out_dist    n uint32 over the union, DG_INF_DIST where unreachable
 *   out_sweeps  host array of `graphs` entries or NULL: for each graph the
 *               first sweep in which it changed no distance (0 = none within
 *               max_sweeps) */
dg_status dg_set_sssp(dg_set* s, const uint32_t* sources, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                      uint32_t flags, uint32_t* out_dist, int out_on_device, uint32_t* out_sweeps,
                      dg_stats* stats, void* hip_stream);

/* Serving loop (a form beyond the paper: many independent queries arriving
 * over time on resident graphs).  The server keeps a queue per (graph, query
 * kind) and pools of 64-lane batches swept by the batched kernels
 * (dg_sssp_batch / dg_ppr_batch semantics per lane).  Batching is
 * continuous: at every sweep boundary queued requests take free lanes of the
 * running batches (their lanes are initialised while the other lanes keep
 * their state), finished lanes hand over their rows and become free, and a
 * pool grows by one batch when it has no free lane and the state budget
 * allows.  A request's result is therefore the same as the batched call's for
 * its source: bit-identical for SSSP in every mode and, in synchronous mode,
 * for PPR as well.
 * The graphs must outlive the server; one server is driven by one thread. */
typedef struct dg_server dg_server;
typedef enum { DG_QUERY_SSSP = 0, DG_QUERY_PPR = 1 } dg_query;
typedef struct {
  uint64_t hbm_budget;   /* bytes of batch state over all pools; 0 = no limit */
  uint32_t max_batches;  /* batches per (graph, kind); 0 = no limit but the budget */
  dg_mode mode;          /* commit mode of every sweep */
  uint32_t d;            /* commit interval (delayed) */
  double damping;        /* PPR: 0 <= damping < 1 */
  double tol;            /* PPR: per-query stopping tolerance (L1 change), > 0 */
  dg_dtype dtype;        /* PPR storage */
} dg_server_opts;
typedef struct {
  uint32_t graph;
  dg_query kind;
  uint32_t source;
  uint32_t sweeps;       /* sweeps from admission to the stopping one */
  uint32_t state;        /* 0 queued, 1 running, 2 finished, 3 fetched */
  uint64_t submit_step, admit_step, finish_step;
} dg_request_info;
typedef struct {
  uint32_t queued, running, finished;  /* finished = results not yet fetched */
  uint32_t batches;
  uint64_t state_bytes;
  uint64_t steps;
} dg_server_status;
/* graphs: `count` resident graphs (not owned).  Work runs on hip_stream. */
dg_status dg_server_create(dg_graph* const* graphs, uint32_t count, const dg_server_opts* opts, void* hip_stream,
                           dg_server** out);
dg_status dg_server_destroy(dg_server* s);
/* Queues a query: SSSP from `source` (the graph needs weights) or PPR with
 * restart vertex `source`.  Ids start at 1. */
dg_status dg_server_submit(dg_server* s, uint32_t graph, dg_query kind, uint32_t source, uint64_t* out_id);
/* One step: admission, one sweep of every pool with running queries,
 * retirement.  Writes up to `cap` ids of requests finished so far and not yet
 * reported to out_finished (the rest are reported by later steps). */
dg_status dg_server_step(dg_server* s, uint64_t* out_finished, uint32_t cap, uint32_t* out_count);
/* Request status (info) and, when out != NULL, its result: n uint32
 * distances (SSSP) or n float64 scores summing to 1 (PPR), device memory
 * when out_on_device != 0.  Fetching releases the result. */
dg_status dg_server_fetch(dg_server* s, uint64_t id, void* out, int out_on_device, dg_request_info* info);
dg_status dg_server_status_get(const dg_server* s, dg_server_status* status);

/* Gather-rate probe (measurement support, not a sweep): the time of random
 * 4-byte loads from a table of table_bytes (a power of two in [4 KiB,
 * 4 GiB]), the access a single query's pull sweep makes once per in-edge
 * (section III-A: every in-neighbour's value is read from the global array).
 * workgroups x 256 threads each make per_thread (a multiple of 16, at most
 * 4096) loads, 16 in flight, at indices uniform over the table; streamed = 1
 * reads each index from a coalesced 4-byte index stream (as a sweep reads
 * its in-edge stream), streamed = 0 computes it.  The call allocates its
 * table and stream with hipMalloc, runs one warm-up launch, and returns the
 * best of three timed launches in *out_seconds (events on hip_stream).
 * Total loads per launch must stay below 2^32. */
dg_status dg_probe_gather(uint64_t table_bytes, int streamed, uint32_t per_thread, uint32_t workgroups,
                          double* out_seconds, void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dg_sssp on a resident
 * graph with no allocation of any kind during the call.  The sweeps' value
 * arrays, staging and per-sweep state live in one fixed device array of the
 * library, DG_NOALLOC_SCRATCH_BYTES (96 MiB) per GPU, held from the first
 * call on that GPU until the process ends.  Results, sweep counts and the
 * kernels are those of dg_sssp (bit-identical distances in every mode).
 *   mode        DG_SYNC, DG_ASYNC or DG_DELAYED (not DG_DELAYED_LOCAL)
 *   max_sweeps  1 <= max_sweeps <= 65535
 *   out_dist    as for dg_sssp (device or host memory)
 *   stats       as for dg_sssp, except that `seconds` is host wall time from
 *               the first sweep launch to the host seeing the stopping flag
 *               (the call uses no events)
 * Needs (n + K) x 4 bytes (twice in DG_SYNC), plus n x 4 for the delayed
 * modes' shadow staging when d is large, plus n x 4 for host output, plus
 * about 24 x max_sweeps + 24 x workers bytes, each part rounded up to 256:
 * a call that needs more returns DG_ERR_UNSUPPORTED and does nothing.  K is
 * dg_graph_info.hot_vertices.  Not for the union graph of a set
 * (DG_ERR_UNSUPPORTED).  Every call on a GPU uses that GPU's one array:
 * calls that overlap in time on the same GPU (from several threads, or on
 * several streams) race and give undefined results; serialise them. */
#define DG_NOALLOC_SCRATCH_BYTES 100663296u
dg_status dg_sssp_noalloc(dg_graph* g, uint32_t src, dg_mode mode, uint32_t d, uint32_t max_sweeps,
                          uint32_t* out_dist, int out_on_device, dg_stats* stats, void* hip_stream);

/* Static name of a status code. */
const char* dg_status_str(dg_status s);

/* Message describing the last error on the calling thread ("" if none). */
const char* dg_last_error(void);

/* Library version string. */
const char* dg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */

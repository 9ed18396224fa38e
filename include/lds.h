/*
 * liblds — MI355X (gfx950) library for the convex-programming locally
 * densest subgraph method of arXiv 2504.10937 (LDScvx / LTDScvx).
 *
 * C ABI: plain pointers and sizes, no C++ types, no exceptions.  Every call
 * returns an lds_status; on failure the outputs are left untouched and
 * lds_last_error() returns a message (thread-local).  Device work is issued
 * on the HIP stream passed as `hip_stream` (a hipStream_t, NULL = the legacy
 * default stream).
 *
 * Vertex ids are the caller's ids 0..n-1 (int32).  Inside the library
 * vertices are renumbered; every tie that the method breaks is broken on the
 * caller's ids (see lds_frank_wolfe).
 *
 * Modes: LDS_EDGE   = edge density |E|/|V| (Section 3, Eq. cp),
 *        LDS_TRIANGLE = triangle density |T|/|V| (Section 6, Eq. trcp),
 *        LDS_CLIQUE4 = 4-clique density |K4|/|V|, the h-clique program that
 *                      Eq. trcp generalises, with h = 4 (Frank-Wolfe only:
 *                      lds_frank_wolfe, lds_loads, lds_splits, lds_sweep_info,
 *                      lds_fw_elapsed, lds_cliques4; the other calls take
 *                      LDS_EDGE and LDS_TRIANGLE).
 *
 * Exact arithmetic.  Frank-Wolfe with step gamma_i = 2/(i+2) keeps every load
 * r_u^(i) and every split alpha^(i) on the common denominator
 * D_i = (i+1)(i+2) (edges), 3(i+1)(i+2) (triangles) or 2(i+1)(i+2)
 * (4-cliques); the library stores the
 * integer numerators, so every decision (argmin of r over a pattern) is
 * exact and results do not depend on launch configuration or batching.
 * Float views are produced on output only.
 */
#ifndef LDS_H
#define LDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lds_graph_s* lds_graph;

typedef enum { LDS_EDGE = 2, LDS_TRIANGLE = 3, LDS_CLIQUE4 = 4 } lds_mode;

typedef enum {
    LDS_OK = 0,
    LDS_E_INVALID = 1,  /* bad argument (ids out of range, n < 0, iters < 0, ...) */
    LDS_E_NOMEM = 2,    /* device or host allocation failed */
    LDS_E_DEVICE = 3,   /* HIP runtime error */
    LDS_E_OVERFLOW = 4, /* an exact numerator would exceed its width: 64-bit loads (see
                           lds_frank_wolfe) or 32-bit splits (D_iters > 2^32 - 1, see
                           lds_sort_prefix) */
    LDS_E_BUSY = 5      /* resource in use (server slots, budget) */
} lds_status;

/* Flags of lds_create_graph. */
#define LDS_INPUT_DEVICE 1u /* src/dst are device pointers (else host) */
#define LDS_STRICT 2u       /* self-loops and duplicate pairs are errors (else dropped) */

/* Thread-local message describing the last failing call ("" if none). */
const char* lds_last_error(void);

/* Optional device allocator used for all library-owned device memory
 * (e.g. PyTorch's caching allocator).  alloc(bytes, stream, ctx) returns a
 * device pointer or NULL; free(ptr, ctx) releases it.  Pass NULLs to return
 * to hipMalloc/hipFree.  Must be set before any graph is created. */
typedef void* (*lds_alloc_fn)(size_t bytes, void* hip_stream, void* ctx);
typedef void (*lds_free_fn)(void* ptr, void* ctx);
lds_status lds_set_allocator(lds_alloc_fn alloc, lds_free_fn free_fn, void* ctx);

/* Graph ingest (the undirected simple graph G=(V,E) of Section 3).
 * n: number of vertices (0 <= n < 2^31).  src/dst: npairs int32 endpoint
 * ids in [0,n), host or device memory (LDS_INPUT_DEVICE); the caller keeps
 * ownership and may free them on return.  Pairs are undirected; self-loops
 * and duplicates are dropped unless LDS_STRICT (then LDS_E_INVALID).  At
 * most 2^31 - 1 unique edges (LDS_E_OVERFLOW beyond: the symmetric CSR's
 * slots are sorted per row with 32-bit counts).
 * On success *out owns its device memory until lds_destroy_graph. */
lds_status lds_create_graph(int64_t n, int64_t npairs, const int32_t* src, const int32_t* dst, uint32_t flags,
                            void* hip_stream, lds_graph* out);
lds_status lds_destroy_graph(lds_graph g);

/* n, number of unique edges m, number of triangles (-1 until listed) and
 * the device bytes the graph currently holds.  Any output may be NULL. */
lds_status lds_graph_info(lds_graph g, int64_t* n, int64_t* m, int64_t* n_triangles, size_t* device_bytes);

/* Triangle listing: the set T of Eq. (trcp) / Alg. 6 (the paper uses T but
 * does not say how it is obtained).  Lists T on the device (once; cached in
 * the graph) and returns |T|.  If tri_out (host, 3*|T| int32) is non-NULL
 * and cap >= |T|, writes every triangle as ascending caller ids (a<b<c), in
 * lexicographic order.  If tcount_out (host, n int64) is non-NULL, writes
 * t_u per vertex. */
lds_status lds_triangles(lds_graph g, int64_t* n_triangles, int32_t* tri_out, int64_t cap, int64_t* tcount_out,
                         void* hip_stream);

/* 4-clique listing: the pattern set of the h-clique program (h = 4) that
 * Eq. (trcp) generalises.  Lists the 4-cliques on the device (once, after the
 * triangles; cached in the graph) and returns their number.  If q_out (host,
 * 4 int32 per clique) is non-NULL and cap >= the count, writes every clique
 * as ascending caller ids (a<b<c<d), in lexicographic order.  If qcount_out
 * (host, n int64) is non-NULL, writes the number of 4-cliques at each vertex.
 * LDS_E_OVERFLOW when the count reaches 2^31. */
lds_status lds_cliques4(lds_graph g, int64_t* n_cliques, int32_t* q_out, int64_t cap, int64_t* qcount_out,
                        void* hip_stream);

/* Frank-Wolfe on CP(G) (Alg. 1, edges), on the triangle program (Alg. 6) or
 * on the 4-clique program (the same iteration over 4-cliques), `iters` >= 0
 * iterations from the initial split alpha = 1/2 (resp. 1/3, 1/4).
 * Iteration i gives every pattern's unit weight to its vertex of smallest
 * r^(i-1) (synchronous: all decisions read r^(i-1)); exact ties go to the
 * larger caller id.  Then alpha <- (1-gamma) alpha + gamma alpha_hat with
 * gamma = 2/(i+2), and r = sum alpha, i.e. r <- (1-gamma) r + gamma b where
 * b_u counts the units u received.
 * Outputs (each optional, NULL to skip), all indexed by caller id:
 *   r_out    device float[n]: r_u^(iters) rounded to FP32 (from the exact
 *            rational, via FP64)
 *   r64_out  host double[n]: r_u^(iters) rounded to FP64
 *   num_out  host uint64[n]: exact numerator A_u with r_u = A_u / D_iters
 *   gap_out  host double[iters]: FW duality gap at r^(i-1), i = 1..iters,
 *            2 (sum_u r_u^2 - sum_patterns min_{u in p} r_u), evaluated
 *            from exact integer sums
 * The state (loads, splits) stays on the device for lds_loads, lds_splits,
 * lds_sort_prefix, lds_stable_groups and lds_topk.  Returns LDS_E_OVERFLOW if a numerator could exceed the
 * 64-bit packed key (max degree (resp. triangle or 4-clique count) times the
 * largest per-vertex increment). */
lds_status lds_frank_wolfe(lds_graph g, lds_mode mode, int32_t iters, float* r_out, double* r64_out,
                           uint64_t* num_out, double* gap_out, void* hip_stream);

/* lds_frank_wolfe without any device allocation, for callers that cannot
 * allocate (tight serving loops, code that must not call hipMalloc): the same
 * sweep kernel (hub rows pulled rather than pushed: the push's per-workgroup
 * counters do not fit the fixed scratch) and the same exact result (loads bit
 * for bit; gap within FP64 rounding, as it is formed on the device from the
 * same exact sums).
 * The graph's FW state for this mode must already be sized for `iters`
 * iterations by an earlier lds_frank_wolfe (or lds_batch_create) with at
 * least `iters` iterations, and triangles (4-cliques) must be listed;
 * otherwise LDS_E_INVALID and nothing runs.  Outputs (optional): r_out
 * device float[n] by caller id, gap_out host double[iters].  With gap_out
 * the per-workgroup partial sums live in a fixed 4 MiB device array per GPU
 * (held until the process ends): iters is limited to
 * 4 MiB / (8 * (4 * compute units + 5)) = 509 on a 256-CU MI355X, and to
 * 4 MiB / (8 * (8 * compute units + 5)) = 255 for an edge graph whose
 * two-dimensional heavy-row sweep is switched on (LDS_HEAVY_DEG; its
 * finishing kernel adds a workgroup per CU) (LDS_E_INVALID beyond, with the
 * limit in the message).  Every call on one GPU shares that array: calls
 * with gap_out that overlap in time on the same GPU race and must be
 * serialised by the caller.  Leaves the state as lds_frank_wolfe does,
 * except that lds_loads reports no gap afterwards; with gap_out the call
 * waits for the stream. */
lds_status lds_frank_wolfe_noalloc(lds_graph g, lds_mode mode, int32_t iters, float* r_out, double* gap_out,
                                   void* hip_stream);

/* Exact split numerators alpha_{x,p} * D of the last lds_frank_wolfe run
 * (Eq. cp / Eq. trcp variables).  One entry per incidence (vertex x,
 * pattern p): edges 2m entries, triangles 3|T|, 4-cliques 4|K4|.  verts_out (host
 * int32, h entries per incidence: x first, then the other vertices of p, as
 * caller ids) and num_out (host uint64 per incidence).  Entries appear in an
 * unspecified order.  cap = capacity in incidences. */
lds_status lds_splits(lds_graph g, lds_mode mode, int32_t* verts_out, uint64_t* num_out, int64_t cap,
                      int64_t* count_out, void* hip_stream);

/* Alg. 2, sort and prefix step, on the state of the last lds_frank_wolfe run of this
 * mode: sort of the vertices by r descending (ties: caller id ascending),
 * prefix pattern counts and the candidate set I.  Host outputs, each
 * optional: order_out[j] = caller id at 0-based position j (n entries);
 * E_out[j] = number of edges (triangles) induced by the first j+1 vertices;
 * inI_out[j] = 1 iff j+1 = argmax_{k >= j+1} E_{k-1}/k with ties to the larger
 * index, i.e. E_j/(j+1) exceeds every later E_k/(k+1).
 * The stable-group pass holds split numerators in 32 bits: LDS_E_OVERFLOW
 * when the last run's D_iters exceeds 2^32 - 1 (edges from iters = 65535,
 * triangles from iters = 37836); lds_stable_groups, lds_topk and
 * lds_server_submit check the same limit before any work. */
lds_status lds_sort_prefix(lds_graph g, lds_mode mode, int32_t* order_out, int64_t* E_out, uint8_t* inI_out,
                           void* hip_stream);

/* Alg. 2, stable-group scan: stable groups (Def. 5 for edges, Def. trsg for
 * triangles) from the candidates of lds_sort_prefix.  A candidate run is
 * merged with the next one until it is a stable group of the restricted
 * solution: every edge (triangle) touching the tested group gives its weight
 * only to its vertices in the lowest group it touches (accepted groups above,
 * the tested group, all vertices below), shares freed from higher vertices go
 * to the lowest-r vertex of that group; a group is accepted iff its
 * restricted loads are strictly below every accepted vertex and strictly
 * above every vertex below.  Outputs (host): *ngroups; gstart/gend (cap
 * entries): 0-based position range [start, end) of each group, top first;
 * lo_out/hi_out (n entries, by caller id): restricted min / max numerator of
 * the vertex's group (bounds of Lemma phi-bounds, over D_iters), -1 for
 * vertices of the unaccepted tail.  Any output may be NULL. */
lds_status lds_stable_groups(lds_graph g, lds_mode mode, int64_t* ngroups, int64_t* gstart, int64_t* gend, int64_t cap,
                             int64_t* lo_out, int64_t* hi_out, void* hip_stream);

/* Profile of the last stable-group scan of this graph and mode (host int64
 * out[14]): [0] accepted groups, [1] rounds (one per accepted group, plus
 * the last unfinished one), [2] verified boundaries, [3..6] phases of each
 * kind run by the whole grid (search, update walk, min / max, acceptance;
 * the rest ran in the leading workgroup alone), [7..10] wall-clock
 * microseconds spent in each kind, [11] positions searched, [12] records
 * walked, [13] workgroups of the launch.  LDS_E_INVALID if no scan has run. */
lds_status lds_sg_scan_info(lds_graph g, lds_mode mode, int64_t* out);

/* GPU time of the sweep launches of the last lds_frank_wolfe call for this
 * graph and mode, from HIP events recorded on that call's stream right before
 * the first and after the last sweep launch (waits for the end event).
 * *launches = number of sweep launches (= iters when the graph has
 * patterns).  Any output may be NULL. */
lds_status lds_fw_elapsed(lds_graph g, lds_mode mode, float* ms, int32_t* launches);

/* Shape of the sweep over incidence slots (Alg. 1 / Alg. 6 pull form):
 * rows (vertices with >= 1 incidence), slots (2m or 3|T|), hub rows (one
 * workgroup each), row-aligned chunks (one wave64 each) and decision words
 * per iteration (64 slots per word, word-aligned per chunk / hub row).
 * For LDS_TRIANGLE the triangles are listed first if needed. */
lds_status lds_sweep_info(lds_graph g, lds_mode mode, int64_t* rows, int64_t* slots, int64_t* hub_rows,
                          int64_t* chunks, int64_t* words, void* hip_stream);

/* Denominator D_iters of the loads after `iters` iterations. */
uint64_t lds_denominator(lds_mode mode, int32_t iters);

/* Current Frank-Wolfe state of a mode without running anything: the loads
 * left by the last lds_frank_wolfe or lds_batch_run of this graph and mode.
 * r_out (device float, n, by caller id), r64_out (host double), num_out
 * (host uint64 numerators over lds_denominator(mode, iters)), gap_out (host,
 * iters entries; only after a run that computed the gap); *iters_out = the
 * iteration count of that run.  Any output may be NULL.  LDS_E_INVALID if no
 * run has been made for the mode. */
lds_status lds_loads(lds_graph g, lds_mode mode, float* r_out, double* r64_out, uint64_t* num_out, double* gap_out,
                     int32_t* iters_out, void* hip_stream);

/* Certified bounds of the last lds_frank_wolfe run that computed the gap,
 * per iteration i = 1..iters (host arrays of iters entries, each optional):
 *   lb_out[i-1]       LB_i = 2 sum_patterns min_u r_u - sum_u r_u^2 at
 *                     r^(i-1), a lower bound on the optimum f* of Eq. cp /
 *                     Eq. trcp (f = sum r^2 minus its linear gap);
 *   cert_gap_out[i-1] Gamma_i = min_{j<=i} f_j - max_{j<=i} LB_j with
 *                     f_j = sum r^2 at r^(j-1): the certified gap, >= 0
 *                     and non-increasing in i.
 * Both follow from the exact integer sums of the sweep (rounded once to
 * FP64).  LDS_E_INVALID when the last run did not compute the gap. */
lds_status lds_fw_bounds(lds_graph g, lds_mode mode, double* lb_out, double* cert_gap_out);

/* Measurement: the achievable device-memory bandwidth that the roofline of
 * the sweep is read against.  Copies `bytes` (a positive multiple of 16)
 * from src to dst (device pointers, 16-byte aligned, not overlapping) with a
 * grid-strided 16-byte streaming copy kernel, once untimed and then `reps`
 * times on hip_stream; *ms_out = mean GPU milliseconds of one copy (HIP
 * events; 2 * bytes cross HBM per copy).  Waits for the stream. */
lds_status lds_copy_bandwidth(void* dst, const void* src, size_t bytes, int32_t reps, void* hip_stream,
                              float* ms_out);

/* Measurement: the rate of random 2-byte gathers, the access the Frank-Wolfe
 * sweep makes for every incidence whose other vertex is outside its LDS
 * cache of codes.  Reads n int32 indices idx (device; each in [0, entries),
 * which the caller guarantees: they are not checked) and the uint16 table
 * entries they name (device, `entries` of them), eight per thread in flight,
 * once untimed and then `reps` times on hip_stream; sink (device uint32,
 * 8 * 256 * compute units entries) receives per-thread sums.  *ms_out = mean
 * GPU milliseconds of one pass over the n indices.  Waits for the stream. */
lds_status lds_gather_rate(const int32_t* idx, int64_t n, const uint16_t* table, int64_t entries, uint32_t* sink,
                           int32_t reps, void* hip_stream, float* ms_out);

/* ---- Batched Frank-Wolfe over many independent graphs ----------------------
 * A batch runs lds_frank_wolfe(graphs[i], modes[i], iters[i]) for every i in
 * one persistent kernel launch, captured into a hipGraph at creation and
 * replayed by lds_batch_run.  Each workgroup takes whole graphs from a device
 * work queue (largest first) and runs all their iterations with workgroup
 * barriers, keys in LDS for graphs with at most lds_vertices vertices.
 * Graphs whose work (incidences + vertices) * iters exceeds max_kernel_cost
 * run one by one (lds_frank_wolfe's own launches) on the same stream.  The
 * arithmetic is exact, so after lds_batch_run every graph holds bit for bit
 * the state that lds_frank_wolfe leaves (loads, splits, gap); lds_loads,
 * lds_splits, lds_stable_groups and lds_topk read it. */
typedef struct lds_batch_s* lds_batch;

/* Launch shape of the batched kernel (lds_tune_default, lds_batch_autotune). */
typedef struct {
    int32_t threads;          /* workgroup size: 256, 512 or 1024 */
    int32_t wg_per_cu;        /* persistent workgroups per compute unit, 1..8 */
    int32_t lds_vertices;     /* graphs with at most this many vertices keep keys in LDS, 0..8192 */
    int32_t longest_first;    /* 1: queue ordered by work, largest first */
    int64_t max_kernel_cost;  /* larger graphs run one by one */
} lds_tune;

#define LDS_BATCH_GAP 1u /* compute the duality gap of every graph (lds_loads gap_out) */

void lds_tune_default(lds_tune* out);

/* graphs, modes, iters: count entries; a (graph, mode) pair may appear once.
 * r_out: NULL or count device pointers (each NULL or n floats, by caller
 * id) that receive the final loads at every run.  tune: NULL = defaults.
 * The graphs must outlive the batch and must not be used by other calls
 * while lds_batch_run executes.  Lists triangles and sizes every graph's FW
 * buffers; synchronises hip_stream. */
lds_status lds_batch_create(const lds_graph* graphs, const lds_mode* modes, const int32_t* iters, float* const* r_out,
                            int32_t count, uint32_t flags, const lds_tune* tune, void* hip_stream, lds_batch* out);
/* One run of the whole batch on hip_stream (asynchronous unless
 * LDS_BATCH_GAP, which waits for the gap sums). */
lds_status lds_batch_run(lds_batch b, void* hip_stream);
/* kernel_graphs / plain_graphs: graphs in the batched kernel / run one by
 * one; kernel_ms: GPU time of the captured launch of the last run (waits for
 * it); tune: the launch shape.  Any output may be NULL. */
lds_status lds_batch_info(lds_batch b, int32_t* kernel_graphs, int32_t* plain_graphs, float* kernel_ms,
                          lds_tune* tune);
lds_status lds_batch_destroy(lds_batch b);

/* Autotuner: times the candidate launch shapes (workgroup size x workgroups
 * per CU x the LDS-resident vertex threshold lds_vertices in {8192, 4096,
 * 2048, 0}, where the workgroups' key buffers fit a CU's LDS together; then
 * queue order; then the per-graph work cutoff) on this batch, `reps` timed
 * runs each after one warm-up, and returns the fastest in *best.  With cache_path, a JSON file
 * keyed by a coarse signature of the batch (graph count, total work, largest
 * graph, edge / triangle mix, CU count, each rounded to a power of two) is
 * read first (no timing when the signature is present, *best_ms = -1) and
 * updated after timing.  Runs the batch, so it overwrites the graphs' FW
 * state like lds_batch_run. */
lds_status lds_batch_autotune(const lds_graph* graphs, const lds_mode* modes, const int32_t* iters, int32_t count,
                              const char* cache_path, int32_t reps, lds_tune* best, double* best_ms,
                              void* hip_stream);

/* Core numbers that bound the compact numbers (Section 4.3): LDS_EDGE gives
 * the k-core number of every vertex (the largest k such that the vertex lies
 * in a subgraph whose vertices all have degree >= k in it), LDS_TRIANGLE the
 * tr-core number (the same with triangles of the subgraph at each vertex);
 * core / 2 <= phi <= core for edges, tr-core / 3 <= phi <= tr-core for
 * triangles.  alive: NULL for the whole graph, else n host bytes by caller
 * id: the numbers of the subgraph induced by the vertices with alive != 0
 * (the residual graph of Pruning rule 2, Alg. 3), -1 for the other vertices.
 * core_out: host int64, n entries by caller id.  Runs level-synchronous
 * peeling on the device on hip_stream and synchronises it; lists the
 * triangles first if needed (LDS_TRIANGLE). */
lds_status lds_core_numbers(lds_graph g, lds_mode mode, const uint8_t* alive, int64_t* core_out, void* hip_stream);

/* Result of lds_topk, allocated by the library; release with
 * lds_result_free.  Set i (0 <= i < count) has the caller ids
 * vertices[offsets[i] .. offsets[i+1]) in ascending order and the exact
 * density dens_num[i] / dens_den[i] (reduced fraction: edges (triangles) of
 * the induced subgraph over its vertex count).  Sets are ordered by density
 * descending, ties by smallest caller id ascending.  The stats fields report
 * the work of the search: candidates taken, FW + ExtractSG runs on induced
 * subgraphs, candidates split by a min cut, min-cut computations and
 * vertices removed by the pruning rules; the ms fields the wall-clock time of
 * the phases (host copy of the graph, core numbers, first FW + ExtractSG,
 * pruning, candidate search); refine_rounds the batched FW launches that
 * carried the refinements (candidates that fail IsDensest with the same
 * bound are refined together). */
typedef struct {
    int32_t count;
    int64_t* offsets;   /* count + 1 */
    int32_t* vertices;  /* offsets[count] */
    int64_t* dens_num;  /* count */
    int64_t* dens_den;  /* count */
    int64_t popped, refinements, flow_splits, maxflows, pruned;
    double ms_copy, ms_core, ms_fw, ms_prune, ms_search;  /* wall-clock phases */
    int64_t refine_rounds;
} lds_result;

/* Top-k LDS (Problem LDS, Section 3; mode LDS_EDGE) or LTDS (Problem LTDS,
 * Section 6; mode LDS_TRIANGLE) by the LDScvx search (Alg. 5): iters FW
 * iterations (Alg. 1 / Alg. 6) and ExtractSG (Alg. 2) on the graph give
 * bounds on every compact number, together with core (tr-core) numbers;
 * Pruning (Alg. 3) removes vertices outside every LDS; candidates are
 * verified exactly by IsDensest (one min cut) and IsLDS (Alg. 4) / IsLTDS
 * (Alg. 7 with ExtMaximal, Alg. 8); a candidate that fails IsDensest is split
 * by FW + ExtractSG on its induced subgraph (or by the min cut when that does
 * not split it).  Returns the k densest LDSs (fewer when the graph has fewer
 * with positive density).  Synchronises the stream: verification runs on the
 * host, except the min cuts of vertex networks (LDS_EDGE) with at least
 * 131072 nodes, which run as a push-relabel on the device, on hip_stream
 * (environment: LDS_FLOW_GPU_MIN sets the node count, LDS_FLOW_GPU_WG the
 * grid width).  Smaller ones run on the host: from 524288 nodes (when the
 * device threshold is raised) a parallel push-relabel on up to 16 host
 * threads (LDS_FLOW_THREADS sets the thread count, 1 = sequential;
 * LDS_FLOW_PARALLEL_MIN the node count).  Pattern networks (LDS_TRIANGLE)
 * use the sequential host push-relabel.
 * Replaces the graph's FW state of this mode with an iters-iteration
 * run.  *out is overwritten; on error it is left zeroed.  LDS_E_INVALID for
 * k < 1, iters < 0 or a bad mode; LDS_E_OVERFLOW when D_iters exceeds
 * 2^32 - 1 (see lds_sort_prefix), before any work. */
lds_status lds_topk(lds_graph g, lds_mode mode, int32_t k, int32_t iters, lds_result* out, void* hip_stream);

/* Pruning (Alg. 3, Section 5.2) as lds_topk runs it, without the search:
 * iters FW iterations and ExtractSG on the graph give bounds on every compact
 * number (with the core / tr-core bounds of Section 4.3); rule 1 (Cor.
 * uv-prune) removes every vertex with a neighbour whose lower bound exceeds
 * its upper bound, then rule 2 (Lemma uu-prune) removes, until nothing
 * changes, every vertex whose core (tr-core) number in the graph of the
 * remaining vertices is below its lower bound.  No removed vertex lies in an
 * LDS (LTDS).  Both rules run on the device.  Outputs (each optional):
 * rule_out (host int8, n, by caller id) = the rule that removed the vertex
 * (1 or 2), 0 for the survivors; *pruned_out = removed vertices; *ms_out =
 * wall-clock ms of the pruning itself.  Replaces the graph's FW state of this
 * mode with an iters-iteration run; synchronises the stream. */
lds_status lds_prune(lds_graph g, lds_mode mode, int32_t iters, int8_t* rule_out, int64_t* pruned_out,
                     double* ms_out, void* hip_stream);

/* Frees the arrays of a result filled by lds_topk and zeroes it; NULL and
 * zeroed results are accepted. */
void lds_result_free(lds_result* r);

/* ---- Serving: continuous batching of top-k queries on resident graphs -----
 * Queries (graph, mode, k, iters) are queued with their arrival time.  A
 * scheduler thread admits queued queries in arrival order while the device
 * memory they add (lds_footprint) fits the budget and a slot is free.  Each
 * admitted query works on its own view of its graph (the graph's device data
 * shared, its own FW and stable-group state), so queries on one (graph,
 * mode) run at once.  The queries admitted together whose FW cost ((pattern
 * incidences + vertices) x iters) is at most 2^22 run their Frank-Wolfe
 * iterations in one batched launch (as lds_batch_run); larger ones run FW on
 * their worker's stream (the environment variable LDS_SERVE_KERNEL_COST,
 * read at lds_server_create, changes the cutoff).  Worker threads finish
 * each query (lds_topk's search, on their own streams), taking the oldest
 * query whose batched FW has finished, while the scheduler already admits
 * and launches the next batch.  Each query starts from the canonical initial
 * point, so its result equals lds_topk(g, mode, k, iters) run alone.  Graphs
 * must stay alive until their queries complete; while the server runs, the
 * caller's own calls on a graph wait for the server's use of it. */
typedef struct lds_server_s* lds_server;

typedef struct {
    uint64_t tag;
    int32_t status;        /* lds_status of the query */
    lds_result result;     /* valid when status == LDS_OK; free with lds_result_free */
    double t_arrive;       /* seconds on the server clock (lds_server_clock) */
    double t_admit;        /* when the query was admitted (-1 if never) */
    double t_done;
    char error[160];       /* message when status != LDS_OK */
} lds_completion;

typedef struct {
    int64_t submitted, completed, batches, max_batch, pending, active;
    size_t inflight_bytes, peak_inflight_bytes;
    double batch_ms;  /* wall time spent in batched FW launches */
} lds_server_info;

/* Device bytes one query adds to its resident graph (FW state for `iters`
 * iterations, stable-group buffers, temporaries): an upper estimate, used
 * for admission.  LDS_TRIANGLE needs the triangles listed (lds_triangles). */
lds_status lds_footprint(lds_graph g, lds_mode mode, int32_t iters, size_t* bytes);

/* hbm_budget: device bytes that admitted queries may add together (0 = 90%
 * of the device memory free now); max_slots: queries admitted at once;
 * workers: verification threads (1..64).  A query whose footprint exceeds
 * the budget completes with LDS_E_NOMEM.  The server runs 5 + workers
 * streams; the HIP runtime maps a process's streams onto GPU_MAX_HW_QUEUES
 * hardware queues (4 unless set before the runtime starts), and with more
 * queues (e.g. 16) the workers' small kernels stop waiting behind each
 * other. */
lds_status lds_server_create(size_t hbm_budget, int32_t max_slots, int32_t workers, lds_server* out);
/* t_arrive < 0: now.  For a triangle query on a graph whose triangles are
 * not listed yet, lists them first (the call waits for it). */
lds_status lds_server_submit(lds_server s, lds_graph g, lds_mode mode, int32_t k, int32_t iters, uint64_t tag,
                             double t_arrive);
/* Up to max completions into out (waits up to wait_s seconds for the first
 * one when none is ready); *n_out = number written. */
lds_status lds_server_poll(lds_server s, lds_completion* out, int32_t max, double wait_s, int32_t* n_out);
lds_status lds_server_clock(lds_server s, double* now);
lds_status lds_server_stats(lds_server s, lds_server_info* out);
/* Drops queued queries that were not admitted, waits for the admitted ones
 * and stops the threads; completions not yet polled are discarded. */
lds_status lds_server_destroy(lds_server s);

#ifdef __cplusplus
}
#endif
#endif /* LDS_H */

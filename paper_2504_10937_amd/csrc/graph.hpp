// Internal graph and Frank-Wolfe state of the LDS / LTDS library.
//
// Vertex numbering.  Callers use their own ("original") ids 0..n-1.  Inside
// the library vertices are renumbered by degree, descending, ties by
// original id ascending, so that vertices with the most incident slots come
// first (high-degree rows become the "hub" prefix processed one workgroup
// per row) and isolated vertices come last.  Every decision that the method
// takes on ties uses the ORIGINAL id, never the internal one.
//
// Incidence CSR.  The Frank-Wolfe sweep is a pull over "slots": for edges
// (h = 2) every vertex u has one slot per incident edge holding the other
// endpoint; for triangles (h = 3) one slot per incident triangle holding the
// other two vertices.  Rows are "compact": only vertices with at least one
// slot, ordered by slot count (descending), mapped to internal ids by rowid.
//
// Sweep plan.  Rows with more than kChunk slots are hubs, one workgroup
// each.  The remaining rows are cut into chunks: chunk c holds the rows whose
// first slot lies in [c*kChunk, (c+1)*kChunk) (relative to the first
// non-hub slot), so a chunk spans fewer than 2*kChunk slots and always
// starts at a row start.  Each chunk is one wave64.  The decision bits of one
// iteration are stored per chunk from a 64-bit-word-aligned offset (cwo),
// followed by the hub rows (hwo); a per-chunk "head" bitmap marks row starts.
#pragma once
#include <memory>

#include "common.hpp"

namespace lds {

constexpr int kChunk = 1024;  // target slots per wave; spans < 2*kChunk = 32 words
constexpr int kPiece = 2048;  // slots of a hub-row piece (a multiple of 64)
// LDS bytes of the persistent edge sweep for the staged codes and, with the
// hub push, the per-workgroup win counters of the hub rows
constexpr int64_t kSweepLds = 155648;
constexpr int kHeavyRows = 8192;   // rows of a block of the 2D part (at most 2^16)
constexpr int kHeavySlab = 24576;  // neighbour ids of a slab of the 2D part (at most 2^16)

// denominator of the loads after i iterations with gamma_i = 2/(i+2):
// (i+1)(i+2) for edges (mode 2), 3(i+1)(i+2) for triangles (mode 3),
// 2(i+1)(i+2) for 4-cliques (mode 4); D_0 / h is an integer in each case
inline uint64_t fw_denom(int mode, int64_t i) {
    const uint64_t c = mode == 3 ? 3 : (mode == 4 ? 2 : 1);
    return c * (uint64_t)(i + 1) * (uint64_t)(i + 2);
}

// The split numerator of an incidence never exceeds D_N (it is at most D_N
// minus the other members' initial shares), and the stable-group pass, the
// split gathers and the warm-started min cuts hold it in 32 bits.  Raises
// ST_OVERFLOW when D_iters does not fit, before any work is done: edges from
// N = 65,535 on, triangles from N = 37,836 on.
inline void check_split_width(int mode, int64_t iters) {
    if (iters >= 0 && (uint64_t)(iters + 1) * (uint64_t)(iters + 2) * (mode == 3 ? 3u : (mode == 4 ? 2u : 1u)) >
                          (uint64_t)UINT32_MAX)
        throw Error(ST_OVERFLOW, "split numerators of this many iterations exceed 32 bits (D_N > 2^32 - 1)");
}

// index of a mode's Frank-Wolfe / stable-group state: edges 0, triangles 1, 4-cliques 2
inline int mode_slot(int mode) { return mode - 2; }

// Heavy rows of a large edge plan, swept in two dimensions.  The rows of
// degree >= a threshold (a prefix of the degree-ordered ids) are cut into
// blocks of at most R rows and their neighbours into slabs of C consecutive
// ids.  Segment (b, j) lists the slots of block b whose neighbour lies in slab
// j, by (row, neighbour), each as ((row - first row of b) | run head << 15)
// << 16 | (neighbour - first id of j), where the run head bit marks a row's
// first slot in the segment, padded to whole 64-slot words.  Blocks hold at
// most R rows and, where rows are long, fewer (a cap on their slots).  A part is a range of slabs
// of one block; a workgroup sweeping a part keeps the block's codes and win
// counts and one slab of codes at a time in LDS, so every code it compares
// comes from LDS.  The parts of a block leave partial win counts, which a
// second kernel sums per row.
struct HeavyPlan {
    int64_t n_heavy = 0;          // rows [0, n_heavy) (0: no 2D part)
    int R = 0, C = 0;             // most rows of a block (stride of the per-block arrays), ids per slab
    int64_t P = 0;                // slabs: ceil(n / C)
    int64_t n_blocks = 0, n_parts = 0;
    int64_t positions = 0;        // padded slots of all segments (multiple of 64)
    int64_t word0 = 0;            // first decision word of the heavy region in an iteration's words
    DBuf<int64_t> seg;            // n_blocks * P + 1 first positions
    DBuf<uint32_t> pay;           // positions: packed (row, neighbour), 0xffffffff for padding
    DBuf<uint32_t> csr;           // positions: CSR slot, 0xffffffff for padding
    DBuf<int32_t> part_blk, part_j0, part_j1;  // per part: block and slab range [j0, j1)
    DBuf<int64_t> part_lo, part_hi;            // per part: its positions [lo, hi), within the block's
    DBuf<int32_t> blk_part;       // n_blocks + 1: first part of each block
    DBuf<int64_t> blk_row;        // n_blocks + 1: first row of each block
    DBuf<int32_t> row_blk;        // n_heavy: block of each heavy row
    DBuf<uint32_t> part_cnt;      // n_parts * R partial win counts (rewritten every sweep)
    size_t device_bytes() const {
        return seg.bytes() + pay.bytes() + csr.bytes() + part_blk.bytes() + part_j0.bytes() + part_j1.bytes() +
               part_lo.bytes() + part_hi.bytes() + blk_part.bytes() + blk_row.bytes() + row_blk.bytes() +
               part_cnt.bytes();
    }
};

struct SweepPlan {
    int h = 2;                  // pattern arity: 2 edges, 3 triangles
    int64_t nrows = 0;          // compact rows
    int64_t nslots = 0;
    const int32_t* rid = nullptr;  // compact row -> internal vertex (nullptr: identity)
    const int64_t* rp = nullptr;   // nrows + 1 slot offsets
    const int32_t* py = nullptr;   // nslots * (h - 1) vertex ids (internal)
    DBuf<int32_t> own_rid;         // storage when the plan owns rid / rp / py
    DBuf<int64_t> own_rp;
    DBuf<int32_t> own_py;
    DBuf<int32_t> own_tos;         // triangles: slot -> triangle index
    DBuf<int32_t> own_row_of;      // triangles: internal vertex -> compact row, -1 if none
    int64_t n_big = 0;             // rows [0, n_big) have >= 64 slots (rows are ordered by slot count)
    int64_t n_hub = 0;          // rows [0, n_hub) are hubs
    DBuf<int64_t> hwo;          // n_hub + 1 word offsets (relative to hub region)
    int64_t n_pieces = 0;       // hub rows cut into word-aligned pieces of <= kPiece slots, one wave each
    DBuf<int32_t> hp_row;       // per piece: hub row
    DBuf<int32_t> hp_off;       // per piece: first slot, relative to the row start (a multiple of 64)
    DBuf<unsigned long long> hub_ctr;  // n_hub: (pieces done << 40) | wins so far (zero between sweeps)
    // Hub push (edge plans in internal order, n_push = n_hub > 0, else 0): a
    // hub row compares itself only with the other hub rows (its first
    // hub_pre[r] slots; rows are sorted by neighbour id), and every other row
    // adds a hub's wins against it to the hub's counter in LDS (push_nc codes
    // are staged beside those counters).  The hub rows' other slots get no
    // decision bits; their splits follow from the mirror slots.
    int64_t n_push = 0;
    int64_t push_nc = 0;
    DBuf<int32_t> hub_pre;      // n_push: slots of hub row r whose neighbour is a hub row
    int64_t n_ppieces = 0;      // pieces of those prefixes (as hp_row / hp_off)
    DBuf<int32_t> pp_row;
    DBuf<int32_t> pp_off;
    int64_t n_chunks = 0;
    DBuf<int64_t> chunk_row;    // n_chunks + 1 (compact row index)
    DBuf<int64_t> cwo;          // n_chunks + 1 word offsets
    DBuf<uint64_t> head;        // chunk_words words: row-start flags
    int64_t chunk_words = 0, hub_words = 0, total_words = 0;
    DBuf<int64_t> bitbase;      // per compact row: bit index of its first slot (-1: heavy row)
    HeavyPlan heavy;            // edge plans of large graphs only
    size_t device_bytes() const {
        return own_rid.bytes() + own_rp.bytes() + own_py.bytes() + own_tos.bytes() + own_row_of.bytes() + hwo.bytes() + chunk_row.bytes() + cwo.bytes() +
               head.bytes() + bitbase.bytes() + hp_row.bytes() + hp_off.bytes() + hub_ctr.bytes() + hub_pre.bytes() +
               pp_row.bytes() + pp_off.bytes() + heavy.device_bytes();
    }
};

struct FwState {
    int iters = 0;               // iterations run
    int cur = 0;                 // keys live in K[cur]
    DBuf<uint64_t> K[2];         // packed keys (A << B) | (idmask - orig_id), internal order
    DBuf<uint16_t> Q[2];         // 16-bit monotone codes of A (gathered first)
    DBuf<uint64_t> bits;         // iters * total_words decision words
    DBuf<uint64_t> partial;      // iters * blocks * 4 gap partial sums
    DBuf<uint32_t> push_part;    // hub push: per sweep workgroup, the hub rows' win counts (two 16-bit halves a word)
    std::vector<double> gap, lb, fval;  // per iteration, filled on request: gap, lower bound, sum r^2 at r^(i-1)
    hipEvent_t ev[2] = {nullptr, nullptr};  // around the sweep launches of the last run
    int launches = 0;
    bool ran = false;            // keys hold the result of a completed run of `iters` iterations
    bool timed = false;          // ev[] bracket the last run (plain runs only)
    size_t device_bytes() const {
        return K[0].bytes() + K[1].bytes() + Q[0].bytes() + Q[1].bytes() + bits.bytes() + partial.bytes() +
               push_part.bytes();
    }
};

// Sort, prefix counts and stable groups (Alg. 2) of the last FW run of a mode
struct SgState {
    bool valid = false;
    int iters = -1;
    DBuf<int32_t> order;         // position -> internal vertex (r descending, caller id ascending)
    DBuf<int64_t> pos;           // internal vertex -> position
    DBuf<int64_t> E;             // patterns inside the first j+1 positions
    DBuf<uint8_t> inI;           // position j+1 (1-based) is a strict suffix maximum of E/j
    DBuf<uint32_t> a_slot;       // split numerator of every incidence slot
    DBuf<uint32_t> a_tri;        // triangles: the three split numerators per triangle
    // compact per-slot records in position order (the records of the vertex
    // at position j are [rec_P[j], rec_P[j+1])): the position of the slot's
    // own vertex, the positions of the pattern's other vertices and the
    // split numerators.  Built by the sort / prefix pass, which counts from
    // them, read by the stable-group scan and released after it.
    DBuf<int64_t> rec_P;         // n + 1
    DBuf<int32_t> rec_own;
    DBuf<int2> rec2;             // edges: (position of the other end, a_x)
    DBuf<int4> rec3;             // triangles: (position v, position w, a_x, a_v)
    DBuf<uint32_t> rec3w;        // triangles: a_w
    DBuf<int64_t> R, T;          // built with the records: by position, the restricted load when every earlier
                                 // vertex is above (R) and when S = [0, j] (T, which the scan then changes)
    std::vector<int64_t> gstart, gend;  // accepted groups (position ranges)
    DBuf<int64_t> lo, hi;        // per internal vertex: restricted min / max of its group, -1 if none
    int64_t rounds = 0, verifications = 0;
    // last scan's phase profile: grid-wide phases of each kind (search,
    // update walk, min / max, acceptance), microseconds in each kind,
    // positions searched, records walked
    int64_t scan_profile[10] = {};
    int64_t scan_wg = 0;  // workgroups of the last scan launch (0: none yet)
    size_t device_bytes() const {
        return order.bytes() + pos.bytes() + E.bytes() + inI.bytes() + a_slot.bytes() + a_tri.bytes() + lo.bytes() +
               hi.bytes() + rec_P.bytes() + rec_own.bytes() + rec2.bytes() + rec3.bytes() + rec3w.bytes() + R.bytes() +
               T.bytes();
    }
};

struct HostCache;  // host-side resident data of the top-k search (topk.hpp)

struct Graph {
    int64_t n = 0, m = 0;        // vertices, unique undirected edges
    int64_t n_nz = 0;            // vertices with degree > 0 (internal ids [0, n_nz))
    int idbits = 1;              // B: bits of the packed original-id code
    int vbits = 1;               // bits to hold values 0..n
    int32_t max_deg = 0;
    DBuf<int32_t> orig_of;       // internal -> original id
    DBuf<int32_t> int_of;        // original -> internal id
    DBuf<int32_t> deg;           // internal order
    DBuf<int64_t> rowptr;        // symmetric CSR, internal ids, n + 1
    DBuf<int32_t> col;           // 2m; ascending per row once col_sorted
    bool col_sorted = false;
    SweepPlan edge_plan;         // slots = CSR (rowid identity over [0, n_nz))
    // triangles (built on first use)
    int64_t T = -1;
    DBuf<int32_t> tri;           // 3T internal ids, per triangle (a > b > c internal)
    DBuf<int32_t> tcount;        // per internal vertex
    int64_t t_max = 0;
    SweepPlan tri_plan;
    // 4-cliques (built on first use)
    int64_t Q4 = -1;
    DBuf<int32_t> q4;            // 4 Q4 internal ids, per clique (a > b > c > d internal)
    DBuf<int32_t> qcount;        // per internal vertex
    int64_t q_max = 0;
    SweepPlan clique_plan;
    FwState fw[3];               // indexed by mode_slot: edges, triangles, 4-cliques
    SgState sg[3];               // sort / prefix / stable groups of the last run per mode (edges, triangles)
    std::shared_ptr<HostCache> host;  // host copy of the adjacency, triangles and core numbers, built on first use
    Graph* origin = nullptr;     // a per-query view: the resident graph whose device data it borrows
    hipStream_t stream = nullptr;
    size_t device_bytes() const;
    ~Graph();
};

// ingest.hip
void build_graph(Graph& g, int64_t n, int64_t npairs, const int32_t* src, const int32_t* dst, bool on_device,
                 bool strict, hipStream_t s);
void build_sweep_plan(SweepPlan& p, hipStream_t s, int64_t n_vertices = 0);  // needs h, nrows, nslots, rowptr, pay, rowid;
                                                                             // n_vertices > 0 allows the 2D heavy part (edges)
void sort_rows(Graph& g, hipStream_t s);             // CSR rows ascending (triangle listing)
// A per-query view of a resident graph: borrows every device array of g and
// its sweep plans, with its own Frank-Wolfe and stable-group state and its
// own sweep counters (zeroed on s), so that queries on one graph run at once.
// g must outlive the view and must not be changed while it exists.
std::unique_ptr<Graph> graph_view(Graph& g, hipStream_t s);

// triangles.hip
void list_triangles(Graph& g, hipStream_t s);
void list_cliques4(Graph& g, hipStream_t s);  // lists triangles first if needed
// per-vertex incident triangles (ascending), into host memory: trp (n + 1), tinc (3T)
void vertex_triangle_lists(const Graph& g, int64_t* trp_host, int32_t* tinc_host, hipStream_t s);

inline SweepPlan& plan_of(Graph& g, int mode) {
    return mode == 2 ? g.edge_plan : (mode == 3 ? g.tri_plan : g.clique_plan);
}
inline const SweepPlan& plan_of(const Graph& g, int mode) {
    return mode == 2 ? g.edge_plan : (mode == 3 ? g.tri_plan : g.clique_plan);
}

// sg.hip
void sg_sort_prefix(Graph& g, int mode, hipStream_t s);
void sg_stable_groups(Graph& g, int mode, hipStream_t s);
// lo / hi of the last stable-group scan, by original id, into host memory
void sg_copy_bounds(const Graph& g, int mode, int64_t* lo_out, int64_t* hi_out, hipStream_t s);
// out[i] = the FW split numerator at idx[i] (edges: CSR slot; triangles:
// 3 * triangle + member) of the graph's last stable-group run, for host idx /
// out of n elements; raises on an index out of range
void gather_split(const Graph& g, int mode, const int64_t* idx, int64_t n, uint32_t* out, hipStream_t s);

// cores.hip: core (mode 2) / tr-core (mode 3) numbers of the subgraph induced
// by alive (device bytes, internal order; nullptr = all vertices) into core
// (device, internal order; -2 for vertices outside).  Lists triangles if needed.
void core_numbers_gpu(Graph& g, int mode, const uint8_t* alive, int32_t* core, hipStream_t s);
// the same with host arrays by caller id (-1 outside); synchronises s
void core_numbers_caller(Graph& g, int mode, const uint8_t* alive_host, int64_t* core_host, hipStream_t s);

// fw.hip
unsigned __int128 fw_max_numerator(const Graph& g, int mode, int iters);
// lists triangles if needed, checks the key width and sizes the FW buffers
// (keys, codes, decision words) for `iters` iterations
void fw_prepare(Graph& g, int mode, int iters, hipStream_t s);
// gap and lower bound per iteration from the exact sums sum A^2, sum_patterns min A
// (4 words per iteration: low/high of each)
void fw_gap_from_sums(FwState& f, int mode, int iters, const uint64_t* sums);
void fw_run(Graph& g, int mode, int iters, bool want_gap, hipStream_t s);
// fw_run without any device allocation (lds_frank_wolfe_noalloc): the FW
// state must already be sized for iters; gap scratch from the device array
void fw_run_noalloc(Graph& g, int mode, int iters, float* r32_dev, double* gap_host, hipStream_t s);

// copy.hip: mean GPU ms of one 16-byte streaming copy of `bytes` (reps timed copies)
float copy_bandwidth(void* dst, const void* src, size_t bytes, int reps, hipStream_t s);
// mean GPU ms of n random 2-byte gathers table[idx[i]] (idx streamed; reps timed runs)
float gather_rate(const int32_t* idx, int64_t n, const uint16_t* table, int64_t entries, uint32_t* sink,
                  int reps, hipStream_t s);
void fw_loads(const Graph& g, int mode, float* r32_dev, double* r64_host, uint64_t* A_host, hipStream_t s);
void fw_splits(const Graph& g, int mode, int32_t* verts_host, uint64_t* num_host, hipStream_t s);

}  // namespace lds

// C ABI of liblds (declared in include/lds.h): argument checking, error
// translation (C++ exceptions never cross the boundary), allocator hooks.
#include "lds.h"

#include <algorithm>
#include <array>
#include <memory>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "batch.hpp"
#include "graph.hpp"
#include "handles.hpp"
#include "server.hpp"
#include "topk.hpp"
#include "tune.hpp"


struct lds_batch_s {
    lds::Batch b;
    std::vector<lds_graph> handles;  // distinct graphs, sorted (lock order)
};

namespace lds {

namespace {
thread_local std::string t_last_error;
lds_alloc_fn g_alloc = nullptr;
lds_free_fn g_free = nullptr;
void* g_ctx = nullptr;
std::atomic<int64_t> g_live{0};
}  // namespace

void set_last_error(const std::string& msg) { t_last_error = msg; }

void* dev_alloc(size_t bytes, hipStream_t s) {
    void* p = nullptr;
    if (g_alloc) {
        p = g_alloc(bytes, (void*)s, g_ctx);
        if (!p) throw Error(ST_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(ST_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
    }
    g_live.fetch_add(1);
    return p;
}

void dev_free(void* p) {
    if (!p) return;
    if (g_free)
        g_free(p, g_ctx);
    else
        (void)hipFree(p);
    g_live.fetch_sub(1);
}

}  // namespace lds

#define API_TRY try {
#define API_CATCH                                                   \
    }                                                               \
    catch (const lds::Error& e) {                                   \
        lds::set_last_error(e.what());                              \
        return (lds_status)e.code;                                  \
    }                                                               \
    catch (const std::bad_alloc&) {                                 \
        lds::set_last_error("host allocation failed");              \
        return LDS_E_NOMEM;                                         \
    }                                                               \
    catch (const std::exception& e) {                               \
        lds::set_last_error(e.what());                              \
        return LDS_E_DEVICE;                                        \
    }                                                               \
    return LDS_OK;

extern "C" {

const char* lds_last_error(void) { return lds::t_last_error.c_str(); }

lds_status lds_set_allocator(lds_alloc_fn alloc, lds_free_fn free_fn, void* ctx) {
    API_TRY
    LDS_CHECK((alloc == nullptr) == (free_fn == nullptr), lds::ST_INVALID, "alloc and free must both be set or both NULL");
    LDS_CHECK(lds::g_live.load() == 0, lds::ST_BUSY, "device memory is live: destroy all graphs first");
    lds::g_alloc = alloc;
    lds::g_free = free_fn;
    lds::g_ctx = ctx;
    API_CATCH
}

lds_status lds_create_graph(int64_t n, int64_t npairs, const int32_t* src, const int32_t* dst, uint32_t flags,
                            void* hip_stream, lds_graph* out) {
    API_TRY
    LDS_CHECK(out != nullptr, lds::ST_INVALID, "out must not be NULL");
    LDS_CHECK((flags & ~(LDS_INPUT_DEVICE | LDS_STRICT)) == 0, lds::ST_INVALID, "unknown flags");
    std::unique_ptr<lds_graph_s> h(new lds_graph_s());
    lds::build_graph(h->g, n, npairs, src, dst, (flags & LDS_INPUT_DEVICE) != 0, (flags & LDS_STRICT) != 0,
                     (hipStream_t)hip_stream);
    *out = h.release();
    API_CATCH
}

lds_status lds_destroy_graph(lds_graph g) {
    API_TRY
    if (g) {
        (void)hipStreamSynchronize(g->g.stream);
        delete g;
    }
    API_CATCH
}

lds_status lds_graph_info(lds_graph g, int64_t* n, int64_t* m, int64_t* n_triangles, size_t* device_bytes) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    if (n) *n = g->g.n;
    if (m) *m = g->g.m;
    if (n_triangles) *n_triangles = g->g.T;
    if (device_bytes) *device_bytes = g->g.device_bytes();
    API_CATCH
}

lds_status lds_triangles(lds_graph g, int64_t* n_triangles, int32_t* tri_out, int64_t cap, int64_t* tcount_out,
                         void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    lds::Graph& G = g->g;
    if (G.T < 0) lds::list_triangles(G, s);
    if (n_triangles) *n_triangles = G.T;
    const int64_t n = G.n, T = G.T;
    std::vector<int32_t> orig(n);
    if ((tri_out || tcount_out) && n > 0) {
        LDS_HIP(hipMemcpyAsync(orig.data(), G.orig_of.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    if (tri_out) {
        LDS_CHECK(cap >= T, lds::ST_INVALID, "tri_out capacity is smaller than the triangle count");
        std::vector<int32_t> t(3 * T);
        if (T > 0) {
            LDS_HIP(hipMemcpyAsync(t.data(), G.tri.p, 3 * T * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        std::vector<std::array<int32_t, 3>> v((size_t)T);
        for (int64_t i = 0; i < T; ++i) {
            std::array<int32_t, 3> x{orig[t[3 * i]], orig[t[3 * i + 1]], orig[t[3 * i + 2]]};
            std::sort(x.begin(), x.end());
            v[i] = x;
        }
        std::sort(v.begin(), v.end());
        for (int64_t i = 0; i < T; ++i)
            for (int j = 0; j < 3; ++j) tri_out[3 * i + j] = v[i][j];
    }
    if (tcount_out) {
        std::vector<int32_t> tc(n);
        if (n > 0) {
            LDS_HIP(hipMemcpyAsync(tc.data(), G.tcount.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        for (int64_t i = 0; i < n; ++i) tcount_out[orig[i]] = tc[i];
    }
    API_CATCH
}

lds_status lds_cliques4(lds_graph g, int64_t* n_cliques, int32_t* q_out, int64_t cap, int64_t* qcount_out,
                        void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    lds::Graph& G = g->g;
    if (G.Q4 < 0) lds::list_cliques4(G, s);
    if (n_cliques) *n_cliques = G.Q4;
    const int64_t n = G.n, Q = G.Q4;
    std::vector<int32_t> orig(n);
    if ((q_out || qcount_out) && n > 0) {
        LDS_HIP(hipMemcpyAsync(orig.data(), G.orig_of.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    if (q_out) {
        LDS_CHECK(cap >= Q, lds::ST_INVALID, "q_out capacity is smaller than the 4-clique count");
        std::vector<int32_t> q(4 * Q);
        if (Q > 0) {
            LDS_HIP(hipMemcpyAsync(q.data(), G.q4.p, 4 * Q * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        std::vector<std::array<int32_t, 4>> v((size_t)Q);
        for (int64_t i = 0; i < Q; ++i) {
            std::array<int32_t, 4> x{orig[q[4 * i]], orig[q[4 * i + 1]], orig[q[4 * i + 2]], orig[q[4 * i + 3]]};
            std::sort(x.begin(), x.end());
            v[i] = x;
        }
        std::sort(v.begin(), v.end());
        for (int64_t i = 0; i < Q; ++i)
            for (int j = 0; j < 4; ++j) q_out[4 * i + j] = v[i][j];
    }
    if (qcount_out) {
        std::vector<int32_t> qc(n);
        if (n > 0) {
            LDS_HIP(hipMemcpyAsync(qc.data(), G.qcount.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        for (int64_t i = 0; i < n; ++i) qcount_out[orig[i]] = qc[i];
    }
    API_CATCH
}

lds_status lds_frank_wolfe(lds_graph g, lds_mode mode, int32_t iters, float* r_out, double* r64_out,
                           uint64_t* num_out, double* gap_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    LDS_CHECK(iters >= 0, lds::ST_INVALID, "iters must be >= 0");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    lds::Graph& G = g->g;
    lds::fw_run(G, (int)mode, iters, gap_out != nullptr, s);
    if (r_out || r64_out || num_out) lds::fw_loads(G, (int)mode, r_out, r64_out, num_out, s);
    if (gap_out) {
        const auto& f = G.fw[lds::mode_slot((int)mode)];
        std::copy(f.gap.begin(), f.gap.end(), gap_out);
    }
    API_CATCH
}

lds_status lds_frank_wolfe_noalloc(lds_graph g, lds_mode mode, int32_t iters, float* r_out, double* gap_out,
                                   void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    LDS_CHECK(iters >= 0, lds::ST_INVALID, "iters must be >= 0");
    std::lock_guard<std::mutex> lk(g->mu);
    lds::fw_run_noalloc(g->g, (int)mode, iters, r_out, gap_out, (hipStream_t)hip_stream);
    API_CATCH
}

lds_status lds_splits(lds_graph g, lds_mode mode, int32_t* verts_out, uint64_t* num_out, int64_t cap,
                      int64_t* count_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    std::lock_guard<std::mutex> lk(g->mu);
    lds::Graph& G = g->g;
    const lds::SweepPlan& p = lds::plan_of(G, (int)mode);
    LDS_CHECK(mode == LDS_EDGE || (mode == LDS_TRIANGLE ? G.T >= 0 : G.Q4 >= 0), lds::ST_INVALID,
              "no pattern state for this mode: run lds_frank_wolfe first");
    if (count_out) *count_out = p.nslots;
    if (verts_out || num_out) {
        LDS_CHECK(verts_out && num_out, lds::ST_INVALID, "verts_out and num_out must both be given");
        LDS_CHECK(cap >= p.nslots, lds::ST_INVALID, "capacity is smaller than the incidence count");
        lds::fw_splits(G, (int)mode, verts_out, num_out, (hipStream_t)hip_stream);
    }
    API_CATCH
}

lds_status lds_sort_prefix(lds_graph g, lds_mode mode, int32_t* order_out, int64_t* E_out, uint8_t* inI_out,
                           void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    lds::Graph& G = g->g;
    lds::sg_sort_prefix(G, (int)mode, s);
    const lds::SgState& q = G.sg[mode == LDS_EDGE ? 0 : 1];
    const int64_t n = G.n;
    if (n > 0 && order_out) {
        std::vector<int32_t> ord(n), orig(n);
        LDS_HIP(hipMemcpyAsync(ord.data(), q.order.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipMemcpyAsync(orig.data(), G.orig_of.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        for (int64_t j = 0; j < n; ++j) order_out[j] = orig[ord[j]];
    }
    if (n > 0 && E_out) LDS_HIP(hipMemcpyAsync(E_out, q.E.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (n > 0 && inI_out) LDS_HIP(hipMemcpyAsync(inI_out, q.inI.p, n, hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    API_CATCH
}

lds_status lds_stable_groups(lds_graph g, lds_mode mode, int64_t* ngroups, int64_t* gstart, int64_t* gend, int64_t cap,
                             int64_t* lo_out, int64_t* hi_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    lds::Graph& G = g->g;
    lds::sg_stable_groups(G, (int)mode, s);
    const lds::SgState& q = G.sg[mode == LDS_EDGE ? 0 : 1];
    const int64_t ng = (int64_t)q.gstart.size();
    if (ngroups) *ngroups = ng;
    if (gstart || gend) {
        LDS_CHECK(cap >= ng, lds::ST_INVALID, "group capacity too small");
        for (int64_t i = 0; i < ng; ++i) {
            if (gstart) gstart[i] = q.gstart[i];
            if (gend) gend[i] = q.gend[i];
        }
    }
    lds::sg_copy_bounds(G, (int)mode, lo_out, hi_out, s);
    API_CATCH
}

lds_status lds_sg_scan_info(lds_graph g, lds_mode mode, int64_t* out) {
    API_TRY
    LDS_CHECK(g != nullptr && out != nullptr, lds::ST_INVALID, "graph or output is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    std::lock_guard<std::mutex> lk(g->mu);
    const lds::SgState& q = g->g.sg[mode == LDS_EDGE ? 0 : 1];
    LDS_CHECK(q.scan_wg > 0, lds::ST_INVALID, "no stable-group scan has run for this mode");
    out[0] = (int64_t)q.gstart.size();
    out[1] = q.rounds;
    out[2] = q.verifications;
    for (int k = 0; k < 4; ++k) out[3 + k] = q.scan_profile[k];
    for (int k = 0; k < 4; ++k) out[7 + k] = q.scan_profile[4 + k];
    out[11] = q.scan_profile[8];
    out[12] = q.scan_profile[9];
    out[13] = q.scan_wg;
    API_CATCH
}

lds_status lds_fw_elapsed(lds_graph g, lds_mode mode, float* ms, int32_t* launches) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    std::lock_guard<std::mutex> lk(g->mu);
    const auto& f = g->g.fw[lds::mode_slot((int)mode)];
    LDS_CHECK(f.timed && f.ev[0] != nullptr, lds::ST_INVALID, "no timed lds_frank_wolfe run for this mode");
    if (ms) {
        LDS_HIP(hipEventSynchronize(f.ev[1]));
        LDS_HIP(hipEventElapsedTime(ms, f.ev[0], f.ev[1]));
    }
    if (launches) *launches = f.launches;
    API_CATCH
}

lds_status lds_sweep_info(lds_graph g, lds_mode mode, int64_t* rows, int64_t* slots, int64_t* hub_rows,
                          int64_t* chunks, int64_t* words, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    std::lock_guard<std::mutex> lk(g->mu);
    lds::Graph& G = g->g;
    if (mode == LDS_TRIANGLE && G.T < 0) lds::list_triangles(G, (hipStream_t)hip_stream);
    if (mode == LDS_CLIQUE4 && G.Q4 < 0) lds::list_cliques4(G, (hipStream_t)hip_stream);
    const lds::SweepPlan& p = lds::plan_of(G, (int)mode);
    if (rows) *rows = p.nrows;
    if (slots) *slots = p.nslots;
    if (hub_rows) *hub_rows = p.n_hub;
    if (chunks) *chunks = p.n_chunks;
    if (words) *words = p.total_words;
    API_CATCH
}

uint64_t lds_denominator(lds_mode mode, int32_t iters) {
    if (iters < 0 || mode < LDS_EDGE || mode > LDS_CLIQUE4) return 0;
    return lds::fw_denom((int)mode, iters);
}

namespace {

// lds_result from the driver's sets (host arrays from malloc)
void fill_result(const std::vector<lds::TopkSet>& sets, const lds::TopkStats& st, lds_result* out) {
    int64_t total = 0;
    for (const auto& t : sets) total += (int64_t)t.vertices.size();
    const size_t c = sets.size();
    lds_result r;
    std::memset(&r, 0, sizeof(r));
    r.offsets = (int64_t*)std::malloc((c + 1) * sizeof(int64_t));
    r.vertices = (int32_t*)std::malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    r.dens_num = (int64_t*)std::malloc((c > 0 ? c : 1) * sizeof(int64_t));
    r.dens_den = (int64_t*)std::malloc((c > 0 ? c : 1) * sizeof(int64_t));
    if (!r.offsets || !r.vertices || !r.dens_num || !r.dens_den) {
        lds_result_free(&r);
        throw lds::Error(lds::ST_NOMEM, "host allocation of the result failed");
    }
    r.count = (int32_t)c;
    int64_t at = 0;
    for (size_t i = 0; i < c; ++i) {
        r.offsets[i] = at;
        std::copy(sets[i].vertices.begin(), sets[i].vertices.end(), r.vertices + at);
        at += (int64_t)sets[i].vertices.size();
        r.dens_num[i] = sets[i].num;
        r.dens_den[i] = sets[i].den;
    }
    r.offsets[c] = at;
    r.popped = st.popped;
    r.refinements = st.refinements;
    r.flow_splits = st.flow_splits;
    r.maxflows = st.maxflows;
    r.pruned = st.pruned;
    r.ms_copy = st.ms_copy;
    r.ms_core = st.ms_core;
    r.ms_fw = st.ms_fw;
    r.ms_prune = st.ms_prune;
    r.ms_search = st.ms_search;
    r.refine_rounds = st.refine_rounds;
    *out = r;
}

}  // namespace

lds_status lds_topk(lds_graph g, lds_mode mode, int32_t k, int32_t iters, lds_result* out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr && out != nullptr, lds::ST_INVALID, "graph and out must not be NULL");
    std::memset(out, 0, sizeof(*out));
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(k >= 1, lds::ST_INVALID, "k must be >= 1");
    LDS_CHECK(iters >= 0, lds::ST_INVALID, "iters must be >= 0");
    std::lock_guard<std::mutex> lk(g->mu);
    std::vector<lds::TopkSet> sets;
    lds::TopkStats st;
    lds::topk_run(g->g, (int)mode, k, iters, (hipStream_t)hip_stream, sets, st);
    lds_result r;
    fill_result(sets, st, &r);
    *out = r;
    API_CATCH
}

lds_status lds_prune(lds_graph g, lds_mode mode, int32_t iters, int8_t* rule_out, int64_t* pruned_out,
                     double* ms_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(iters >= 0, lds::ST_INVALID, "iters must be >= 0");
    std::lock_guard<std::mutex> lk(g->mu);
    const int64_t n = g->g.n;
    std::vector<int8_t> rule((size_t)std::max<int64_t>(n, 1), 0);
    std::vector<lds::TopkSet> sets;
    lds::TopkStats st;
    if (n > 0) lds::topk_run(g->g, (int)mode, 1, iters, (hipStream_t)hip_stream, sets, st, false, rule.data());
    if (rule_out) std::copy(rule.begin(), rule.begin() + n, rule_out);
    if (pruned_out) *pruned_out = st.pruned;
    if (ms_out) *ms_out = st.ms_prune;
    API_CATCH
}

void lds_result_free(lds_result* r) {
    if (!r) return;
    std::free(r->offsets);
    std::free(r->vertices);
    std::free(r->dens_num);
    std::free(r->dens_den);
    std::memset(r, 0, sizeof(*r));
}

lds_status lds_loads(lds_graph g, lds_mode mode, float* r_out, double* r64_out, uint64_t* num_out, double* gap_out,
                     int32_t* iters_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    std::lock_guard<std::mutex> lk(g->mu);
    lds::Graph& G = g->g;
    const auto& f = G.fw[lds::mode_slot((int)mode)];
    LDS_CHECK(f.ran, lds::ST_INVALID, "no Frank-Wolfe run for this mode");
    LDS_CHECK(gap_out == nullptr || (int)f.gap.size() == f.iters, lds::ST_INVALID,
              "the last run did not compute the gap");
    if (r_out || r64_out || num_out) lds::fw_loads(G, (int)mode, r_out, r64_out, num_out, (hipStream_t)hip_stream);
    if (gap_out) std::copy(f.gap.begin(), f.gap.end(), gap_out);
    if (iters_out) *iters_out = f.iters;
    API_CATCH
}

lds_status lds_fw_bounds(lds_graph g, lds_mode mode, double* lb_out, double* cert_gap_out) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE || mode == LDS_CLIQUE4, lds::ST_INVALID,
              "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    std::lock_guard<std::mutex> lk(g->mu);
    const auto& f = g->g.fw[lds::mode_slot((int)mode)];
    LDS_CHECK(f.ran, lds::ST_INVALID, "no Frank-Wolfe run for this mode");
    LDS_CHECK((int)f.lb.size() == f.iters && (int)f.fval.size() == f.iters, lds::ST_INVALID,
              "the last run did not compute the gap");
    double fmin = 0.0, lbmax = 0.0;
    for (int i = 0; i < f.iters; ++i) {
        fmin = (i == 0) ? f.fval[i] : std::min(fmin, f.fval[i]);
        lbmax = (i == 0) ? f.lb[i] : std::max(lbmax, f.lb[i]);
        if (lb_out) lb_out[i] = f.lb[i];
        if (cert_gap_out) cert_gap_out[i] = fmin - lbmax;
    }
    API_CATCH
}

lds_status lds_gather_rate(const int32_t* idx, int64_t n, const uint16_t* table, int64_t entries, uint32_t* sink,
                           int32_t reps, void* hip_stream, float* ms_out) {
    API_TRY
    LDS_CHECK(ms_out != nullptr, lds::ST_INVALID, "ms_out must not be NULL");
    *ms_out = lds::gather_rate(idx, n, table, entries, sink, reps, (hipStream_t)hip_stream);
    API_CATCH
}

lds_status lds_copy_bandwidth(void* dst, const void* src, size_t bytes, int32_t reps, void* hip_stream,
                              float* ms_out) {
    API_TRY
    LDS_CHECK(ms_out != nullptr, lds::ST_INVALID, "ms_out must not be NULL");
    *ms_out = lds::copy_bandwidth(dst, src, bytes, reps, (hipStream_t)hip_stream);
    API_CATCH
}

lds_status lds_core_numbers(lds_graph g, lds_mode mode, const uint8_t* alive, int64_t* core_out, void* hip_stream) {
    API_TRY
    LDS_CHECK(g != nullptr, lds::ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(core_out != nullptr || g->g.n == 0, lds::ST_INVALID, "core_out is NULL");
    std::lock_guard<std::mutex> lk(g->mu);
    lds::core_numbers_caller(g->g, (int)mode, alive, core_out, (hipStream_t)hip_stream);
    API_CATCH
}

void lds_tune_default(lds_tune* out) {
    if (!out) return;
    const lds::BatchTune t;
    out->threads = t.threads;
    out->wg_per_cu = t.wg_per_cu;
    out->lds_vertices = t.lds_vertices;
    out->longest_first = t.longest_first;
    out->max_kernel_cost = t.max_kernel_cost;
}

namespace {

lds::BatchTune to_tune(const lds_tune* t) {
    lds::BatchTune b;
    if (t) {
        b.threads = t->threads;
        b.wg_per_cu = t->wg_per_cu;
        b.lds_vertices = t->lds_vertices;
        b.longest_first = t->longest_first;
        b.max_kernel_cost = t->max_kernel_cost;
    }
    return b;
}

void from_tune(const lds::BatchTune& b, lds_tune* t) {
    t->threads = b.threads;
    t->wg_per_cu = b.wg_per_cu;
    t->lds_vertices = b.lds_vertices;
    t->longest_first = b.longest_first;
    t->max_kernel_cost = b.max_kernel_cost;
}

// checks the batch arguments and fills the graph list; returns the distinct handles sorted
std::vector<lds_graph> batch_setup(lds::Batch& b, const lds_graph* graphs, const lds_mode* modes, const int32_t* iters,
                                   float* const* r_out, int32_t count) {
    LDS_CHECK(count >= 0, lds::ST_INVALID, "count must be >= 0");
    LDS_CHECK(count == 0 || (graphs && modes && iters), lds::ST_INVALID, "graphs, modes and iters must be given");
    std::vector<std::pair<lds_graph, int>> seen;
    for (int32_t i = 0; i < count; ++i) {
        LDS_CHECK(graphs[i] != nullptr, lds::ST_INVALID, "graph is NULL");
        LDS_CHECK(modes[i] == LDS_EDGE || modes[i] == LDS_TRIANGLE, lds::ST_INVALID, "bad mode");
        LDS_CHECK(iters[i] >= 0, lds::ST_INVALID, "iters must be >= 0");
        seen.push_back({graphs[i], (int)modes[i]});
        b.gs.push_back(&graphs[i]->g);
        b.modes.push_back((int)modes[i]);
        b.iters.push_back(iters[i]);
        b.r_out.push_back(r_out ? r_out[i] : nullptr);
    }
    std::sort(seen.begin(), seen.end());
    LDS_CHECK(std::adjacent_find(seen.begin(), seen.end()) == seen.end(), lds::ST_INVALID,
              "a (graph, mode) pair appears twice in the batch");
    std::vector<lds_graph> hs;
    for (auto& x : seen) hs.push_back(x.first);
    hs.erase(std::unique(hs.begin(), hs.end()), hs.end());
    return hs;
}

struct MultiLock {
    std::vector<std::unique_lock<std::mutex>> locks;
    explicit MultiLock(const std::vector<lds_graph>& hs) {
        for (lds_graph h : hs) locks.emplace_back(h->mu);  // sorted: one global order
    }
};

}  // namespace

lds_status lds_batch_create(const lds_graph* graphs, const lds_mode* modes, const int32_t* iters, float* const* r_out,
                            int32_t count, uint32_t flags, const lds_tune* tune, void* hip_stream, lds_batch* out) {
    API_TRY
    LDS_CHECK(out != nullptr, lds::ST_INVALID, "out must not be NULL");
    LDS_CHECK((flags & ~LDS_BATCH_GAP) == 0, lds::ST_INVALID, "unknown flags");
    std::unique_ptr<lds_batch_s> h(new lds_batch_s());
    h->handles = batch_setup(h->b, graphs, modes, iters, r_out, count);
    h->b.want_gap = (flags & LDS_BATCH_GAP) != 0;
    h->b.tune = to_tune(tune);
    MultiLock lk(h->handles);
    lds::batch_build(h->b, (hipStream_t)hip_stream);
    *out = h.release();
    API_CATCH
}

lds_status lds_batch_run(lds_batch b, void* hip_stream) {
    API_TRY
    LDS_CHECK(b != nullptr, lds::ST_INVALID, "batch is NULL");
    MultiLock lk(b->handles);
    lds::batch_run(b->b, (hipStream_t)hip_stream);
    API_CATCH
}

lds_status lds_batch_info(lds_batch b, int32_t* kernel_graphs, int32_t* plain_graphs, float* kernel_ms,
                          lds_tune* tune) {
    API_TRY
    LDS_CHECK(b != nullptr, lds::ST_INVALID, "batch is NULL");
    if (kernel_graphs) *kernel_graphs = (int32_t)b->b.kernel_items.size();
    if (plain_graphs) *plain_graphs = (int32_t)b->b.plain_items.size();
    if (kernel_ms) {
        LDS_CHECK(b->b.runs > 0, lds::ST_INVALID, "the batch has not run");
        LDS_HIP(hipEventSynchronize(b->b.ev[1]));
        LDS_HIP(hipEventElapsedTime(kernel_ms, b->b.ev[0], b->b.ev[1]));
    }
    if (tune) from_tune(b->b.tune, tune);
    API_CATCH
}

lds_status lds_batch_destroy(lds_batch b) {
    API_TRY
    delete b;
    API_CATCH
}

lds_status lds_batch_autotune(const lds_graph* graphs, const lds_mode* modes, const int32_t* iters, int32_t count,
                              const char* cache_path, int32_t reps, lds_tune* best, double* best_ms,
                              void* hip_stream) {
    API_TRY
    LDS_CHECK(best != nullptr, lds::ST_INVALID, "best must not be NULL");
    LDS_CHECK(reps >= 1, lds::ST_INVALID, "reps must be >= 1");
    lds_batch_s tmp;
    tmp.handles = batch_setup(tmp.b, graphs, modes, iters, nullptr, count);
    MultiLock lk(tmp.handles);
    bool cached = false;
    double ms = -1;
    const lds::BatchTune t =
        lds::autotune(tmp.b, cache_path ? std::string(cache_path) : std::string(), reps, (hipStream_t)hip_stream,
                      &cached, &ms);
    from_tune(t, best);
    if (best_ms) *best_ms = cached ? -1.0 : ms;
    API_CATCH
}

struct lds_server_s {
    lds::Server* s = nullptr;
    ~lds_server_s() { delete s; }
};

lds_status lds_footprint(lds_graph g, lds_mode mode, int32_t iters, size_t* bytes) {
    API_TRY
    LDS_CHECK(g != nullptr && bytes != nullptr, lds::ST_INVALID, "graph and bytes must not be NULL");
    LDS_CHECK(mode == LDS_EDGE || mode == LDS_TRIANGLE, lds::ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(iters >= 0, lds::ST_INVALID, "iters must be >= 0");
    std::lock_guard<std::mutex> lk(g->mu);
    LDS_CHECK(mode == LDS_EDGE || g->g.T >= 0, lds::ST_INVALID, "triangles not listed yet (lds_triangles)");
    *bytes = lds::topk_footprint(g->g, (int)mode, iters);
    API_CATCH
}

lds_status lds_server_create(size_t hbm_budget, int32_t max_slots, int32_t workers, lds_server* out) {
    API_TRY
    LDS_CHECK(out != nullptr, lds::ST_INVALID, "out must not be NULL");
    LDS_CHECK(max_slots >= 1, lds::ST_INVALID, "max_slots must be >= 1");
    LDS_CHECK(workers >= 1 && workers <= 64, lds::ST_INVALID, "workers must be in [1, 64]");
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        LDS_HIP(hipMemGetInfo(&fr, &tot));
        hbm_budget = fr / 10 * 9;
    }
    std::unique_ptr<lds_server_s> h(new lds_server_s());
    h->s = new lds::Server(hbm_budget, max_slots, workers);
    *out = h.release();
    API_CATCH
}

lds_status lds_server_submit(lds_server s, lds_graph g, lds_mode mode, int32_t k, int32_t iters, uint64_t tag,
                             double t_arrive) {
    API_TRY
    LDS_CHECK(s != nullptr, lds::ST_INVALID, "server is NULL");
    s->s->submit(g, (int)mode, k, iters, tag, t_arrive);
    API_CATCH
}

lds_status lds_server_poll(lds_server s, lds_completion* out, int32_t max, double wait_s, int32_t* n_out) {
    API_TRY
    LDS_CHECK(s != nullptr && n_out != nullptr, lds::ST_INVALID, "server and n_out must not be NULL");
    LDS_CHECK(max >= 0 && (max == 0 || out != nullptr), lds::ST_INVALID, "bad output array");
    std::vector<lds::SDone> got;
    s->s->poll(got, (size_t)max, wait_s);
    for (size_t i = 0; i < got.size(); ++i) {
        lds_completion& c = out[i];
        std::memset(&c, 0, sizeof(c));
        c.tag = got[i].tag;
        c.status = got[i].status;
        c.t_arrive = got[i].t_arrive;
        c.t_admit = got[i].t_admit;
        c.t_done = got[i].t_done;
        std::strncpy(c.error, got[i].error.c_str(), sizeof(c.error) - 1);
        if (got[i].status == lds::ST_OK) fill_result(got[i].sets, got[i].st, &c.result);
    }
    *n_out = (int32_t)got.size();
    API_CATCH
}

lds_status lds_server_clock(lds_server s, double* now) {
    API_TRY
    LDS_CHECK(s != nullptr && now != nullptr, lds::ST_INVALID, "server and now must not be NULL");
    *now = s->s->clock();
    API_CATCH
}

lds_status lds_server_stats(lds_server s, lds_server_info* out) {
    API_TRY
    LDS_CHECK(s != nullptr && out != nullptr, lds::ST_INVALID, "server and out must not be NULL");
    const lds::SStats st = s->s->stats();
    out->submitted = st.submitted;
    out->completed = st.completed;
    out->batches = st.batches;
    out->max_batch = st.max_batch;
    out->pending = st.pending;
    out->active = st.active;
    out->inflight_bytes = st.inflight;
    out->peak_inflight_bytes = st.peak_inflight;
    out->batch_ms = st.batch_ms;
    API_CATCH
}

lds_status lds_server_destroy(lds_server s) {
    API_TRY
    delete s;
    API_CATCH
}

}  // extern "C"

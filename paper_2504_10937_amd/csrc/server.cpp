// Serving loop for top-k LDS / LTDS queries on resident graphs, with
// continuous batching:
//   * submit() queues a query (graph handle, mode, k, iterations) with its
//     arrival time; graphs stay resident (CSR, triangle list, FW buffers).
//   * the scheduler thread admits queued queries in arrival order while the
//     device-memory budget and the slot count allow (a query's footprint is
//     the FW / stable-group state it adds to its graph); every admitted query
//     works on its own view of its graph (the graph's device data borrowed,
//     its own FW and stable-group state), so queries on one graph and mode run
//     at once; all queries admitted together run their Frank-Wolfe
//     iterations in ONE batched launch (the persistent kernel of batch.hip),
//     then go to the verification workers.
//   * worker threads run the rest of the top-k search (stable groups,
//     pruning, exact verification, refinements) on their own streams, so the
//     next batch's kernel overlaps with the verification of the previous one;
//     when a query completes its memory and slot are released and the
//     scheduler admits more.
// Every query starts FW from the canonical initial point, so its result is a
// pure function of (graph, mode, k, iterations), whatever else is in flight.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <set>
#include <thread>

#include "batch.hpp"
#include "handles.hpp"
#include "server.hpp"
#include "topk.hpp"

namespace lds {

InFlight::~InFlight() {
    if (done) (void)hipEventDestroy(done);
}

namespace {

constexpr int kBatchStreams = 4;  // batched launches in flight at once
// (incidences + vertices) * iters kept in the batched kernel; the
// environment variable LDS_SERVE_KERNEL_COST overrides it
constexpr int64_t kServeKernelCost = 1ll << 22;
constexpr int kReadyPollUs = 500;  // a worker with only unfinished batched FW queued looks again after this

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct Server::Impl {
    size_t budget;
    int max_slots;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::mutex mu;
    std::condition_variable cv_sched, cv_work, cv_done;
    std::deque<SQuery> pending, verify;
    std::deque<SDone> done;
    size_t inflight = 0;
    int active = 0;
    bool stop = false;          // scheduler: admit nothing more
    bool stop_workers = false;  // workers: exit once the verification queue is empty
    SStats stats;
    std::thread sched;
    std::vector<std::thread> workers;
    hipStream_t sched_stream = nullptr;   // triangle listing at submission
    hipStream_t bstream[kBatchStreams] = {};
    int next_stream = 0;
    int device = 0;
    int64_t kernel_cost = kServeKernelCost;

    void finish(SQuery& q, SDone&& d) {
        std::lock_guard<std::mutex> lk(mu);
        d.tag = q.tag;
        d.t_arrive = q.t_arrive;
        d.t_admit = q.t_admit;
        d.t_done = now_s(t0);
        if (q.admitted) {
            inflight -= q.fp;
            --active;
        }
        stats.completed++;
        done.push_back(std::move(d));
        cv_done.notify_all();
        cv_sched.notify_all();
    }

    void scheduler() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            std::vector<SQuery> adm;
            std::vector<SQuery> rejected;
            for (;;) {
                if (stop) return;
                adm.clear();
                for (auto it = pending.begin(); it != pending.end();) {
                    if (active + (int)adm.size() >= max_slots) break;
                    if (it->fp > budget) {  // can never fit
                        rejected.push_back(std::move(*it));
                        it = pending.erase(it);
                        continue;
                    }
                    size_t add = it->fp;
                    for (const auto& a : adm) add += a.fp;
                    if (inflight + add > budget) break;  // memory is granted in arrival order
                    adm.push_back(std::move(*it));
                    it = pending.erase(it);
                }
                if (!adm.empty() || !rejected.empty()) break;
                cv_sched.wait(lk);
            }
            for (auto& q : adm) {
                q.admitted = true;
                q.t_admit = now_s(t0);
                inflight += q.fp;
                ++active;
            }
            stats.batches += adm.empty() ? 0 : 1;
            stats.max_batch = std::max<int64_t>(stats.max_batch, (int64_t)adm.size());
            stats.peak_inflight = std::max(stats.peak_inflight, inflight);
            lk.unlock();
            for (auto& q : rejected) {
                SDone d;
                d.status = ST_NOMEM;
                d.error = "the query's device footprint exceeds the server's memory budget";
                finish(q, std::move(d));
            }
            // graphs too large for one workgroup run FW on their worker's own
            // stream (their many per-iteration launches would otherwise keep
            // this thread from admitting); the rest share one batched launch
            std::vector<SQuery> solo;
            {
                std::vector<SQuery> keep;
                for (auto& q : adm) {
                    int64_t cost = 0;
                    {
                        std::lock_guard<std::mutex> g(q.h->mu);
                        cost = batch_cost(q.h->g, q.mode, q.iters);
                    }
                    (cost > kernel_cost ? solo : keep).push_back(std::move(q));
                }
                adm.swap(keep);
            }
            if (!solo.empty()) {
                std::lock_guard<std::mutex> g(mu);
                for (auto& q : solo) verify.push_back(std::move(q));
                cv_work.notify_all();
            }
            if (!adm.empty()) {
                // one batched FW launch for everything admitted together
                std::string err;
                int code = ST_OK;
                const auto tb = std::chrono::steady_clock::now();
                auto fl = std::make_shared<InFlight>();
                hipStream_t bs = bstream[next_stream];
                next_stream = (next_stream + 1) % kBatchStreams;
                try {
                    // launched, not waited for: the workers wait on the event
                    for (auto& q : adm) {
                        std::lock_guard<std::mutex> g(q.h->mu);
                        q.view = graph_view(q.h->g, bs);
                    }
                    fl->b.reset(new Batch);
                    Batch& b = *fl->b;
                    b.capture = false;
                    // latency first: a graph whose FW would keep one
                    // workgroup busy for more than a few ms runs on its own
                    // launches (the whole GPU per iteration) instead
                    b.tune.max_kernel_cost = kernel_cost;
                    for (auto& q : adm) {
                        b.gs.push_back(q.view.get());
                        b.modes.push_back(q.mode);
                        b.iters.push_back(q.iters);
                    }
                    batch_build(b, bs);
                    batch_run(b, bs);
                    LDS_HIP(hipEventCreateWithFlags(&fl->done, hipEventDisableTiming));
                    LDS_HIP(hipEventRecord(fl->done, bs));
                } catch (const Error& e) {
                    code = e.code;
                    err = e.what();
                } catch (const std::exception& e) {
                    code = ST_DEVICE;
                    err = e.what();
                }
                {
                    std::lock_guard<std::mutex> g(mu);
                    stats.batch_ms +=
                        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tb).count();
                }
                if (code != ST_OK) {
                    (void)hipStreamSynchronize(bs);  // nothing of the failed batch may still run
                    fl.reset();
                    for (auto& q : adm) {
                        SDone d;
                        d.status = code;
                        d.error = err;
                        finish(q, std::move(d));
                    }
                } else {
                    std::lock_guard<std::mutex> g(mu);
                    for (auto& q : adm) {
                        q.fw = fl;
                        verify.push_back(std::move(q));
                    }
                    cv_work.notify_all();
                }
            }
            lk.lock();
        }
    }

    void worker() {
        (void)hipSetDevice(device);
        topk_single_thread(true);  // the other workers use the other cores
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
        for (;;) {
            SQuery q;
            {
                // the oldest query that can run now: its batched FW has
                // finished (or it has none), so the worker never sits on a
                // launch that other queries' verification could overlap
                std::unique_lock<std::mutex> lk(mu);
                auto ready = verify.end();
                for (;;) {
                    cv_work.wait(lk, [&] { return stop_workers || !verify.empty(); });
                    if (verify.empty()) break;  // stopping and nothing left
                    ready = std::find_if(verify.begin(), verify.end(), [](const SQuery& x) {
                        return !x.fw || !x.fw->done || hipEventQuery(x.fw->done) != hipErrorNotReady;
                    });
                    if (ready != verify.end()) break;
                    cv_work.wait_for(lk, std::chrono::microseconds(kReadyPollUs));
                }
                if (verify.empty()) break;
                q = std::move(*ready);
                verify.erase(ready);
            }
            SDone d;
            try {
                if (q.fw && q.fw->done) LDS_HIP(hipStreamWaitEvent(s, q.fw->done, 0));
                if (!q.view) {  // a query that was not in a batched launch runs its own FW here
                    std::lock_guard<std::mutex> g(q.h->mu);
                    q.view = graph_view(q.h->g, s);
                }
                topk_run(*q.view, q.mode, q.k, q.iters, s, d.sets, d.st, q.fw != nullptr);
                d.status = ST_OK;
            } catch (const Error& e) {
                d.status = e.code;
                d.error = e.what();
            } catch (const std::bad_alloc&) {
                d.status = ST_NOMEM;
                d.error = "host allocation failed";
            } catch (const std::exception& e) {
                d.status = ST_DEVICE;
                d.error = e.what();
            }
            if (s) (void)hipStreamSynchronize(s);
            q.view.reset();  // the query's FW and stable-group state
            q.fw.reset();    // the batch's tables are freed with its last query
            finish(q, std::move(d));
        }
        if (s) (void)hipStreamDestroy(s);
    }
};

Server::Server(size_t budget, int max_slots, int workers) : p(new Impl) {
    p->budget = budget;
    p->max_slots = max_slots;
    if (const char* e = std::getenv("LDS_SERVE_KERNEL_COST"))
        if (*e) p->kernel_cost = std::max<int64_t>(0, std::atoll(e));
    LDS_HIP(hipGetDevice(&p->device));
    LDS_HIP(hipStreamCreateWithFlags(&p->sched_stream, hipStreamNonBlocking));
    for (auto& bs : p->bstream) LDS_HIP(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
    p->sched = std::thread([this] { p->scheduler(); });
    for (int i = 0; i < workers; ++i) p->workers.emplace_back([this] { p->worker(); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop = true;
        p->pending.clear();  // queued queries that were never admitted are dropped
    }
    p->cv_sched.notify_all();
    if (p->sched.joinable()) p->sched.join();  // finishes the batch it is running, if any
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop_workers = true;
    }
    p->cv_work.notify_all();
    for (auto& t : p->workers)
        if (t.joinable()) t.join();  // the admitted queries are finished
    for (auto& bs : p->bstream)
        if (bs) {
            (void)hipStreamSynchronize(bs);
            (void)hipStreamDestroy(bs);
        }
    if (p->sched_stream) (void)hipStreamDestroy(p->sched_stream);
    delete p;
}

void Server::submit(lds_graph h, int mode, int k, int iters, uint64_t tag, double t_arrive) {
    LDS_CHECK(h != nullptr, ST_INVALID, "graph is NULL");
    LDS_CHECK(mode == 2 || mode == 3, ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(k >= 1, ST_INVALID, "k must be >= 1");
    LDS_CHECK(iters >= 0, ST_INVALID, "iters must be >= 0");
    check_split_width(mode, iters);
    SQuery q;
    q.h = h;
    q.mode = mode;
    q.k = k;
    q.iters = iters;
    q.tag = tag;
    {
        // the footprint needs the triangle count: list triangles once, on the
        // graph's first triangle query
        std::lock_guard<std::mutex> g(h->mu);
        if (mode == 3 && h->g.T < 0) {
            list_triangles(h->g, p->sched_stream);
            LDS_HIP(hipStreamSynchronize(p->sched_stream));
        }
        q.fp = topk_footprint(h->g, mode, iters);
    }
    std::lock_guard<std::mutex> lk(p->mu);
    LDS_CHECK(!p->stop, ST_INVALID, "server is stopping");
    q.t_arrive = t_arrive >= 0 ? t_arrive : now_s(p->t0);
    p->pending.push_back(std::move(q));
    p->stats.submitted++;
    p->cv_sched.notify_all();
}

size_t Server::poll(std::vector<SDone>& out, size_t max, double wait_s) {
    std::unique_lock<std::mutex> lk(p->mu);
    if (p->done.empty() && wait_s > 0)
        p->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s), [&] { return !p->done.empty(); });
    size_t c = 0;
    while (c < max && !p->done.empty()) {
        out.push_back(std::move(p->done.front()));
        p->done.pop_front();
        ++c;
    }
    return c;
}

double Server::clock() const { return now_s(p->t0); }

SStats Server::stats() {
    std::lock_guard<std::mutex> lk(p->mu);
    SStats s = p->stats;
    s.pending = (int64_t)p->pending.size();
    s.active = p->active;
    s.inflight = p->inflight;
    return s;
}

}  // namespace lds

// Continuous-batching query server (server.cpp).
#pragma once
#include <memory>
#include <string>
#include <vector>

#include "lds.h"
#include "topk.hpp"

namespace lds {

struct Batch;

// a batched FW launch in flight: the batch (its device tables stay alive
// until every query of it is verified) and the event that marks its end
struct InFlight {
    std::unique_ptr<Batch> b;
    hipEvent_t done = nullptr;
    ~InFlight();
};

struct SQuery {
    std::shared_ptr<InFlight> fw;  // the launch that computed this query's FW state
    std::shared_ptr<Graph> view;   // the query's view of its graph (own FW / stable-group state)
    lds_graph h = nullptr;
    int mode = 2, k = 1, iters = 0;
    uint64_t tag = 0;
    size_t fp = 0;  // device bytes the query adds to its graph
    double t_arrive = 0, t_admit = -1;
    bool admitted = false;
};

struct SDone {
    uint64_t tag = 0;
    int status = 0;
    std::string error;
    std::vector<TopkSet> sets;
    TopkStats st;
    double t_arrive = 0, t_admit = -1, t_done = 0;
};

struct SStats {
    int64_t submitted = 0, completed = 0, batches = 0, max_batch = 0, pending = 0, active = 0;
    size_t inflight = 0, peak_inflight = 0;
    double batch_ms = 0;  // wall time of the scheduler's batched FW launches
};

class Server {
public:
    Server(size_t budget, int max_slots, int workers);
    ~Server();
    void submit(lds_graph h, int mode, int k, int iters, uint64_t tag, double t_arrive);
    size_t poll(std::vector<SDone>& out, size_t max, double wait_s);
    double clock() const;  // seconds since creation (the time base of arrivals and completions)
    SStats stats();

private:
    struct Impl;
    Impl* p;
};

}  // namespace lds

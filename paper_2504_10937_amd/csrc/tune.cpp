// Autotuner of the batched Frank-Wolfe launch: times a small set of launch
// shapes on the caller's batch (workgroup size x workgroups per CU, queue
// order, the work above which a graph runs on its own launches) and keeps
// the fastest, with a JSON cache keyed
// by a coarse signature of the batch (graph count, total work, largest graph,
// edge / triangle mix, compute units), so that later batches of the same
// shape skip the timing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "batch.hpp"
#include "tune.hpp"

namespace lds {

namespace {

int cus() {
    int dev = 0, c = 0;
    LDS_HIP(hipGetDevice(&dev));
    LDS_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    return c;
}

int log2i(double x) { return x <= 1 ? 0 : (int)std::lround(std::log2(x)); }

std::string entry_json(const std::string& key, const BatchTune& t, double ms) {
    std::ostringstream o;
    o << "{\"key\": \"" << key << "\", \"threads\": " << t.threads << ", \"wg_per_cu\": " << t.wg_per_cu
      << ", \"lds_vertices\": " << t.lds_vertices << ", \"max_kernel_cost\": " << t.max_kernel_cost
      << ", \"longest_first\": " << t.longest_first << ", \"ms\": " << ms << "}";
    return o.str();
}

// value of "name": <integer> inside one entry line
bool field(const std::string& line, const char* name, int64_t* v) {
    const std::string pat = std::string("\"") + name + "\": ";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    *v = std::strtoll(line.c_str() + p + pat.size(), nullptr, 10);
    return true;
}

}  // namespace

std::string tune_signature(const std::vector<Graph*>& gs, const std::vector<int>& modes,
                           const std::vector<int>& iters) {
    double cost = 0;
    int64_t maxn = 0, ne = 0;
    for (size_t i = 0; i < gs.size(); ++i) {
        cost += (double)batch_cost(*gs[i], modes[i], iters[i]);
        maxn = std::max(maxn, gs[i]->n);
        ne += modes[i] == 2 ? 1 : 0;
    }
    std::ostringstream o;
    o << "v2/count=" << log2i((double)gs.size()) << "/cost=" << log2i(cost) << "/maxn=" << log2i((double)maxn)
      << "/edgefrac=" << (gs.empty() ? 0 : (int)(4 * ne / (int64_t)gs.size())) << "/cus=" << cus();
    return o.str();
}

bool tune_cache_lookup(const std::string& path, const std::string& key, BatchTune* out) {
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    const std::string kq = "\"key\": \"" + key + "\"";
    while (std::getline(f, line)) {
        if (line.find(kq) == std::string::npos) continue;
        int64_t v;
        BatchTune t;
        if (!field(line, "threads", &v)) return false;
        t.threads = (int)v;
        if (!field(line, "wg_per_cu", &v)) return false;
        t.wg_per_cu = (int)v;
        if (!field(line, "lds_vertices", &v)) return false;
        t.lds_vertices = (int)v;
        if (!field(line, "max_kernel_cost", &v)) return false;
        t.max_kernel_cost = v;
        if (!field(line, "longest_first", &v)) return false;
        t.longest_first = (int)v;
        *out = t;
        return true;
    }
    return false;
}

void tune_cache_store(const std::string& path, const std::string& key, const BatchTune& t, double ms) {
    // one entry per line inside {"entries": [ ... ]}; an entry with the same
    // key is replaced
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line;
        const std::string kq = "\"key\": \"" + key + "\"";
        while (f && std::getline(f, line)) {
            if (line.find("\"key\": ") == std::string::npos || line.find(kq) != std::string::npos) continue;
            while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
            size_t b = line.find('{');
            if (b != std::string::npos) keep.push_back(line.substr(b));
        }
    }
    keep.push_back(entry_json(key, t, ms));
    const std::string tmp = path + ".tmp";
    {
        std::ofstream o(tmp);
        LDS_CHECK((bool)o, ST_INVALID, "cannot write the autotune cache " + path);
        o << "{\"entries\": [\n";
        for (size_t i = 0; i < keep.size(); ++i) o << "  " << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
        o << "]}\n";
    }
    LDS_CHECK(std::rename(tmp.c_str(), path.c_str()) == 0, ST_INVALID, "cannot replace the autotune cache " + path);
}

// launch shapes: workgroup size x workgroups per CU x the largest graph
// whose keys live in LDS (two 8-byte buffers per vertex); a shape whose
// workgroups' key buffers do not fit one CU's 160 KB of LDS together is left
// out, since its extra workgroups could not be resident
std::vector<BatchTune> tune_candidates() {
    std::vector<BatchTune> c;
    for (int th : {256, 512, 1024})
        for (int wpc : {1, 2, 4})
            for (int lv : {8192, 4096, 2048, 0}) {
                if (th * wpc > 2048) continue;
                if ((size_t)wpc * 2 * 8 * (size_t)lv > (size_t)150 * 1024) continue;
                BatchTune t;
                t.threads = th;
                t.wg_per_cu = wpc;
                t.lds_vertices = lv;
                c.push_back(t);
            }
    return c;
}

double time_batch(Batch& b, int reps, hipStream_t s) {
    batch_build(b, s);
    batch_run(b, s);  // warm-up
    LDS_HIP(hipStreamSynchronize(s));
    std::vector<double> t;
    for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        batch_run(b, s);
        LDS_HIP(hipStreamSynchronize(s));
        t.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

BatchTune autotune(Batch& b, const std::string& cache, int reps, hipStream_t s, bool* from_cache, double* best_ms) {
    // triangle lists first: the signature counts triangle incidences
    for (size_t i = 0; i < b.gs.size(); ++i) fw_prepare(*b.gs[i], b.modes[i], b.iters[i], s);
    const std::string key = tune_signature(b.gs, b.modes, b.iters);
    BatchTune t;
    if (!cache.empty() && tune_cache_lookup(cache, key, &t)) {
        *from_cache = true;
        *best_ms = -1;
        return t;
    }
    *from_cache = false;
    double best = 1e300;
    BatchTune bt;
    // shape of the workgroups and the LDS-resident threshold
    for (const BatchTune& c : tune_candidates()) {
        b.tune = c;
        const double ms = time_batch(b, reps, s);
        if (ms < best) {
            best = ms;
            bt = c;
        }
    }
    // queue order
    {
        BatchTune c = bt;
        c.longest_first = 0;
        b.tune = c;
        const double ms = time_batch(b, reps, s);
        if (ms < best) {
            best = ms;
            bt = c;
        }
    }
    // which graphs are too large for one workgroup
    for (int64_t cut : {1ll << 24, 1ll << 30}) {
        BatchTune c = bt;
        c.max_kernel_cost = cut;
        b.tune = c;
        const double ms = time_batch(b, reps, s);
        if (ms < best) {
            best = ms;
            bt = c;
        }
    }
    *best_ms = best;
    if (!cache.empty()) tune_cache_store(cache, key, bt, best);
    return bt;
}

}  // namespace lds

// Autotuner of the batched launch (tune.cpp).
#pragma once
#include <string>
#include <vector>

#include "batch.hpp"

namespace lds {

std::string tune_signature(const std::vector<Graph*>& gs, const std::vector<int>& modes,
                           const std::vector<int>& iters);
bool tune_cache_lookup(const std::string& path, const std::string& key, BatchTune* out);
void tune_cache_store(const std::string& path, const std::string& key, const BatchTune& t, double ms);
std::vector<BatchTune> tune_candidates();
// median wall time (ms) of `reps` runs of the batch with its current tune
double time_batch(Batch& b, int reps, hipStream_t s);
// best tune for the batch: from the cache when its signature is there, else
// timed over the candidates (and stored)
BatchTune autotune(Batch& b, const std::string& cache, int reps, hipStream_t s, bool* from_cache, double* best_ms);

}  // namespace lds

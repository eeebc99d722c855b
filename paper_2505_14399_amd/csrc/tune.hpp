// Autotuner: per-(kernel, shape) choice of a launch variant, measured with HIP events on first
// use while tuning is enabled, kept in memory and optionally saved to / loaded from JSON.
#pragma once

#include <functional>
#include <string>

#include "qmg_internal.hpp"

namespace qmg {

bool tune_enabled();
void tune_enable(bool on);
// cached choice for key, or -1
int tune_lookup(const std::string& key);
void tune_store(const std::string& key, int choice);
// time every candidate (run(c) enqueues one launch of variant c on st) and store the fastest;
// returns the chosen candidate.  Skipped (returns candidates[0]) while st is being captured.
int tune_measure(const std::string& key, const int* candidates, int n, hipStream_t st,
                 const std::function<void(int)>& run);
int tune_save(const char* path);
int tune_load(const char* path);

}  // namespace qmg

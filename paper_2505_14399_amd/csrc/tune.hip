// Autotuner cache (see tune.hpp).  JSON format: {"key": choice, ...}.
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "tune.hpp"

namespace qmg {

namespace {
std::mutex g_mu;
std::map<std::string, int> g_cache;
int g_on = -1;  // -1: not yet read from QMG_TUNE
}  // namespace

bool tune_enabled() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_on < 0) {
    const char* e = std::getenv("QMG_TUNE");
    g_on = (e && e[0] == '1') ? 1 : 0;
  }
  return g_on == 1;
}

void tune_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on ? 1 : 0;
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key);
  return it == g_cache.end() ? -1 : it->second;
}

void tune_store(const std::string& key, int choice) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = choice;
}

int tune_measure(const std::string& key, const int* cand, int n, hipStream_t st,
                 const std::function<void(int)>& run) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  QMG_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return cand[0];
  hipEvent_t e0, e1;
  QMG_HIP(hipEventCreate(&e0));
  QMG_HIP(hipEventCreate(&e1));
  int best = cand[0];
  float best_ms = 1e30f;
  for (int i = 0; i < n; ++i) {
    run(cand[i]);  // warm-up
    QMG_HIP(hipEventRecord(e0, st));
    for (int rep = 0; rep < 3; ++rep) run(cand[i]);
    QMG_HIP(hipEventRecord(e1, st));
    QMG_HIP(hipEventSynchronize(e1));
    float ms = 0;
    QMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = cand[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_store(key, best);
  return best;
}

int tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ofstream f(path);
  if (!f) return -1;
  f << "{";
  bool first = true;
  for (auto& kv : g_cache) {
    f << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": " << kv.second;
    first = false;
  }
  f << "\n}\n";
  return f ? 0 : -1;
}

int tune_load(const char* path) {
  std::ifstream f(path);
  if (!f) return -1;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  int n = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) return -1;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t colon = s.find(':', end);
    if (colon == std::string::npos) return -1;
    const int v = std::atoi(s.c_str() + colon + 1);
    tune_store(key, v);
    ++n;
    pos = s.find_first_of(",}", colon);
    if (pos == std::string::npos) break;
  }
  return n;
}

}  // namespace qmg

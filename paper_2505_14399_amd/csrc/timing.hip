// Optional per-kernel-family timing: when enabled, each launch of an instrumented kernel is
// bracketed by a pair of HIP events recorded on the launch stream, and the launcher adds the
// algorithmic bytes and flops of that launch.  Off by default (no events are recorded).
#include <map>
#include <mutex>
#include <string>

#include "timing.hpp"

namespace qmg {

namespace {
struct Family {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double bytes = 0, flops = 0;
};
std::mutex g_mu;
bool g_on = false;
std::map<std::string, Family> g_fam;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  QMG_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

bool timing_on() { return g_on; }

TimedLaunch::TimedLaunch(const char* family, hipStream_t st, double bytes, double flops)
    : fam_(family), st_(st), bytes_(bytes), flops_(flops) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  e0_ = get_event();
  e1_ = get_event();
  QMG_HIP(hipEventRecord(e0_, st_));
}

TimedLaunch::~TimedLaunch() {
  if (!e0_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(e1_, st_);
  Family& f = g_fam[fam_];
  f.ev.emplace_back(e0_, e1_);
  f.bytes += bytes_;
  f.flops += flops_;
}

void timing_enable(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_fam)
    for (auto& p : kv.second.ev) {
      g_pool.push_back(p.first);
      g_pool.push_back(p.second);
    }
  g_fam.clear();
  g_on = on;
}

void timing_query(const char* family, int64_t* n, double* ms, double* bytes, double* flops) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_fam.find(family);
  *n = 0;
  *ms = 0;
  *bytes = 0;
  *flops = 0;
  if (it == g_fam.end()) return;
  for (auto& p : it->second.ev) {
    QMG_HIP(hipEventSynchronize(p.second));
    float t = 0;
    QMG_HIP(hipEventElapsedTime(&t, p.first, p.second));
    *ms += t;
  }
  *n = int64_t(it->second.ev.size());
  *bytes = it->second.bytes;
  *flops = it->second.flops;
}

}  // namespace qmg

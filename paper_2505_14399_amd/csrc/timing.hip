// Optional per-kernel-family timing: when enabled, each launch of an instrumented kernel gets
// a pair of HIP events (attached to the dispatch itself, so they hold the kernel's own start
// and end), and the launcher adds the algorithmic bytes and flops of that launch.  Off by
// default (no events are recorded).  With sampling n > 1, the first launch of each family and
// then about one launch in n, picked by a hash of its call index (so the sample does not lean
// towards the launches at the start of a measured region, or follow a periodic launch pattern),
// is timed (and its bytes and flops added), which keeps the event traffic out of the measured
// region; every call is counted.
// Family names may have a sub-name after '/' (one per launch form, e.g. "dslash/dir"); a query
// for "dslash" sums every "dslash/..." family.
#include <map>
#include <mutex>
#include <string>

#include "timing.hpp"

namespace qmg {

namespace {
struct Family {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double bytes = 0, flops = 0;
  long calls = 0;
};
std::mutex g_mu;
bool g_on = false;
int g_every = 1;
constexpr long kAlwaysTimed = 1;  // the first launch of a family is always timed
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

namespace {
thread_local TimedLaunch* t_current = nullptr;
}

TimedLaunch* TimedLaunch::current() { return t_current; }

TimedLaunch::TimedLaunch(const char* family, hipStream_t st, double bytes, double flops, bool kernel)
    : fam_(family), st_(st), bytes_(bytes), flops_(flops), kernel_(kernel) {
  prev_ = t_current;
  t_current = this;
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st_, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;  // no events in graphs
  std::lock_guard<std::mutex> lk(g_mu);
  const long call = g_fam[fam_].calls++;
  if (g_every > 1 && call >= kAlwaysTimed) {  // sample a pseudo-random 1 / every of the launches
    uint64_t x = uint64_t(call) + 0x9E3779B97F4A7C15ull;  // (no aliasing with periodic launch patterns)
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    if (x % uint64_t(g_every) != 0) return;
  }
  e0_ = get_event();
  e1_ = get_event();
  if (!kernel_) {
    QMG_HIP(hipEventRecord(e0_, st_));
    taken_ = true;
  }
}

bool TimedLaunch::take(hipEvent_t* e0, hipEvent_t* e1) {
  if (!e0_ || taken_ || !kernel_) return false;
  taken_ = true;
  *e0 = e0_;
  *e1 = e1_;
  return true;
}

TimedLaunch::~TimedLaunch() {
  t_current = prev_;
  if (!e0_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!taken_) {  // nothing was launched through qmg::launch: return the events unused
    g_pool.push_back(e0_);
    g_pool.push_back(e1_);
    return;
  }
  if (!kernel_) (void)hipEventRecord(e1_, st_);
  Family& f = g_fam[fam_];
  f.ev.emplace_back(e0_, e1_);
  f.bytes += bytes_;
  f.flops += flops_;
}

void timing_enable(int every) {
  std::lock_guard<std::mutex> lk(g_mu);
  const bool on = every > 0;
  g_every = on ? every : 1;
  for (auto& kv : g_fam)
    for (auto& p : kv.second.ev) {
      g_pool.push_back(p.first);
      g_pool.push_back(p.second);
    }
  g_fam.clear();
  g_on = on;
}

int64_t timing_calls(const char* family) {
  std::lock_guard<std::mutex> lk(g_mu);
  const std::string q(family), pre = q + "/";
  int64_t n = 0;
  for (auto& kv : g_fam)
    if (kv.first == q || kv.first.compare(0, pre.size(), pre) == 0) n += kv.second.calls;
  return n;
}

std::string timing_families() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::string out;
  for (auto& kv : g_fam) {
    if (!out.empty()) out += '\n';
    out += kv.first;
  }
  return out;
}

void timing_query(const char* family, int64_t* n, double* ms, double* bytes, double* flops) {
  std::lock_guard<std::mutex> lk(g_mu);
  *n = 0;
  *ms = 0;
  *bytes = 0;
  *flops = 0;
  const std::string q(family), pre = q + "/";
  for (auto& kv : g_fam) {
    if (kv.first != q && kv.first.compare(0, pre.size(), pre) != 0) continue;
    for (auto& p : kv.second.ev) {
      QMG_HIP(hipEventSynchronize(p.second));
      float t = 0;
      QMG_HIP(hipEventElapsedTime(&t, p.first, p.second));
      *ms += t;
    }
    *n += int64_t(kv.second.ev.size());
    *bytes += kv.second.bytes;
    *flops += kv.second.flops;
  }
}

}  // namespace qmg

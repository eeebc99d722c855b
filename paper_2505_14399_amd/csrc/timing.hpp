// Per-kernel-family launch timing (see timing.hip).
#pragma once

#include <hip/hip_ext.h>

#include <string>

#include "qmg_internal.hpp"

namespace qmg {

bool timing_on();
void timing_enable(int every);  // 0: off; n >= 1: time every n-th launch of each family
void timing_query(const char* family, int64_t* n, double* ms, double* bytes, double* flops);
int64_t timing_calls(const char* family);  // every launch since timing was enabled, timed or not
std::string timing_families();              // newline-separated names of the families launched

// RAII scope around one instrumented launch; events exist only while timing is enabled.
// With kernel = true (default) the pair is attached to the next kernel started through
// qmg::launch() inside the scope, so it holds that dispatch's own start and end timestamps;
// with kernel = false the events are recorded on the stream at scope entry and exit and
// bracket everything launched in between.
class TimedLaunch {
 public:
  TimedLaunch(const char* family, hipStream_t st, double bytes, double flops, bool kernel = true);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;
  // the innermost live scope of this thread, or nullptr
  static TimedLaunch* current();
  // hands out the event pair once (kernel mode); false when there is nothing to attach
  bool take(hipEvent_t* e0, hipEvent_t* e1);

 private:
  const char* fam_;
  hipStream_t st_;
  double bytes_, flops_;
  bool kernel_, taken_ = false;
  hipEvent_t e0_ = nullptr, e1_ = nullptr;
  TimedLaunch* prev_ = nullptr;
};

// kernel<<<grid, block, lds, st>>>(args...), with the events of the enclosing TimedLaunch (if
// any) attached to the dispatch
template <class... KArgs, class... Args>
void launch(void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t lds, hipStream_t st, Args... args) {
  static_assert(sizeof...(KArgs) == sizeof...(Args), "argument count");
  hipEvent_t e0, e1;
  TimedLaunch* tl = TimedLaunch::current();
  if (tl && tl->take(&e0, &e1))
    hipExtLaunchKernelGGL(kernel, grid, block, lds, st, e0, e1, 0u, KArgs(args)...);
  else
    kernel<<<grid, block, lds, st>>>(KArgs(args)...);
}

}  // namespace qmg

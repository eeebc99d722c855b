// Per-kernel-family launch timing (see timing.hip).
#pragma once

#include "qmg_internal.hpp"

namespace qmg {

bool timing_on();
void timing_enable(bool on);
void timing_query(const char* family, int64_t* n, double* ms, double* bytes, double* flops);

// RAII bracket around one kernel launch: events are recorded only while timing is enabled.
class TimedLaunch {
 public:
  TimedLaunch(const char* family, hipStream_t st, double bytes, double flops);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;

 private:
  const char* fam_;
  hipStream_t st_;
  double bytes_, flops_;
  hipEvent_t e0_ = nullptr, e1_ = nullptr;
};

}  // namespace qmg

// Scope guard that brackets one kernel launch with HIP events when timing is on.
#pragma once
#include <hip/hip_runtime.h>

namespace pidk {

class KernelTimer {
 public:
  // Records the start event now and the stop event when destroyed.  With
  // by_launch, nothing is recorded here: the single kernel launch passes
  // start()/stop() to hipExtLaunchKernelGGL, which takes both timestamps
  // from the kernel's own dispatch (no dispatch latency in the interval).
  KernelTimer(const char* name, hipStream_t st, bool by_launch = false);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;
  hipEvent_t start() const { return a_; }   // nullptr when timing is off
  hipEvent_t stop() const { return b_; }

 private:
  const char* name_;
  hipStream_t st_;
  bool by_launch_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace pidk

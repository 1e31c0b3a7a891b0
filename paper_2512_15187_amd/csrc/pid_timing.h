// Scope guard that brackets one kernel launch with HIP events when timing is on.
#pragma once
#include <hip/hip_runtime.h>

namespace pidk {

class KernelTimer {
 public:
  KernelTimer(const char* name, hipStream_t st);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace pidk

// pid_both_static: the combined all-pairs + PID-mean call with its workspace
// in a fixed device array of the library instead of a caller-provided buffer,
// for callers that cannot allocate device memory.  Host code plus the array;
// the kernels are those of pid_both.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pid.h"

namespace pidapi {
pid_status workspace_size(const pid_ensemble*, const pid_iso*, int, int, size_t*);
pid_status run_both(const pid_ensemble*, const pid_iso*, int, const pid_out*, const pid_out*, void*, size_t, void*);
pid_status set_error(pid_status, const char*);
}  // namespace pidapi

namespace {
constexpr size_t kScratchBytes = PID_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace

// One copy per GPU, allocated with the code object when the library is
// loaded on that device and kept until the process ends.  In host code this
// name is only a handle for hipGetSymbolAddress: its device address is
// looked up once per device and used from then on.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device.
pid_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return pidapi::set_error(PID_ERR_DEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return pidapi::set_error(PID_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return pidapi::set_error(PID_ERR_DEVICE, "hipGetSymbolAddress of the static scratch failed");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PID_OK;
}

}  // namespace

extern "C" pid_status pid_both_static(const pid_ensemble* ens, const pid_iso* iso, int gemm,
                                      const pid_out* pairs_out, const pid_out* mean_out, void* stream) {
  size_t need = 0;
  pid_status s = pidapi::workspace_size(ens, iso, 2, gemm, &need);
  if (s != PID_OK) return s;
  if (need > kScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof(msg), "this call needs %zu bytes of workspace; the static scratch holds %zu",
             need, kScratchBytes);
    return pidapi::set_error(PID_ERR_UNSUPPORTED, msg);
  }
  void* ws = nullptr;
  s = scratch_address(&ws);
  if (s != PID_OK) return s;
  return pidapi::run_both(ens, iso, gemm, pairs_out, mean_out, ws, kScratchBytes, stream);
}

// Stand-alone driver for hardware-counter runs (rocprofv3 --pmc), without
// torch: it fills its inputs on the device and runs one of
//   copy [R]   a plain copy of 1 GiB (reads 1 GiB, writes 1 GiB), R times:
//              the calibration of the byte counters;
//   both [R]   pid_both on N = 256 members x M = 262144 points (FP32 masks,
//              FP16 MFMA Gram, inclusion matrix and both rankings), R times.
// It prints one line per mode with the bytes or the status.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/pid.h"

namespace {

// Membership-like values in [0, 1] from a hash of the index (the counters do
// not depend on the values).
__global__ void fill_kernel(float* u, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t h = (uint32_t)i * 2654435761u;
  h ^= h >> 16;
  h *= 2246822519u;
  h ^= h >> 13;
  u[i] = (float)(h >> 8) * (1.0f / 16777216.0f);
}

__global__ void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

bool ok(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return false;
  }
  return true;
}

int run_copy(int reps) {
  const size_t bytes = (size_t)1 << 30, count = bytes / 4;
  float *src = nullptr, *dst = nullptr;
  if (!ok(hipMalloc(&src, bytes), "hipMalloc") || !ok(hipMalloc(&dst, bytes), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, 0, src, count);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, 0, reinterpret_cast<const float4*>(src),
                       reinterpret_cast<float4*>(dst), count / 4);
  if (!ok(hipDeviceSynchronize(), "copy")) return 1;
  printf("copy: %d launches, each reads %zu and writes %zu bytes\n", reps, bytes, bytes);
  hipFree(src);
  hipFree(dst);
  return 0;
}

int run_both(int reps) {
  const int64_t n = 256, m = 262144;
  float* U = nullptr;
  if (!ok(hipMalloc(&U, (size_t)(n * m) * 4), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, 0, U, (size_t)(n * m));
  pid_ensemble e{};
  e.n = n;
  e.m = m;
  e.ld = m;
  e.dtype = PID_F32;
  e.data = U;
  e.weights = nullptr;
  pid_iso iso{};
  iso.kind = PID_ISO_NONE;
  iso.side = 1;
  size_t wsb = 0;
  if (pid_workspace_size(&e, &iso, 2, PID_GEMM_F16, &wsb) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  void* ws = nullptr;
  double* d = nullptr;
  int32_t* r32 = nullptr;
  if (!ok(hipMalloc(&ws, wsb), "hipMalloc") || !ok(hipMalloc(&d, (size_t)(n * n + 8 * n) * 8), "hipMalloc") ||
      !ok(hipMalloc(&r32, (size_t)4 * n * 4), "hipMalloc"))
    return 1;
  pid_out po{d, d + n * n, d + n * n + n, d + n * n + 2 * n, d + n * n + 3 * n, r32, r32 + n};
  pid_out mo{nullptr, d + n * n + 4 * n, d + n * n + 5 * n, d + n * n + 6 * n, d + n * n + 7 * n, r32 + 2 * n,
             r32 + 3 * n};
  for (int r = 0; r < reps; ++r) {
    if (pid_both(&e, &iso, PID_GEMM_F16, &po, &mo, ws, wsb, nullptr) != PID_OK) {
      fprintf(stderr, "pid_both: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "pid_both")) return 1;
  printf("both: %d calls of pid_both, N=%lld M=%lld FP32, FP16 Gram\n", reps, (long long)n, (long long)m);
  hipFree(U);
  hipFree(ws);
  hipFree(d);
  hipFree(r32);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2 || (strcmp(argv[1], "copy") != 0 && strcmp(argv[1], "both") != 0)) {
    fprintf(stderr, "usage: %s copy|both [reps]\n", argv[0]);
    return 2;
  }
  const int reps = argc > 2 ? atoi(argv[2]) : 3;
  if (reps < 1 || reps > 1000) {
    fprintf(stderr, "reps must be 1..1000\n");
    return 2;
  }
  return strcmp(argv[1], "copy") == 0 ? run_copy(reps) : run_both(reps);
}

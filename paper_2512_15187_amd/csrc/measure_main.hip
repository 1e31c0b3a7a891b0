// Stand-alone driver for hardware-counter runs (rocprofv3 --pmc), without
// torch: it fills its inputs on the device and runs one of
//   copy [R]          a plain copy of 1 GiB (reads 1 GiB, writes 1 GiB), R times:
//                     the calibration of the byte counters;
//   both [R] [C]      pid_both on N = 256 members x M = 262144 points (FP32 masks,
//                     FP16 MFMA Gram, inclusion matrix and both rankings), R times,
//                     cycling over C resident copies of the masks (default 4, so
//                     that every call reads them from HBM, not from the cache);
//   fields [R]        the scalar-field workload, N = 128 FP32 fields on 128^3,
//                     isovalue ~ N(0.5, 0.05^2): pid_all_pairs (FP16 MFMA), the
//                     thresholded pid_all_pairs (INT8 MFMA) and pid_mean, R times each;
//   mean3d [R]        pid_mean on N = 64 FP16 masks on 256^3 with FP32 point
//                     weights, R times;
//   bits [R]          binary PID-mean on N = 20000 masks on 50^3 (random 0/1
//                     bytes), as U8 masks and packed by pid_pack_bits, R times each;
//   fieldsbin [R]     PID-mean of the scalar-field workload thresholded at 0.5
//                     (N = 128 FP32 fields on 128^3), R times;
//   peaks [R]         achievable peaks, timed with events (best of R runs): a
//                     copy of 1 GiB, a read of 1 GiB, and a loop of FP16 MFMA
//                     32x32x16 instructions on registers.
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

// Field-like values in [0.3, 0.7) (around the isovalue 0.5).
__global__ void fill_field_kernel(float* u, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t h = (uint32_t)i * 2654435761u + 12345u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  u[i] = 0.3f + 0.4f * (float)(h >> 8) * (1.0f / 16777216.0f);
}

__global__ void fill_half_kernel(_Float16* u, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t h = (uint32_t)i * 2654435761u + 777u;
  h ^= h >> 16;
  h *= 2246822519u;
  u[i] = (_Float16)((float)(h >> 8) * (1.0f / 16777216.0f));
}

// 0/1 bytes from a hash of the index.
__global__ void fill_bits_kernel(uint8_t* u, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t h = (uint32_t)i * 2654435761u + 99u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  u[i] = (uint8_t)((h >> 7) & 1u);
}

// Reads n4 16-byte vectors, grid-strided, and writes one sum per thread.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void read_kernel(const f32x4_t* __restrict__ src, size_t n4, float* __restrict__ out) {
  float s = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    const f32x4_t v = __builtin_nontemporal_load(src + i);
    s += v[0] + v[1] + v[2] + v[3];
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float16_t __attribute__((ext_vector_type(16)));

// Four independent accumulators of v_mfma_f32_32x32x16_f16 per wave, iters
// rounds; one value per thread is written so that nothing is folded away.
__global__ __launch_bounds__(256) void mfma_loop_kernel(float* __restrict__ out, int iters) {
  half8_t a, b;
  for (int k = 0; k < 8; ++k) {
    a[k] = (_Float16)((threadIdx.x + k) & 7);
    b[k] = (_Float16)((threadIdx.x * 3 + k) & 5);
  }
  float16_t c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c3, 0, 0, 0);
  }
  float s = 0.f;
  for (int r = 0; r < 16; ++r) s += c0[r] + c1[r] + c2[r] + c3[r];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
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

pid_ensemble ensemble(int64_t n, int64_t m, int dtype, const void* data, const float* w) {
  pid_ensemble e{};
  e.n = n;
  e.m = m;
  e.ld = m;
  e.dtype = dtype;
  e.data = data;
  e.weights = w;
  return e;
}

struct Outs {
  double* d = nullptr;
  int32_t* r = nullptr;
  pid_out pairs{}, mean{};
  bool alloc(int64_t n) {
    if (!ok(hipMalloc(&d, (size_t)(n * n + 8 * n) * 8), "hipMalloc") || !ok(hipMalloc(&r, (size_t)4 * n * 4), "hipMalloc"))
      return false;
    pairs = pid_out{d, d + n * n, d + n * n + n, d + n * n + 2 * n, d + n * n + 3 * n, r, r + n};
    mean = pid_out{nullptr, d + n * n + 4 * n, d + n * n + 5 * n, d + n * n + 6 * n, d + n * n + 7 * n, r + 2 * n,
                   r + 3 * n};
    return true;
  }
  ~Outs() {
    if (d) hipFree(d);
    if (r) hipFree(r);
  }
};

int run_both(int reps, int copies) {
  const int64_t n = 256, m = 262144;
  float* U = nullptr;
  if (!ok(hipMalloc(&U, (size_t)(n * m) * 4 * copies), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n * m * copies + 255) / 256)), dim3(256), 0, 0, U,
                     (size_t)(n * m * copies));
  pid_iso iso{};
  iso.kind = PID_ISO_NONE;
  iso.side = 1;
  pid_ensemble e0 = ensemble(n, m, PID_F32, U, nullptr);
  size_t wsb = 0;
  if (pid_workspace_size(&e0, &iso, 2, PID_GEMM_F16, &wsb) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  void* ws = nullptr;
  Outs o;
  if (!ok(hipMalloc(&ws, wsb), "hipMalloc") || !o.alloc(n)) return 1;
  for (int r = 0; r < reps; ++r) {
    pid_ensemble e = ensemble(n, m, PID_F32, U + (size_t)(r % copies) * n * m, nullptr);
    if (pid_both(&e, &iso, PID_GEMM_F16, &o.pairs, &o.mean, ws, wsb, nullptr) != PID_OK) {
      fprintf(stderr, "pid_both: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "pid_both")) return 1;
  printf("both: %d calls of pid_both, N=%lld M=%lld FP32, FP16 Gram, %d copies of the masks\n", reps, (long long)n,
         (long long)m, copies);
  hipFree(U);
  hipFree(ws);
  return 0;
}

int run_fields(int reps) {
  const int64_t n = 128, m = 128 * 128 * 128;
  float* F = nullptr;
  if (!ok(hipMalloc(&F, (size_t)(n * m) * 4), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_field_kernel, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, 0, F, (size_t)(n * m));
  pid_ensemble e = ensemble(n, m, PID_F32, F, nullptr);
  pid_iso gauss{PID_ISO_GAUSSIAN, 1, 0.5, 0.05};
  pid_iso step{PID_ISO_STEP, 1, 0.5, 0.0};
  size_t w1 = 0, w2 = 0, w3 = 0;
  if (pid_workspace_size(&e, &gauss, 0, PID_GEMM_F16, &w1) != PID_OK ||
      pid_workspace_size(&e, &step, 0, PID_GEMM_I8, &w2) != PID_OK ||
      pid_workspace_size(&e, &gauss, 1, 0, &w3) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  const size_t wsb = w1 > w2 ? (w1 > w3 ? w1 : w3) : (w2 > w3 ? w2 : w3);
  void* ws = nullptr;
  Outs o;
  if (!ok(hipMalloc(&ws, wsb), "hipMalloc") || !o.alloc(n)) return 1;
  for (int r = 0; r < reps; ++r) {
    if (pid_all_pairs(&e, &gauss, PID_GEMM_F16, &o.pairs, ws, wsb, nullptr) != PID_OK ||
        pid_all_pairs(&e, &step, PID_GEMM_I8, &o.pairs, ws, wsb, nullptr) != PID_OK ||
        pid_mean(&e, &gauss, &o.mean, ws, wsb, nullptr) != PID_OK) {
      fprintf(stderr, "fields: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "fields")) return 1;
  printf("fields: %d x (FP16 all-pairs, INT8 all-pairs, PID-mean), N=%lld M=%lld FP32 fields\n", reps,
         (long long)n, (long long)m);
  hipFree(F);
  hipFree(ws);
  return 0;
}

int run_mean3d(int reps) {
  const int64_t n = 64, m = (int64_t)256 * 256 * 256;
  _Float16* U = nullptr;
  float* w = nullptr;
  if (!ok(hipMalloc(&U, (size_t)(n * m) * 2), "hipMalloc") || !ok(hipMalloc(&w, (size_t)m * 4), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_half_kernel, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, 0, U, (size_t)(n * m));
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, 0, w, (size_t)m);
  pid_ensemble e = ensemble(n, m, PID_F16, U, w);
  pid_iso iso{PID_ISO_NONE, 1, 0.0, 0.0};
  size_t wsb = 0;
  if (pid_workspace_size(&e, &iso, 1, 0, &wsb) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  void* ws = nullptr;
  Outs o;
  if (!ok(hipMalloc(&ws, wsb), "hipMalloc") || !o.alloc(n)) return 1;
  for (int r = 0; r < reps; ++r) {
    if (pid_mean(&e, &iso, &o.mean, ws, wsb, nullptr) != PID_OK) {
      fprintf(stderr, "pid_mean: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "mean3d")) return 1;
  printf("mean3d: %d calls of pid_mean, N=%lld M=%lld FP16 + FP32 weights\n", reps, (long long)n, (long long)m);
  hipFree(U);
  hipFree(w);
  hipFree(ws);
  return 0;
}

int run_bits(int reps) {
  const int64_t n = 20000, m = 125000;
  const int64_t ldp = (m + 127) / 128 * 128;   // packed rows of 16-byte multiples, in points
  uint8_t* U = nullptr;
  uint32_t* P = nullptr;
  if (!ok(hipMalloc(&U, (size_t)(n * m)), "hipMalloc") || !ok(hipMalloc(&P, (size_t)(n * ldp / 8)), "hipMalloc"))
    return 1;
  hipLaunchKernelGGL(fill_bits_kernel, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, 0, U, (size_t)(n * m));
  pid_ensemble e = ensemble(n, m, PID_U8, U, nullptr);
  if (pid_pack_bits(&e, P, ldp, nullptr) != PID_OK) {
    fprintf(stderr, "pid_pack_bits: %s\n", pid_last_error());
    return 1;
  }
  pid_ensemble eb = ensemble(n, m, PID_B1, P, nullptr);
  eb.ld = ldp;
  pid_iso iso{PID_ISO_NONE, 1, 0.0, 0.0};
  size_t w1 = 0, w2 = 0;
  if (pid_workspace_size(&e, &iso, 1, 0, &w1) != PID_OK || pid_workspace_size(&eb, &iso, 1, 0, &w2) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  void* ws = nullptr;
  Outs o;
  if (!ok(hipMalloc(&ws, w1 > w2 ? w1 : w2), "hipMalloc") || !o.alloc(n)) return 1;
  for (int r = 0; r < reps; ++r) {
    if (pid_mean(&e, &iso, &o.mean, ws, w1, nullptr) != PID_OK || pid_mean(&eb, &iso, &o.mean, ws, w2, nullptr) != PID_OK) {
      fprintf(stderr, "pid_mean: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "bits")) return 1;
  printf("bits: %d x (U8, packed) pid_mean, N=%lld M=%lld\n", reps, (long long)n, (long long)m);
  hipFree(U);
  hipFree(P);
  hipFree(ws);
  return 0;
}

int run_fieldsbin(int reps) {
  const int64_t n = 128, m = 128 * 128 * 128;
  float* F = nullptr;
  if (!ok(hipMalloc(&F, (size_t)(n * m) * 4), "hipMalloc")) return 1;
  hipLaunchKernelGGL(fill_field_kernel, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, 0, F, (size_t)(n * m));
  pid_ensemble e = ensemble(n, m, PID_F32, F, nullptr);
  pid_iso step{PID_ISO_STEP, 1, 0.5, 0.0};
  size_t wsb = 0;
  if (pid_workspace_size(&e, &step, 1, 0, &wsb) != PID_OK) {
    fprintf(stderr, "workspace size: %s\n", pid_last_error());
    return 1;
  }
  void* ws = nullptr;
  Outs o;
  if (!ok(hipMalloc(&ws, wsb), "hipMalloc") || !o.alloc(n)) return 1;
  for (int r = 0; r < reps; ++r) {
    if (pid_mean(&e, &step, &o.mean, ws, wsb, nullptr) != PID_OK) {
      fprintf(stderr, "pid_mean: %s\n", pid_last_error());
      return 1;
    }
  }
  if (!ok(hipDeviceSynchronize(), "fieldsbin")) return 1;
  printf("fieldsbin: %d x pid_mean of thresholded fields, N=%lld M=%lld FP32\n", reps, (long long)n, (long long)m);
  hipFree(F);
  hipFree(ws);
  return 0;
}

int run_peaks(int reps) {
  const size_t bytes = (size_t)1 << 30, count = bytes / 4;
  float *src = nullptr, *dst = nullptr, *out = nullptr;
  const int blocks = 256 * 32;
  if (!ok(hipMalloc(&src, bytes), "hipMalloc") || !ok(hipMalloc(&dst, bytes), "hipMalloc") ||
      !ok(hipMalloc(&out, (size_t)blocks * 256 * 4), "hipMalloc"))
    return 1;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, 0, src, count);
  hipEvent_t e0, e1;
  if (!ok(hipEventCreate(&e0), "event") || !ok(hipEventCreate(&e1), "event")) return 1;
  auto best_ms = [&](auto launch) -> float {
    float best = 1e30f;
    for (int r = 0; r < reps + 1; ++r) {   // (the first run warms up)
      hipEventRecord(e0, 0);
      launch();
      hipEventRecord(e1, 0);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (r > 0 && ms < best) best = ms;
    }
    return best;
  };
  const float t_copy = best_ms([&] {
    hipLaunchKernelGGL(copy_kernel, dim3(8192), dim3(256), 0, 0, reinterpret_cast<const float4*>(src),
                       reinterpret_cast<float4*>(dst), count / 4);
  });
  const float t_read = best_ms([&] {
    hipLaunchKernelGGL(read_kernel, dim3(blocks), dim3(256), 0, 0, reinterpret_cast<const f32x4_t*>(src), count / 4, out);
  });
  const int iters = 20000;
  const int mblocks = 256 * 8;   // 4 waves each: 32 waves per CU
  const float t_mfma = best_ms([&] { hipLaunchKernelGGL(mfma_loop_kernel, dim3(mblocks), dim3(256), 0, 0, out, iters); });
  if (!ok(hipDeviceSynchronize(), "peaks")) return 1;
  const double flops = (double)mblocks * 4 * 4 * iters * (2.0 * 32 * 32 * 16);
  printf("peaks: copy %.1f GB/s (read + write of 2^30 B each), read %.1f GB/s, FP16 MFMA %.1f TFLOP/s (best of %d)\n",
         2.0 * bytes / (t_copy * 1e-3) / 1e9, bytes / (t_read * 1e-3) / 1e9, flops / (t_mfma * 1e-3) / 1e12, reps);
  hipFree(src);
  hipFree(dst);
  hipFree(out);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  const char* modes[] = {"copy", "both", "fields", "mean3d", "bits", "fieldsbin", "peaks"};
  int mode = -1;
  for (int k = 0; k < 7; ++k)
    if (argc >= 2 && strcmp(argv[1], modes[k]) == 0) mode = k;
  if (mode < 0) {
    fprintf(stderr, "usage: %s copy|both|fields|mean3d|bits|fieldsbin|peaks [reps] [copies]\n", argv[0]);
    return 2;
  }
  const int reps = argc > 2 ? atoi(argv[2]) : 3;
  const int copies = argc > 3 ? atoi(argv[3]) : 4;
  if (reps < 1 || reps > 1000 || copies < 1 || copies > 8) {
    fprintf(stderr, "reps must be 1..1000, copies 1..8\n");
    return 2;
  }
  switch (mode) {
    case 0: return run_copy(reps);
    case 1: return run_both(reps, copies);
    case 2: return run_fields(reps);
    case 3: return run_mean3d(reps);
    case 4: return run_bits(reps);
    case 5: return run_fieldsbin(reps);
    default: return run_peaks(reps);
  }
}

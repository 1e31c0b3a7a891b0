// Host-only test of the C ABI's argument checks, launch plans and workspace
// sizes over a wide range of shapes (including extreme ones), built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer against the library's
// host sources and stand-in launchers (no GPU, no kernels).  Every call must
// return a status -- an accepted shape a plausible workspace size, a rejected
// one a clean error with its text -- and the sanitizers must stay silent.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/pid.h"

static int g_fail = 0;
#define CHECK(c)                                                                         \
  do {                                                                                   \
    if (!(c)) {                                                                          \
      std::fprintf(stderr, "%s:%d: check failed: %s (last error: %s)\n", __FILE__, __LINE__, #c, \
                   pid_last_error());                                                    \
      ++g_fail;                                                                          \
    }                                                                                    \
  } while (0)

static pid_ensemble ens(int64_t n, int64_t m, int dtype, const void* data = (const void*)0x1000,
                        const float* w = nullptr) {
  pid_ensemble e{};
  e.n = n;
  e.m = m;
  e.ld = m;
  e.dtype = dtype;
  e.flags = 0;
  e.data = data;
  e.weights = w;
  return e;
}

static void rejects() {
  size_t b = 0;
  pid_iso none{PID_ISO_NONE, 1, 0.0, 0.0};
  pid_ensemble e = ens(4, 10, PID_F32);
  struct Case { pid_ensemble e; pid_iso iso; const char* msg; };
  std::vector<Case> cases;
  auto bad = [&](auto f, pid_iso iso, const char* msg) {
    pid_ensemble x = e;
    f(x);
    cases.push_back({x, iso, msg});
  };
  bad([](pid_ensemble& x) { x.n = 0; }, none, "n must be");
  bad([](pid_ensemble& x) { x.n = -5; }, none, "n must be");
  bad([](pid_ensemble& x) { x.m = 0; }, none, "m must be");
  bad([](pid_ensemble& x) { x.ld = 5; }, none, "ld");
  bad([](pid_ensemble& x) { x.dtype = 9; }, none, "unknown dtype");
  bad([](pid_ensemble& x) { x.dtype = -1; }, none, "unknown dtype");
  bad([](pid_ensemble& x) { x.data = nullptr; }, none, "data is NULL");
  bad([](pid_ensemble& x) { x.flags = 8; }, none, "unknown flags");
  bad([](pid_ensemble& x) { x.ld = INT64_MAX; x.m = INT64_MAX; }, none, "overflows");
  bad([](pid_ensemble&) {}, pid_iso{7, 1, 0.5, 0.1}, "unknown iso kind");
  bad([](pid_ensemble&) {}, pid_iso{PID_ISO_GAUSSIAN, 1, 0.5, 0.0}, "sigma");
  bad([](pid_ensemble&) {}, pid_iso{PID_ISO_GAUSSIAN, 1, 0.5, std::nan("")}, "sigma");
  bad([](pid_ensemble&) {}, pid_iso{PID_ISO_GAUSSIAN, 3, 0.5, 0.1}, "side");
  bad([](pid_ensemble&) {}, pid_iso{PID_ISO_STEP, 1, std::nan(""), 0.0}, "finite");
  bad([](pid_ensemble&) {}, pid_iso{PID_ISO_STEP, 1, INFINITY, 0.0}, "finite");
  for (const Case& c : cases) {
    for (int variant = 0; variant < 5; ++variant) {
      const pid_status s = pid_workspace_size(&c.e, &c.iso, variant, PID_GEMM_AUTO, &b);
      CHECK(s == PID_ERR_INVALID_ARG);
      CHECK(std::strstr(pid_last_error(), c.msg) != nullptr);
    }
  }
  CHECK(pid_workspace_size(&e, &none, 5, 0, &b) == PID_ERR_INVALID_ARG);
  CHECK(pid_workspace_size(&e, &none, -1, 0, &b) == PID_ERR_INVALID_ARG);
  CHECK(pid_workspace_size(&e, &none, 0, 42, &b) == PID_ERR_INVALID_ARG);
  CHECK(pid_workspace_size(&e, &none, 0, PID_GEMM_I8, &b) == PID_ERR_INVALID_ARG);   // not binary
  CHECK(pid_workspace_size(&e, &none, 0, 0, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_workspace_size(nullptr, &none, 0, 0, &b) == PID_ERR_INVALID_ARG);
  pid_ensemble bw = ens(4, 10, PID_U8, (const void*)0x1000, (const float*)0x2000);
  CHECK(pid_workspace_size(&bw, &none, 0, PID_GEMM_I8, &b) == PID_ERR_INVALID_ARG);  // weights
  pid_out out{};
  CHECK(pid_all_pairs(nullptr, nullptr, 0, &out, (void*)0x10, 1 << 20, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_all_pairs(&e, nullptr, 0, nullptr, (void*)0x10, 1 << 20, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_all_pairs(&e, nullptr, 0, &out, nullptr, 1 << 20, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_all_pairs(&e, nullptr, 0, &out, (void*)0x10, 16, nullptr) == PID_ERR_WORKSPACE_TOO_SMALL);
  CHECK(pid_mean(&e, nullptr, &out, (void*)0x10, 16, nullptr) == PID_ERR_WORKSPACE_TOO_SMALL);
  CHECK(pid_both(&e, nullptr, 0, nullptr, &out, (void*)0x10, 1 << 20, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_rank(nullptr, 3, nullptr, nullptr, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_rank((const double*)0x10, 0, nullptr, nullptr, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_rank((const double*)0x10, 4, nullptr, nullptr, nullptr) == PID_OK);   // nothing asked for
  CHECK(pid_extract(&e, &none, nullptr, PID_F32, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_extract(&e, &none, (void*)0x10, PID_F16, nullptr) == PID_ERR_INVALID_ARG);
  const int32_t* ord = (const int32_t*)0x10;
  uint8_t* bo = (uint8_t*)0x20;
  CHECK(pid_bands(&e, &none, ord, 0, 4, 0.5, bo, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_bands(&e, &none, ord, 3, 2, 0.5, bo, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_bands(&e, &none, ord, 1, 5, 0.5, bo, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_bands(&e, &none, ord, 1, 4, std::nan(""), bo, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_bands(&e, &none, nullptr, 1, 4, 0.5, bo, nullptr) == PID_ERR_INVALID_ARG);
  // a call whose checks pass reaches the (stand-in) launcher: a device error, not a crash
  size_t need = 0;
  CHECK(pid_workspace_size(&e, &none, 0, 0, &need) == PID_OK);
  CHECK(pid_all_pairs(&e, &none, 0, &out, (void*)0x10, need, nullptr) == PID_ERR_DEVICE);
  for (int s = 0; s <= 9; ++s) CHECK(pid_status_string((pid_status)s) != nullptr);
  CHECK(pid_abi_version() == 3);
}

// Every shape, dtype (bit-packed masks included), model, weighting, variant and
// scheme: a status and, when accepted, a size that covers at least the
// per-member outputs.
static void plans() {
  const int64_t ns[] = {1, 2, 31, 32, 33, 64, 127, 128, 129, 255, 256, 257, 1000, 4096, 20000,
                        32768, 32769, 100000, INT64_C(1) << 22, INT64_C(1) << 30};
  const int64_t ms[] = {1, 2, 7, 16, 1000, 4096, 65537, INT64_C(1) << 20, INT64_C(1) << 24,
                        INT64_C(1) << 28, (INT64_C(1) << 31) + 5, INT64_C(1) << 40};
  const pid_iso isos[] = {{PID_ISO_NONE, 1, 0, 0}, {PID_ISO_GAUSSIAN, 1, 0.5, 0.05}, {PID_ISO_STEP, -1, 0.5, 0},
                          {PID_ISO_RAMP, 1, 0.5, 0.1}, {PID_ISO_TENT, 0, 0.5, 0.1}, {PID_ISO_DENSITY, 0, 2.0, 0}};
  int ok = 0, refused = 0;
  for (int64_t n : ns)
    for (int64_t m : ms)
      for (int dt = 0; dt <= 5; ++dt)
        for (const pid_iso& iso : isos)
          for (int wtd = 0; wtd < 2; ++wtd) {
            pid_ensemble e = ens(n, m, dt, (const void*)0x1000, wtd ? (const float*)0x2000 : nullptr);
            if (dt == PID_B1) e.ld = (m + 31) / 32 * 32;   // bit-packed rows: whole 32-bit words
            for (int variant = 0; variant < 5; ++variant)
              for (int g = 0; g <= 6; ++g) {
                if (variant != 0 && variant != 2 && g) continue;
                size_t b = 0;
                const pid_status s = pid_workspace_size(&e, &iso, variant, g, &b);
                if (s == PID_OK) {
                  ++ok;
                  CHECK(b >= (size_t)n * 8);
                  CHECK(b % 256 == 0);
                } else {
                  ++refused;
                  CHECK(s == PID_ERR_INVALID_ARG || s == PID_ERR_UNSUPPORTED);
                  CHECK(std::strlen(pid_last_error()) > 0);
                }
              }
          }
  CHECK(ok > 1000 && refused > 100);
  std::printf("plans: %d accepted, %d refused\n", ok, refused);

  // FP32 values through the Gaussian model on at most 128 rows: two Gram
  // workgroups per CU, so twice the K-splits (256 CUs without a GPU) and
  // twice the partial sub-tiles (10 of 32 x 32 FP32 for 128 rows) of the
  // same values without a model; 129 rows keep one workgroup per CU
  {
    const pid_iso gauss{PID_ISO_GAUSSIAN, 1, 0.5, 0.05}, none{PID_ISO_NONE, 1, 0, 0};
    const pid_ensemble e128 = ens(128, INT64_C(1) << 21, PID_F32);
    size_t bg = 0, bn = 0;
    CHECK(pid_workspace_size(&e128, &gauss, 0, PID_GEMM_F16, &bg) == PID_OK);
    CHECK(pid_workspace_size(&e128, &none, 0, PID_GEMM_F16, &bn) == PID_OK);
    CHECK(bg >= bn + (size_t)256 * 10 * 4096);
    const pid_ensemble e129 = ens(129, INT64_C(1) << 21, PID_F32);
    CHECK(pid_workspace_size(&e129, &gauss, 0, PID_GEMM_F16, &bg) == PID_OK);
    CHECK(pid_workspace_size(&e129, &none, 0, PID_GEMM_F16, &bn) == PID_OK);
    CHECK(bg == bn);
  }
}

static void server_without_gpu() {
  pid_server* s = nullptr;
  CHECK(pid_server_create(0, nullptr, 1 << 20, 4, &s) == PID_ERR_INVALID_ARG);
  CHECK(pid_server_create(0, (void*)0x1000, 1 << 20, 0, &s) == PID_ERR_INVALID_ARG);
  CHECK(pid_server_create(0, (void*)0x1000, 1 << 20, 65, &s) == PID_ERR_INVALID_ARG);
  CHECK(pid_server_create(0, (void*)0x1000, 1 << 20, 4, nullptr) == PID_ERR_INVALID_ARG);
  const pid_status st = pid_server_create(0, (void*)0x1000, 1 << 20, 4, &s);
  CHECK(st == PID_ERR_DEVICE);                   // no GPU here
  CHECK(pid_submit(nullptr, nullptr, nullptr) == PID_ERR_INVALID_ARG);
  CHECK(pid_release(nullptr, 1) == PID_ERR_INVALID_ARG);
  CHECK(pid_server_destroy(nullptr) == PID_ERR_INVALID_ARG);
}

int main() {
  rejects();
  plans();
  server_without_gpu();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("api checks: all passed\n");
  return 0;
}

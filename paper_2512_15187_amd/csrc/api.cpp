// C ABI of the PID library: argument checks, scheme selection, workspace
// layout and launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/pid.h"
#include "pid_internal.h"

namespace {

thread_local std::string g_last_error;

pid_status fail(pid_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

pid_status hip_fail(hipError_t e, const char* what) {
  return fail(PID_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int elem_bytes(int dtype) {
  switch (dtype) {
    case PID_F64: return 8;
    case PID_F32: return 4;
    case PID_F16: case PID_BF16: return 2;
    case PID_U8: case PID_B1: return 1;   // (B1: an upper bound, for the overflow check)
    default: return 0;
  }
}

pid_status check_ensemble(const pid_ensemble* e, const pid_iso* iso, int* iso_kind) {
  if (!e) return fail(PID_ERR_INVALID_ARG, "ensemble is NULL");
  if (e->n < 1) return fail(PID_ERR_INVALID_ARG, "n must be >= 1 (got %lld)", (long long)e->n);
  if (e->n > (1 << 30)) return fail(PID_ERR_UNSUPPORTED, "n too large (%lld)", (long long)e->n);
  if (e->m < 1) return fail(PID_ERR_INVALID_ARG, "m must be >= 1 (got %lld)", (long long)e->m);
  if (e->ld < e->m) return fail(PID_ERR_INVALID_ARG, "ld (%lld) < m (%lld)", (long long)e->ld, (long long)e->m);
  const int eb = elem_bytes(e->dtype);
  if (eb == 0) return fail(PID_ERR_INVALID_ARG, "unknown dtype %d", e->dtype);
  if (e->ld > (int64_t(1) << 56) / e->n / eb) return fail(PID_ERR_INVALID_ARG, "n * ld overflows");
  if (!e->data) return fail(PID_ERR_INVALID_ARG, "data is NULL");
  if (e->flags & ~PID_FLAG_VALIDATE) return fail(PID_ERR_INVALID_ARG, "unknown flags 0x%x", e->flags);
  if (e->dtype == PID_B1) {
    if (e->ld % 32 != 0) return fail(PID_ERR_INVALID_ARG, "PID_B1 rows: ld (%lld) must be a multiple of 32", (long long)e->ld);
    if ((reinterpret_cast<uintptr_t>(e->data) & 3) != 0) return fail(PID_ERR_INVALID_ARG, "PID_B1 data must be 4-byte aligned");
    if (iso && iso->kind != PID_ISO_NONE) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks take PID_ISO_NONE only");
    if (e->weights) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks take no weights (exact integer sums)");
  }
  int kind = iso ? iso->kind : PID_ISO_NONE;
  if (kind < PID_ISO_NONE || kind > PID_ISO_DENSITY) return fail(PID_ERR_INVALID_ARG, "unknown iso kind %d", kind);
  if (kind != PID_ISO_NONE) {
    const bool sided = kind == PID_ISO_GAUSSIAN || kind == PID_ISO_STEP || kind == PID_ISO_RAMP;
    if (sided && iso->side != 1 && iso->side != -1) return fail(PID_ERR_INVALID_ARG, "iso side must be +1 or -1");
    if (!std::isfinite(iso->c)) return fail(PID_ERR_INVALID_ARG, "iso c must be finite");
    const bool widthed = kind == PID_ISO_GAUSSIAN || kind == PID_ISO_RAMP || kind == PID_ISO_TENT;
    if (widthed && !(iso->sigma > 0.0 && std::isfinite(iso->sigma)))
      return fail(PID_ERR_INVALID_ARG, "iso sigma must be finite and > 0");
    if (kind == PID_ISO_DENSITY && !(iso->c > 0.0))
      return fail(PID_ERR_INVALID_ARG, "iso c (the normalising density) must be > 0");
    if (kind >= PID_ISO_RAMP && e->dtype != PID_F64 && e->dtype != PID_F32 && e->dtype != PID_F16)
      return fail(PID_ERR_UNSUPPORTED, "iso kind %d takes F64, F32 or F16 fields", kind);
  }
  *iso_kind = kind;
  return PID_OK;
}

pidk::ExtractHost make_extract(const pid_iso* iso) {
  pidk::ExtractHost x{};
  if (!iso || iso->kind == PID_ISO_NONE) { x.side = 1; return x; }
  x.side = iso->side;
  x.cd = iso->c;
  x.cf = (float)iso->c;
  if (iso->kind == PID_ISO_GAUSSIAN) {
    x.ad = -(double)iso->side / (iso->sigma * std::sqrt(2.0));
    x.af = (float)x.ad;
  } else if (iso->kind >= PID_ISO_RAMP) {
    // t = (f - c) * a: RAMP a = side / (2 h), TENT a = 1 / h, DENSITY c = 0, a = 1 / c
    x.model = iso->kind;
    if (iso->kind == PID_ISO_RAMP) x.ad = (double)iso->side / (2.0 * iso->sigma);
    else if (iso->kind == PID_ISO_TENT) x.ad = 1.0 / iso->sigma;
    else { x.ad = 1.0 / iso->c; x.cd = 0.0; x.cf = 0.0f; }
    x.af = (float)x.ad;
  }
  // largest float <= c and smallest float >= c (exact comparisons of float fields)
  float cf = (float)iso->c;
  float dn = cf, up = cf;
  if ((double)cf > iso->c) dn = std::nextafter(cf, -INFINITY);
  if ((double)cf < iso->c) up = std::nextafter(cf, INFINITY);
  x.c_dn = dn;
  x.c_up = up;
  return x;
}

bool is_binary_input(const pid_ensemble* e, int kind) {
  return kind == PID_ISO_STEP || (e->dtype == PID_U8 && kind == PID_ISO_NONE);
}

pid_status resolve_scheme(const pid_ensemble* e, int kind, int gemm, int* scheme) {
  const bool bin = is_binary_input(e, kind);
  switch (gemm) {
    case PID_GEMM_AUTO:
      if (bin && !e->weights) *scheme = pidk::SCH_I8;
      else if (e->dtype == PID_F64) *scheme = pidk::SCH_F64;
      else if (e->dtype == PID_BF16) *scheme = pidk::SCH_BF16;
      else *scheme = pidk::SCH_F16;
      return PID_OK;
    case PID_GEMM_F64: *scheme = pidk::SCH_F64; return PID_OK;
    case PID_GEMM_F32: *scheme = pidk::SCH_F32; return PID_OK;
    case PID_GEMM_F16: *scheme = pidk::SCH_F16; return PID_OK;
    case PID_GEMM_BF16: *scheme = pidk::SCH_BF16; return PID_OK;
    case PID_GEMM_BF16_SPLIT: *scheme = pidk::SCH_BF16_SPLIT; return PID_OK;
    case PID_GEMM_I8:
      if (!bin) return fail(PID_ERR_INVALID_ARG, "PID_GEMM_I8 needs binary input (U8 masks or PID_ISO_STEP)");
      if (e->weights) return fail(PID_ERR_INVALID_ARG, "PID_GEMM_I8 is exact only without weights");
      *scheme = pidk::SCH_I8;
      return PID_OK;
    default:
      return fail(PID_ERR_INVALID_ARG, "unknown gemm scheme %d", gemm);
  }
}

// Extra workspace after the kernels' own: depth scratch (for ranks; two
// arrays for the combined call), the validation flag, and the scratch of the
// sorting ranks (more than 2048 members).
size_t extra_bytes(int64_t n, int ndepth = 1) {
  return ((size_t)n * 8 * ndepth + 255) / 256 * 256 + 256 + 256 + (size_t)ndepth * pidk::rank_scratch_bytes(n);
}

struct Extras {
  double* depth;
  unsigned int* flag;
  void* rank_scratch;   // nullptr when the ranks need none
};

Extras carve_extras(void* ws, size_t kernel_bytes, int64_t n, int ndepth = 1) {
  char* base = static_cast<char*>(ws) + ((kernel_bytes + 255) / 256) * 256;
  Extras x;
  x.depth = reinterpret_cast<double*>(base);
  const size_t dbytes = ((size_t)n * 8 * ndepth + 255) / 256 * 256;
  x.flag = reinterpret_cast<unsigned int*>(base + dbytes);
  x.rank_scratch = pidk::rank_scratch_bytes(n) ? base + dbytes + 256 : nullptr;
  return x;
}

pid_status run_validate(const pid_ensemble* e, int kind, unsigned int* flag, hipStream_t st) {
  hipError_t err = pidk::launch_validate(*e, kind, flag, st);
  if (err != hipSuccess) return hip_fail(err, "validate launch");
  err = hipStreamSynchronize(st);
  if (err != hipSuccess) return hip_fail(err, "validate sync");
  unsigned int h = 0;
  err = hipMemcpy(&h, flag, sizeof(h), hipMemcpyDeviceToHost);
  if (err != hipSuccess) return hip_fail(err, "validate copy");
  static const char* what[] = {"", "a probability outside [0,1] or NaN", "a U8 value other than 0/1",
                               "a non-finite field value", "a negative or non-finite weight"};
  if (h) return fail(PID_ERR_VALUE_RANGE, "input holds %s", h < 5 ? what[h] : "an invalid value");
  return PID_OK;
}

}  // namespace

namespace pidk {
int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}
}  // namespace pidk

// Internal entry points shared with the server (same arithmetic as the ABI calls).
namespace pidapi {

pid_status workspace_size(const pid_ensemble* ens, const pid_iso* iso, int variant, int gemm,
                          size_t* bytes) {
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!bytes) return fail(PID_ERR_INVALID_ARG, "bytes is NULL");
  size_t kb = 0;
  if (ens->dtype == PID_B1) {
    if (variant != 1) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks are taken by pid_mean only");
    const pidk::B1Plan p = pidk::b1_plan(ens->n, ens->m);
    if (p.unsupported) return fail(PID_ERR_UNSUPPORTED, "n or m beyond the bit-packed launch limits");
    kb = pidk::b1_workspace(p, ens->n, false);
  } else if (variant == 0) {
    int scheme = 0;
    s = resolve_scheme(ens, kind, gemm, &scheme);
    if (s != PID_OK) return s;
    if (!pidk::pairs_supported(ens->dtype, kind, scheme))
      return fail(PID_ERR_UNSUPPORTED, "scheme %d is not built for dtype %d with iso kind %d", gemm, ens->dtype, kind);
    pidk::PairsPlan p = pidk::pairs_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr, scheme);
    if (p.unsupported)
      return fail(PID_ERR_UNSUPPORTED, "all-pairs of n = %lld, m = %lld is beyond this library's limits "
                  "(n <= 32768; pid_pairs_depths and pid_mean take larger ensembles)",
                  (long long)ens->n, (long long)ens->m);
    kb = pidk::pairs_workspace(p, ens->n);
  } else if (variant == 1) {
    pidk::MeanPlan p = pidk::mean_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr);
    if (p.unsupported)
      return fail(PID_ERR_UNSUPPORTED, "n = %lld is beyond the PID-mean launch limits", (long long)ens->n);
    kb = pidk::mean_workspace(p, ens->n, ens->m);
  } else if (variant == 2) {
    size_t kp = 0;
    s = workspace_size(ens, iso, 0, gemm, &kp);   // the all-pairs pass serves both
    if (s != PID_OK) return s;
    kb = kp;
  } else if (variant == 4) {
    if (pidk::rows_plan(ens->n, ens->m, ens->dtype).unsupported)
      return fail(PID_ERR_UNSUPPORTED, "n = %lld is beyond the PID-mean launch limits", (long long)ens->n);
    kb = pidk::mean_weighted_workspace(ens->n, ens->m, ens->dtype);
  } else if (variant == 3) {
    if (pidk::mean_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr).unsupported ||
        pidk::rows_plan(ens->n, ens->m, ens->dtype).unsupported)
      return fail(PID_ERR_UNSUPPORTED, "n = %lld is beyond the PID-mean launch limits", (long long)ens->n);
    kb = pidk::pairs_linear_workspace(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr);
  } else {
    return fail(PID_ERR_INVALID_ARG, "variant must be 0 (all-pairs), 1 (PID-mean), 2 (both), 3 (all-pairs "
                "depths) or 4 (PID-mean with member weights)");
  }
  *bytes = ((kb + 255) / 256) * 256 + extra_bytes(ens->n, variant == 2 ? 2 : 1);
  return PID_OK;
}

// All-pairs and PID-mean outputs of one ensemble from one all-pairs pass: the
// PID-mean numerators are the Gram row sums.
pid_status run_both(const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* pairs_out,
                    const pid_out* mean_out, void* ws, size_t ws_bytes, void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!pairs_out || !mean_out) return fail(PID_ERR_INVALID_ARG, "pairs_out or mean_out is NULL");
  if (!ws) return fail(PID_ERR_INVALID_ARG, "workspace is NULL");
  size_t need = 0;
  s = workspace_size(ens, iso, 2, gemm, &need);
  if (s != PID_OK) return s;
  if (ws_bytes < need)
    return fail(PID_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Extras x = carve_extras(ws, need - extra_bytes(ens->n, 2), ens->n, 2);
  if (ens->flags & PID_FLAG_VALIDATE) {
    s = run_validate(ens, kind, x.flag, st);
    if (s != PID_OK) return s;
  }
  pid_out po = *pairs_out, mo = *mean_out;
  const bool rank_p = po.rank || po.order, rank_m = mo.rank || mo.order;
  if (rank_p && !po.depth) po.depth = x.depth;
  if (rank_m && !mo.depth) mo.depth = x.depth + ens->n;
  pidk::ExtractHost ex = make_extract(iso);
  int scheme = 0;
  resolve_scheme(ens, kind, gemm, &scheme);
  pidk::PairsPlan p = pidk::pairs_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr, scheme);
  hipError_t err = pidk::launch_pid_pairs(p, *ens, kind, ex, po, ws, st, &mo);
  if (err != hipSuccess) return hip_fail(err, "pid_both launch");
  if (rank_p && rank_m) {
    err = pidk::launch_rank2(po.depth, po.rank, po.order, mo.depth, mo.rank, mo.order, ens->n, st, x.rank_scratch);
    if (err != hipSuccess) return hip_fail(err, "rank launch");
  } else if (rank_p || rank_m) {
    const pid_out& r = rank_p ? po : mo;
    err = pidk::launch_rank(r.depth, ens->n, r.rank, r.order, st, x.rank_scratch);
    if (err != hipSuccess) return hip_fail(err, "rank launch");
  }
  return PID_OK;
}

pid_status run(int variant, const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* out,
               void* ws, size_t ws_bytes, void* stream) {
  if (variant != 0 && variant != 1 && variant != 3) return fail(PID_ERR_INVALID_ARG, "variant must be 0, 1 or 3 here");
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!out) return fail(PID_ERR_INVALID_ARG, "out is NULL");
  if (!ws) return fail(PID_ERR_INVALID_ARG, "workspace is NULL");
  size_t need = 0;
  s = workspace_size(ens, iso, variant, gemm, &need);
  if (s != PID_OK) return s;
  if (ws_bytes < need)
    return fail(PID_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  size_t kb = need - extra_bytes(ens->n);
  Extras x = carve_extras(ws, kb, ens->n);
  if ((ens->flags & PID_FLAG_VALIDATE) && ens->dtype != PID_B1) {   // (every bit is a valid mask value)
    s = run_validate(ens, kind, x.flag, st);
    if (s != PID_OK) return s;
  }
  pid_out o = *out;
  const bool want_rank = o.rank || o.order;
  if (want_rank && !o.depth) o.depth = x.depth;
  pidk::ExtractHost ex = make_extract(iso);
  hipError_t err;
  if (variant == 0) {
    int scheme = 0;
    resolve_scheme(ens, kind, gemm, &scheme);
    pidk::PairsPlan p = pidk::pairs_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr, scheme);
    err = pidk::launch_pid_pairs(p, *ens, kind, ex, o, ws, st);
  } else if (variant == 3) {
    o.inclusion = nullptr;
    err = pidk::launch_pairs_linear(*ens, kind, ex, o, ws, st);
  } else if (ens->dtype == PID_B1) {
    err = pidk::launch_b1_mean(*ens, o, ws, st);
  } else {
    pidk::MeanPlan p = pidk::mean_plan(ens->n, ens->m, ens->dtype, kind, ens->weights != nullptr);
    err = pidk::launch_pid_mean(p, *ens, kind, ex, o, ws, st);
  }
  if (err != hipSuccess)
    return hip_fail(err, variant == 0 ? "pid_all_pairs launch" : (variant == 3 ? "pid_pairs_depths launch" : "pid_mean launch"));
  if (want_rank) {
    err = pidk::launch_rank(o.depth, ens->n, o.rank, o.order, st, x.rank_scratch);
    if (err != hipSuccess) return hip_fail(err, "rank launch");
  }
  return PID_OK;
}

}  // namespace pidapi

extern "C" {

pid_status pid_workspace_size(const pid_ensemble* ens, const pid_iso* iso, int variant, int gemm,
                              size_t* bytes) {
  return pidapi::workspace_size(ens, iso, variant, gemm, bytes);
}

pid_status pid_all_pairs(const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* out,
                         void* workspace, size_t ws_bytes, void* stream) {
  return pidapi::run(0, ens, iso, gemm, out, workspace, ws_bytes, stream);
}

pid_status pid_pairs_depths(const pid_ensemble* ens, const pid_iso* iso, const pid_out* out, void* workspace,
                            size_t ws_bytes, void* stream) {
  return pidapi::run(3, ens, iso, PID_GEMM_AUTO, out, workspace, ws_bytes, stream);
}

pid_status pid_mean(const pid_ensemble* ens, const pid_iso* iso, const pid_out* out, void* workspace,
                    size_t ws_bytes, void* stream) {
  return pidapi::run(1, ens, iso, PID_GEMM_AUTO, out, workspace, ws_bytes, stream);
}

pid_status pid_both(const pid_ensemble* ens, const pid_iso* iso, int gemm, const pid_out* pairs_out,
                    const pid_out* mean_out, void* workspace, size_t ws_bytes, void* stream) {
  return pidapi::run_both(ens, iso, gemm, pairs_out, mean_out, workspace, ws_bytes, stream);
}

pid_status pid_mean_weighted(const pid_ensemble* ens, const pid_iso* iso, const double* member_w, const pid_out* out,
                             void* workspace, size_t ws_bytes, void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!member_w) return fail(PID_ERR_INVALID_ARG, "member_w is NULL");
  if (!out) return fail(PID_ERR_INVALID_ARG, "out is NULL");
  if (!workspace) return fail(PID_ERR_INVALID_ARG, "workspace is NULL");
  size_t need = 0;
  s = pidapi::workspace_size(ens, iso, 4, PID_GEMM_AUTO, &need);
  if (s != PID_OK) return s;
  if (ws_bytes < need)
    return fail(PID_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Extras x = carve_extras(workspace, need - extra_bytes(ens->n), ens->n);
  if (ens->flags & PID_FLAG_VALIDATE) {
    s = run_validate(ens, kind, x.flag, st);
    if (s != PID_OK) return s;
  }
  pid_out o = *out;
  o.inclusion = nullptr;
  const bool want_rank = o.rank || o.order;
  if (want_rank && !o.depth) o.depth = x.depth;
  hipError_t err = pidk::launch_pid_mean_weighted(*ens, kind, make_extract(iso), member_w, o, workspace, st);
  if (err != hipSuccess) return hip_fail(err, "pid_mean_weighted launch");
  if (want_rank) {
    err = pidk::launch_rank(o.depth, ens->n, o.rank, o.order, st, x.rank_scratch);
    if (err != hipSuccess) return hip_fail(err, "rank launch");
  }
  return PID_OK;
}

pid_status pid_pack_bits(const pid_ensemble* ens, void* out, int64_t out_ld, void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, nullptr, &kind);
  if (s != PID_OK) return s;
  if (ens->dtype != PID_U8) return fail(PID_ERR_INVALID_ARG, "pid_pack_bits packs PID_U8 masks");
  if (!out) return fail(PID_ERR_INVALID_ARG, "out is NULL");
  if ((reinterpret_cast<uintptr_t>(out) & 3) != 0) return fail(PID_ERR_INVALID_ARG, "out must be 4-byte aligned");
  if (out_ld < ens->m || out_ld % 32 != 0)
    return fail(PID_ERR_INVALID_ARG, "out_ld (%lld) must be a multiple of 32 and >= m", (long long)out_ld);
  if ((ens->n + 15) / 16 > 65535 || (ens->m + 2047) / 2048 / 4 >= INT32_MAX)
    return fail(PID_ERR_UNSUPPORTED, "n or m beyond the packing launch limits");
  hipError_t err = pidk::launch_pack_bits(*ens, static_cast<uint32_t*>(out), out_ld / 32,
                                          reinterpret_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "pid_pack_bits launch");
  return PID_OK;
}

pid_status pid_field_max(const pid_ensemble* ens, double* max_out, void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, nullptr, &kind);
  if (s != PID_OK) return s;
  if (!max_out) return fail(PID_ERR_INVALID_ARG, "max_out is NULL");
  if (ens->dtype == PID_B1) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks are taken by pid_mean only");
  if ((reinterpret_cast<uintptr_t>(max_out) & 7) != 0) return fail(PID_ERR_INVALID_ARG, "max_out must be 8-byte aligned");
  hipError_t err = pidk::launch_field_max(*ens, max_out, reinterpret_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "pid_field_max launch");
  return PID_OK;
}

pid_status pid_extract(const pid_ensemble* ens, const pid_iso* iso, void* u_out, int out_dtype,
                       void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!u_out) return fail(PID_ERR_INVALID_ARG, "u_out is NULL");
  if (ens->dtype == PID_B1) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks are taken by pid_mean only");
  if (out_dtype != PID_F32 && out_dtype != PID_F64)
    return fail(PID_ERR_INVALID_ARG, "out_dtype must be PID_F32 or PID_F64");
  hipError_t err = pidk::launch_extract(*ens, kind, make_extract(iso), u_out, out_dtype,
                                        reinterpret_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "pid_extract launch");
  return PID_OK;
}

pid_status pid_bands(const pid_ensemble* ens, const pid_iso* iso, const int32_t* order, int64_t k_inner,
                     int64_t k_outer, double threshold, uint8_t* out, void* stream) {
  int kind = 0;
  pid_status s = check_ensemble(ens, iso, &kind);
  if (s != PID_OK) return s;
  if (!order) return fail(PID_ERR_INVALID_ARG, "order is NULL");
  if (ens->dtype == PID_B1) return fail(PID_ERR_UNSUPPORTED, "PID_B1 masks are taken by pid_mean only");
  if (!out) return fail(PID_ERR_INVALID_ARG, "out is NULL");
  if (k_inner < 1 || k_inner > k_outer || k_outer > ens->n)
    return fail(PID_ERR_INVALID_ARG, "need 1 <= k_inner <= k_outer <= n (got %lld, %lld, n = %lld)",
                (long long)k_inner, (long long)k_outer, (long long)ens->n);
  if (!std::isfinite(threshold)) return fail(PID_ERR_INVALID_ARG, "threshold must be finite");
  const int eb = elem_bytes(ens->dtype);
  if ((ens->m + 16 / eb - 1) / (16 / eb) > (int64_t)64 * 0x7fffffff)
    return fail(PID_ERR_UNSUPPORTED, "m too large (%lld)", (long long)ens->m);
  hipError_t err = pidk::launch_bands(*ens, kind, make_extract(iso), order, k_inner, k_outer, threshold, out,
                                      reinterpret_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "pid_bands launch");
  return PID_OK;
}

pid_status pid_rank(const double* depth, int64_t n, int32_t* rank, int32_t* order, void* stream) {
  if (!depth) return fail(PID_ERR_INVALID_ARG, "depth is NULL");
  if (n < 1 || n > (1 << 30)) return fail(PID_ERR_INVALID_ARG, "bad n %lld", (long long)n);
  if (!rank && !order) return PID_OK;
  hipError_t err = pidk::launch_rank(depth, n, rank, order, reinterpret_cast<hipStream_t>(stream));
  if (err != hipSuccess) return hip_fail(err, "pid_rank launch");
  return PID_OK;
}

const char* pid_status_string(pid_status s) {
  switch (s) {
    case PID_OK: return "PID_OK";
    case PID_ERR_INVALID_ARG: return "PID_ERR_INVALID_ARG";
    case PID_ERR_UNSUPPORTED: return "PID_ERR_UNSUPPORTED";
    case PID_ERR_WORKSPACE_TOO_SMALL: return "PID_ERR_WORKSPACE_TOO_SMALL";
    case PID_ERR_DEVICE: return "PID_ERR_DEVICE";
    case PID_ERR_VALUE_RANGE: return "PID_ERR_VALUE_RANGE";
    case PID_ERR_OVER_BUDGET: return "PID_ERR_OVER_BUDGET";
    case PID_ERR_CANCELLED: return "PID_ERR_CANCELLED";
    case PID_ERR_INTERNAL: return "PID_ERR_INTERNAL";
    default: return "PID_ERR_UNKNOWN";
  }
}

const char* pid_last_error(void) { return g_last_error.c_str(); }

int pid_abi_version(void) { return 3; }

}  // extern "C"

// Used by the server to record its own errors in the calling thread's slot.
namespace pidapi {
pid_status set_error(pid_status s, const char* msg) { return fail(s, "%s", msg); }
}  // namespace pidapi

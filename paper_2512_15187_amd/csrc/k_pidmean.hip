// PID-mean (Sec. 4.1) as one streaming pass over the ensemble.
//
// Both inclusions of PID-mean share the numerator
//     A_i = sum_x w_x u_i(x) s(x),   s(x) = sum_j u_j(x)   (= N * sum_x w u_i ubar),
// and the denominators are the masses m_i = sum_x w u_i and
// m(ubar) = (1/N) sum_k m_k.  Hence IN_in = A_i / (N m_i) and
// IN_out = A_i / sum_k m_k, and the ensemble has to be read once only: a
// workgroup owns a tile of points and all N members.  Each wave loads a slice
// of the members with 16-byte loads, applies the isovalue model in registers,
// and writes its partial column sums to LDS; after one barrier every lane holds
// s(x) for its points and accumulates m_i and A_i for the members it loaded.
// Per tile the sums are FP32 (FP64 for FP64 input), across tiles FP64; binary
// input uses exact integers throughout.  Per-workgroup partials are reduced
// in a fixed order by pidmean_finalize.
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <type_traits>

namespace pidk {

template <typename T>
using ComputeT = typename std::conditional<sizeof(T) == 8, double, float>::type;

template <int MODE, typename T, typename CT>
__device__ __forceinline__ CT extract_ct(T raw, const Extract& e) {
  if constexpr (std::is_same<CT, double>::value) return extract_d<MODE>(raw, e);
  else return extract_f<MODE>(raw, e);
}

// ---------------------------------------------------------------------------
// Soft path.  SFROM: column sums are read from `sglob` (two-pass mode) and the
// member range of this workgroup is blockIdx.y * nwaves * MPW + ...
// part layout: [grid.x][2][n] doubles (m, A).
template <typename T, int MODE, int MPW, bool WEIGHTED, bool SFROM>
__global__ __launch_bounds__(1024) void pidmean_soft_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, const float* __restrict__ w,
    Extract ex, int64_t ntiles, const void* __restrict__ sglob, double* __restrict__ part, int vec) {
  const bool VEC = vec != 0;
  using CT = ComputeT<T>;
  constexpr int PPL = Vec16<T>::N;
  constexpr int TP = 64 * PPL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CT* sbuf = reinterpret_cast<CT*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int mbase = (SFROM ? blockIdx.y * nw * MPW : 0) + wave * MPW;

  double accm[MPW], acca[MPW];
#pragma unroll
  for (int r = 0; r < MPW; ++r) { accm[r] = 0.0; acca[r] = 0.0; }

  int it = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
    const int64_t x0 = tile * TP + (int64_t)lane * PPL;
    const bool full = (x0 + PPL <= m);
    CT u[MPW][PPL];
    CT sp[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) sp[p] = CT(0);
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const int i = mbase + r;
      if (i < n) {
        const T* row = U + (int64_t)i * ld;
        Vec16<T> v;
        if (VEC && full) v = load16_nt(row + x0);
        else v = load16_guarded(row, x0, m);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          CT val = extract_ct<MODE, T, CT>(v.v[p], ex);
          if (MODE != MODE_NONE && !full) val = (x0 + p < m) ? val : CT(0);
          u[r][p] = val;
          sp[p] += val;
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) u[r][p] = CT(0);
      }
    }

    CT s[PPL];
    if constexpr (SFROM) {
      const CT* sg = reinterpret_cast<const CT*>(sglob);
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] = (x0 + p < m) ? sg[x0 + p] : CT(0);
    } else {
      CT* sb = sbuf + (size_t)(it & 1) * nw * TP;
#pragma unroll
      for (int p = 0; p < PPL; ++p) sb[wave * TP + lane * PPL + p] = sp[p];
      __syncthreads();
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] = CT(0);
      for (int q = 0; q < nw; ++q) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) s[p] += sb[q * TP + lane * PPL + p];
      }
    }

    CT wv[PPL];
    if constexpr (WEIGHTED) {
      if (PPL >= 4 && full && VEC) {
#pragma unroll
        for (int p = 0; p < PPL; p += 4) {
          float4 t = *reinterpret_cast<const float4*>(w + x0 + p);
          wv[p] = t.x; if (p + 1 < PPL) wv[p + 1] = t.y;
          if (p + 2 < PPL) wv[p + 2] = t.z; if (p + 3 < PPL) wv[p + 3] = t.w;
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) wv[p] = (x0 + p < m) ? CT(w[x0 + p]) : CT(0);
      }
    }
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      CT tm = CT(0), ta = CT(0);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        CT wu = WEIGHTED ? wv[p] * u[r][p] : u[r][p];
        tm += wu;
        ta += wu * s[p];
      }
      accm[r] += (double)tm;
      acca[r] += (double)ta;
    }
  }

#pragma unroll
  for (int r = 0; r < MPW; ++r) {
    const double a = wave_sum(accm[r]);
    const double b = wave_sum(acca[r]);
    const int i = mbase + r;
    if (lane == 0 && i < n) {
      part[((size_t)blockIdx.x * 2 + 0) * n + i] = a;
      part[((size_t)blockIdx.x * 2 + 1) * n + i] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// Binary path (U8 masks, or STEP on fields), exact integers.
// part layout: [grid.x][2][n] long long (m, S).
template <typename T, int MODE, int MPW, bool SFROM>
__global__ __launch_bounds__(1024) void pidmean_bin_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, Extract ex, int64_t ntiles,
    const int* __restrict__ sglob, long long* __restrict__ part, int vec) {
  const bool VEC = vec != 0;
  constexpr int PPL = Vec16<T>::N;
  constexpr int TP = 64 * PPL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* sbuf = reinterpret_cast<int*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int mbase = (SFROM ? blockIdx.y * nw * MPW : 0) + wave * MPW;

  long long accm[MPW], acca[MPW];
#pragma unroll
  for (int r = 0; r < MPW; ++r) { accm[r] = 0; acca[r] = 0; }

  int it = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
    const int64_t x0 = tile * TP + (int64_t)lane * PPL;
    const bool full = (x0 + PPL <= m);
    // u8 masks stay packed (4 dwords per member); other inputs become bits.
    constexpr bool PACKED = (sizeof(T) == 1 && MODE == MODE_NONE);
    uint32_t raw[MPW][4];
    int ub[MPW][PACKED ? 1 : PPL];
    int sp[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) sp[p] = 0;
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const int i = mbase + r;
      Vec16<T> v{};
      if (i < n) {
        const T* row = U + (int64_t)i * ld;
        if (VEC && full) v = load16_nt(row + x0);
        else v = load16_guarded(row, x0, m);
      }
      if constexpr (PACKED) {
        uint4 q = __builtin_bit_cast(uint4, v);
        raw[r][0] = q.x; raw[r][1] = q.y; raw[r][2] = q.z; raw[r][3] = q.w;
#pragma unroll
        for (int p = 0; p < PPL; ++p) sp[p] += (raw[r][p >> 2] >> (8 * (p & 3))) & 0xffu;
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          int b = (i < n) ? extract_bit<MODE>(v.v[p], ex) : 0;
          if (!full) b = (x0 + p < m) ? b : 0;
          ub[r][p] = b;
          sp[p] += b;
        }
      }
    }

    int s[PPL];
    if constexpr (SFROM) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] = (x0 + p < m) ? sglob[x0 + p] : 0;
    } else {
      int* sb = sbuf + (size_t)(it & 1) * nw * TP;
#pragma unroll
      for (int p = 0; p < PPL; ++p) sb[wave * TP + lane * PPL + p] = sp[p];
      __syncthreads();
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] = 0;
      for (int q = 0; q < nw; ++q) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) s[p] += sb[q * TP + lane * PPL + p];
      }
    }

#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      int tm = 0, ta = 0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        int b;
        if constexpr (PACKED) b = (raw[r][p >> 2] >> (8 * (p & 3))) & 0xffu;
        else b = ub[r][p];
        tm += b;
        ta += b * s[p];
      }
      accm[r] += tm;
      acca[r] += ta;
    }
  }

#pragma unroll
  for (int r = 0; r < MPW; ++r) {
    const long long a = wave_sum(accm[r]);
    const long long b = wave_sum(acca[r]);
    const int i = mbase + r;
    if (lane == 0 && i < n) {
      part[((size_t)blockIdx.x * 2 + 0) * n + i] = a;
      part[((size_t)blockIdx.x * 2 + 1) * n + i] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// Column sums s(x) for the two-pass case (N larger than one workgroup holds).
template <typename T, int MODE, bool BIN>
__global__ __launch_bounds__(256) void colsum_kernel(const T* __restrict__ U, int64_t ld, int n,
                                                     int64_t m, Extract ex, void* __restrict__ sout) {
  using CT = ComputeT<T>;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m;
       x += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (BIN) {
      int s = 0;
      for (int i = 0; i < n; ++i) s += extract_bit<MODE>(U[(int64_t)i * ld + x], ex);
      reinterpret_cast<int*>(sout)[x] = s;
    } else {
      CT s = CT(0);
      for (int i = 0; i < n; ++i) s += extract_ct<MODE, T, CT>(U[(int64_t)i * ld + x], ex);
      reinterpret_cast<CT*>(sout)[x] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the per-workgroup partials and the depth ratios.
// One workgroup of 256 threads.
template <bool BIN>
__global__ __launch_bounds__(256) void pidmean_finalize(const void* __restrict__ part_v, int nparts,
                                                        int n, double* __restrict__ m_out,
                                                        double* __restrict__ in_in,
                                                        double* __restrict__ in_out,
                                                        double* __restrict__ depth,
                                                        void* __restrict__ scratch) {
#pragma clang fp contract(off)
  __shared__ double red_d[256];
  __shared__ long long red_i[256];
  const int t = threadIdx.x;
  double* Ad = reinterpret_cast<double*>(scratch);            // n
  long long* Ai = reinterpret_cast<long long*>(scratch);      // n (binary)
  double* Md = Ad + n;
  long long* Mi = Ai + n;
  double md_loc = 0.0;
  long long mi_loc = 0;
  for (int i = t; i < n; i += 256) {
    if constexpr (BIN) {
      const long long* part = reinterpret_cast<const long long*>(part_v);
      long long mm = 0, aa = 0;
      for (int b = 0; b < nparts; ++b) {
        mm += part[((size_t)b * 2 + 0) * n + i];
        aa += part[((size_t)b * 2 + 1) * n + i];
      }
      Mi[i] = mm; Ai[i] = aa; mi_loc += mm;
    } else {
      const double* part = reinterpret_cast<const double*>(part_v);
      double mm = 0.0, aa = 0.0;
      for (int b = 0; b < nparts; ++b) {
        mm += part[((size_t)b * 2 + 0) * n + i];
        aa += part[((size_t)b * 2 + 1) * n + i];
      }
      Md[i] = mm; Ad[i] = aa; md_loc += mm;
    }
  }
  red_d[t] = md_loc;
  red_i[t] = mi_loc;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) { red_d[t] += red_d[t + o]; red_i[t] += red_i[t + o]; }
    __syncthreads();
  }
  for (int i = t; i < n; i += 256) {
    double mi, a, tot, ii, oo;
    if constexpr (BIN) {
      mi = (double)Mi[i]; a = (double)Ai[i]; tot = (double)red_i[0];
    } else {
      mi = Md[i]; a = Ad[i]; tot = red_d[0];
    }
    ii = (mi > 0.0) ? a / ((double)n * mi) : 0.0;
    oo = (tot > 0.0) ? a / tot : 0.0;
    if (m_out) m_out[i] = mi;
    if (in_in) in_in[i] = ii;
    if (in_out) in_out[i] = oo;
    if (depth) depth[i] = ii < oo ? ii : oo;
  }
}

// ---------------------------------------------------------------------------
// Host side: plan, workspace and launch.

static int elem_bytes(int dtype) {
  switch (dtype) {
    case PID_F64: return 8;
    case PID_F32: return 4;
    case PID_F16: case PID_BF16: return 2;
    default: return 1;
  }
}

static bool is_binary(int dtype, int iso_kind, bool weighted) {
  if (weighted) return false;
  return iso_kind == PID_ISO_STEP || (dtype == PID_U8 && iso_kind == PID_ISO_NONE);
}

MeanPlan mean_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted) {
  MeanPlan p{};
  p.binary = is_binary(dtype, iso_kind, weighted) ? 1 : 0;
  const int eb = elem_bytes(dtype);
  const int ppl = 16 / eb;
  const int tp = 64 * ppl;
  // members per wave: up to 8 waves with the smallest slice that covers N,
  // then up to 16 waves with 16 members each (N <= 256); beyond: two passes.
  int mpw = 4;
  if (n > 32) mpw = 8;
  if (n > 64) mpw = 16;
  if (eb == 1 && mpw > 8) mpw = 8;          // 16 points per lane: keep registers in check
  int nw = (int)((n + mpw - 1) / mpw);
  const int max_waves = 16;
  p.two_pass = 0;
  p.groups = 1;
  if (nw > max_waves) {
    p.two_pass = 1;
    nw = 8;
    p.groups = (int)((n + (int64_t)nw * mpw - 1) / ((int64_t)nw * mpw));
  }
  p.mpw = mpw;
  p.nwaves = nw;
  p.ntiles = (m + tp - 1) / tp;
  // about eight resident workgroups' worth of waves per CU, capped by the tiles
  int target = device_cu_count() * std::max(1, 32 / nw);
  if (p.two_pass) target = std::max(1, device_cu_count() * 4 / p.groups);
  p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, target));
  const int cb = p.binary ? 4 : (dtype == PID_F64 ? 8 : 4);
  p.lds_bytes = p.two_pass ? 0 : (size_t)2 * nw * tp * cb;
  return p;
}

size_t mean_workspace(const MeanPlan& p, int64_t n, int64_t m) {
  Carve c(nullptr);
  c.take<double>((size_t)p.grid * 2 * n);   // partials (double or long long)
  c.take<double>((size_t)2 * n);            // reduced A and m
  if (p.two_pass) c.take<double>((size_t)m);  // column sums
  return c.off + 256;
}

template <typename T, int MODE, int MPW>
static void launch_soft_t(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                          const void* sglob, double* part, hipStream_t st) {
  dim3 grid(p.grid, p.two_pass ? p.groups : 1);
  dim3 block(64 * p.nwaves);
  const T* U = reinterpret_cast<const T*>(e.data);
  const bool wtd = e.weights != nullptr;
  KernelTimer tm("pidmean", st);
#define PM_LAUNCH(W, S)                                                                       \
  hipLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, W, S>), grid, block, p.lds_bytes, st, U, \
                     e.ld, (int)e.n, e.m, e.weights, ex, p.ntiles, sglob, part, vec ? 1 : 0)
  if (p.two_pass) { if (wtd) PM_LAUNCH(true, true); else PM_LAUNCH(false, true); }
  else { if (wtd) PM_LAUNCH(true, false); else PM_LAUNCH(false, false); }
#undef PM_LAUNCH
}

template <typename T, int MODE, int MPW>
static void launch_bin_t(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                         const int* sglob, long long* part, hipStream_t st) {
  dim3 grid(p.grid, p.two_pass ? p.groups : 1);
  dim3 block(64 * p.nwaves);
  const T* U = reinterpret_cast<const T*>(e.data);
  KernelTimer tm("pidmean", st);
#define PB_LAUNCH(S)                                                                  \
  hipLaunchKernelGGL((pidmean_bin_kernel<T, MODE, MPW, S>), grid, block, p.lds_bytes, st, U, \
                     e.ld, (int)e.n, e.m, ex, p.ntiles, sglob, part, vec ? 1 : 0)
  if (p.two_pass) PB_LAUNCH(true); else PB_LAUNCH(false);
#undef PB_LAUNCH
}

template <typename T, int MODE>
static void dispatch_mpw(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                         const void* sglob, void* part, hipStream_t st) {
  if (p.binary) {
    if constexpr (MODE != MODE_GAUSS) {
      switch (p.mpw) {
        case 4: launch_bin_t<T, MODE, 4>(p, e, ex, vec, (const int*)sglob, (long long*)part, st); break;
        case 8: launch_bin_t<T, MODE, 8>(p, e, ex, vec, (const int*)sglob, (long long*)part, st); break;
        default: launch_bin_t<T, MODE, 16>(p, e, ex, vec, (const int*)sglob, (long long*)part, st); break;
      }
    }
  } else {
    switch (p.mpw) {
      case 4: launch_soft_t<T, MODE, 4>(p, e, ex, vec, sglob, (double*)part, st); break;
      case 8: launch_soft_t<T, MODE, 8>(p, e, ex, vec, sglob, (double*)part, st); break;
      default: launch_soft_t<T, MODE, 16>(p, e, ex, vec, sglob, (double*)part, st); break;
    }
  }
}

template <typename T>
static void dispatch_mode(const MeanPlan& p, const pid_ensemble& e, int iso_kind, const Extract& ex,
                          bool vec, const void* sglob, void* part, hipStream_t st) {
  switch (iso_kind) {
    case PID_ISO_GAUSSIAN: dispatch_mpw<T, MODE_GAUSS>(p, e, ex, vec, sglob, part, st); break;
    case PID_ISO_STEP: dispatch_mpw<T, MODE_STEP>(p, e, ex, vec, sglob, part, st); break;
    default: dispatch_mpw<T, MODE_NONE>(p, e, ex, vec, sglob, part, st); break;
  }
}

template <typename T>
static void launch_colsum(const MeanPlan& p, const pid_ensemble& e, int iso_kind, const Extract& ex,
                          void* sout, hipStream_t st) {
  const T* U = reinterpret_cast<const T*>(e.data);
  int grid = (int)std::min<int64_t>((e.m + 255) / 256, device_cu_count() * 8);
  KernelTimer tm("pidmean_colsum", st);
  if (p.binary) {
    if (iso_kind == PID_ISO_STEP)
      hipLaunchKernelGGL((colsum_kernel<T, MODE_STEP, true>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex, sout);
    else
      hipLaunchKernelGGL((colsum_kernel<T, MODE_NONE, true>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex, sout);
  } else if (iso_kind == PID_ISO_GAUSSIAN) {
    hipLaunchKernelGGL((colsum_kernel<T, MODE_GAUSS, false>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex, sout);
  } else if (iso_kind == PID_ISO_STEP) {
    hipLaunchKernelGGL((colsum_kernel<T, MODE_STEP, false>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex, sout);
  } else {
    hipLaunchKernelGGL((colsum_kernel<T, MODE_NONE, false>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex, sout);
  }
}

hipError_t launch_pid_mean(const MeanPlan& p, const pid_ensemble& e, int iso_kind,
                           const ExtractHost& exh, const pid_out& out, void* ws, hipStream_t st) {
  Extract ex = __builtin_bit_cast(Extract, exh);
  Carve c(ws);
  void* part = c.take<double>((size_t)p.grid * 2 * e.n);
  void* red = c.take<double>((size_t)2 * e.n);
  void* sbuf = p.two_pass ? (void*)c.take<double>((size_t)e.m) : nullptr;
  const int eb = elem_bytes(e.dtype);
  const bool vec = ((reinterpret_cast<uintptr_t>(e.data) & 15) == 0) && ((e.ld * eb) % 16 == 0) &&
                   (e.weights == nullptr || (reinterpret_cast<uintptr_t>(e.weights) & 15) == 0);
  switch (e.dtype) {
    case PID_F64:
      if (p.two_pass) launch_colsum<double>(p, e, iso_kind, ex, sbuf, st);
      dispatch_mode<double>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_F32:
      if (p.two_pass) launch_colsum<float>(p, e, iso_kind, ex, sbuf, st);
      dispatch_mode<float>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_F16:
      if (p.two_pass) launch_colsum<f16>(p, e, iso_kind, ex, sbuf, st);
      dispatch_mode<f16>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_BF16:
      if (p.two_pass) launch_colsum<bf16_t>(p, e, iso_kind, ex, sbuf, st);
      dispatch_mode<bf16_t>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    default:
      if (p.two_pass) launch_colsum<uint8_t>(p, e, iso_kind, ex, sbuf, st);
      dispatch_mode<uint8_t>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  KernelTimer tm("pidmean_finalize", st);
  if (p.binary)
    hipLaunchKernelGGL(pidmean_finalize<true>, 1, 256, 0, st, part, p.grid, (int)e.n, out.mass,
                       out.in_in, out.in_out, out.depth, red);
  else
    hipLaunchKernelGGL(pidmean_finalize<false>, 1, 256, 0, st, part, p.grid, (int)e.n, out.mass,
                       out.in_in, out.in_out, out.depth, red);
  return hipGetLastError();
}

}  // namespace pidk

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
// in a fixed order by pidmean_reduce, and pidmean_ratios forms the depths.
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <cstdlib>
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
// A workgroup handles at most a few tens of tiles, so per-lane FP32 sums stay
// short; lanes are combined in FP64.  Soft masks (MODE_NONE) keep only the
// raw 16-byte vectors in registers and widen them again in the second phase;
// fields keep the extracted probabilities.
// part layout: [2][n][grid.x] doubles (m, then A).
template <typename T, int MODE, int MPW, bool WEIGHTED, bool SFROM, int NWMAX>
__global__ __launch_bounds__(64 * NWMAX) void pidmean_soft_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, const float* __restrict__ w,
    Extract ex, int64_t ntiles, const void* __restrict__ sglob, double* __restrict__ part, int vec) {
  using CT = ComputeT<T>;
  constexpr int PPL = Vec16<T>::N;
  constexpr int TP = 64 * PPL;
  constexpr bool KEEP_RAW = (MODE == MODE_NONE);
  const bool VEC = vec != 0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CT* sbuf = reinterpret_cast<CT*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int nw = blockDim.x >> 6;
  const int mbase = (SFROM ? blockIdx.y * nw * MPW : 0) + wave * MPW;

  CT accm[MPW], acca[MPW];
#pragma unroll
  for (int r = 0; r < MPW; ++r) { accm[r] = CT(0); acca[r] = CT(0); }

  int it = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
    const int64_t x0 = tile * TP + (int64_t)lane * PPL;
    const bool full = (x0 + PPL <= m);
    Vec16<T> raw[KEEP_RAW ? MPW : 1];
    CT u[KEEP_RAW ? 1 : MPW][PPL];
    CT sp[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) sp[p] = CT(0);
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const int i = mbase + r;
      Vec16<T> v{};
      if (i < n) {
        const T* row = U + (int64_t)i * ld;
        if (VEC && full) v = load16_nt(row + x0);
        else v = load16_guarded(row, x0, m);
      }
      if constexpr (KEEP_RAW) {
        raw[r] = v;
#pragma unroll
        for (int p = 0; p < PPL; ++p) sp[p] += extract_ct<MODE, T, CT>(v.v[p], ex);
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          CT val = (i < n) ? extract_ct<MODE, T, CT>(v.v[p], ex) : CT(0);
          if (!full) val = (x0 + p < m) ? val : CT(0);
          u[r][p] = val;
          sp[p] += val;
        }
      }
    }

    if constexpr (KEEP_RAW) {
#pragma unroll
      for (int r = 0; r < MPW; ++r) opaque(raw[r]);   // widen again in phase 2
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
      lds_barrier();
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
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] *= wv[p];      // s now holds w * s
    }
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      CT tm = CT(0), ta = CT(0);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        CT uv;
        if constexpr (KEEP_RAW) uv = extract_ct<MODE, T, CT>(raw[r].v[p], ex);
        else uv = u[r][p];
        tm += WEIGHTED ? wv[p] * uv : uv;
        ta += s[p] * uv;
      }
      accm[r] += tm;
      acca[r] += ta;
    }
  }

  const int ng = gridDim.x;
#pragma unroll
  for (int r = 0; r < MPW; ++r) {
    const double a = wave_sum((double)accm[r]);
    const double b = wave_sum((double)acca[r]);
    const int i = mbase + r;
    if (lane == 0 && i < n) {
      part[(size_t)i * ng + blockIdx.x] = a;
      part[((size_t)n + i) * ng + blockIdx.x] = b;
    }
  }
}

// ---------------------------------------------------------------------------
// Binary path (U8 masks, or STEP on fields), exact integers.
// part layout: [2][n][grid.x] long long (m, S).
template <typename T, int MODE, int MPW, bool SFROM, int NWMAX>
__global__ __launch_bounds__(64 * NWMAX) void pidmean_bin_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, Extract ex, int64_t ntiles,
    const int* __restrict__ sglob, long long* __restrict__ part, int vec) {
  constexpr int PPL = Vec16<T>::N;
  constexpr int TP = 64 * PPL;
  constexpr bool PACKED = (sizeof(T) == 1 && MODE == MODE_NONE);
  const bool VEC = vec != 0;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* sbuf = reinterpret_cast<int*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int nw = blockDim.x >> 6;
  const int mbase = (SFROM ? blockIdx.y * nw * MPW : 0) + wave * MPW;

  // per-lane integer sums stay below 2^31: at most (tiles per workgroup) *
  // PPL * N, and the grid keeps the tiles per workgroup small
  int accm[MPW], acca[MPW];
#pragma unroll
  for (int r = 0; r < MPW; ++r) { accm[r] = 0; acca[r] = 0; }

  int it = 0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, ++it) {
    const int64_t x0 = tile * TP + (int64_t)lane * PPL;
    const bool full = (x0 + PPL <= m);
    uint32_t raw[PACKED ? MPW : 1][4];
    int ub[PACKED ? 1 : MPW][PACKED ? 1 : PPL];
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
      lds_barrier();
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

  const int ng = gridDim.x;
#pragma unroll
  for (int r = 0; r < MPW; ++r) {
    const long long a = wave_sum((long long)accm[r]);
    const long long b = wave_sum((long long)acca[r]);
    const int i = mbase + r;
    if (lane == 0 && i < n) {
      part[(size_t)i * ng + blockIdx.x] = a;
      part[((size_t)n + i) * ng + blockIdx.x] = b;
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
// Fixed-order reduction of the per-workgroup partials: one block per member
// and quantity (grid.y = 2: m, then A); thread t sums the partials
// t, t+256, ... in ascending order, then a fixed tree over the 256 threads.
template <bool BIN>
__global__ __launch_bounds__(256) void pidmean_reduce(const void* __restrict__ part_v, int nparts,
                                                      int n, void* __restrict__ out_v) {
  __shared__ double red_d[256];
  __shared__ long long red_i[256];
  const int i = blockIdx.x, q = blockIdx.y, t = threadIdx.x;
  const size_t base = ((size_t)q * n + i) * nparts;
  if constexpr (BIN) {
    const long long* part = reinterpret_cast<const long long*>(part_v);
    long long s = 0;
    for (int b = t; b < nparts; b += 256) s += part[base + b];
    red_i[t] = s;
  } else {
    const double* part = reinterpret_cast<const double*>(part_v);
    double s = 0.0;
    for (int b = t; b < nparts; b += 256) s += part[base + b];
    red_d[t] = s;
  }
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) {
      if constexpr (BIN) red_i[t] += red_i[t + o];
      else red_d[t] += red_d[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    if constexpr (BIN) reinterpret_cast<long long*>(out_v)[(size_t)q * n + i] = red_i[0];
    else reinterpret_cast<double*>(out_v)[(size_t)q * n + i] = red_d[0];
  }
}

// Depth ratios: IN_in = A_i / (N m_i), IN_out = A_i / sum_k m_k.  One block;
// sum_k m_k by a fixed tree.  Binary sums are exact integers, so each ratio is
// one correctly rounded division.
template <bool BIN>
__global__ __launch_bounds__(256) void pidmean_ratios(const void* __restrict__ red_v, int n,
                                                      double* __restrict__ m_out,
                                                      double* __restrict__ in_in,
                                                      double* __restrict__ in_out,
                                                      double* __restrict__ depth) {
#pragma clang fp contract(off)
  __shared__ double red_d[256];
  __shared__ long long red_i[256];
  const int t = threadIdx.x;
  double md = 0.0;
  long long mi = 0;
  for (int i = t; i < n; i += 256) {
    if constexpr (BIN) mi += reinterpret_cast<const long long*>(red_v)[i];
    else md += reinterpret_cast<const double*>(red_v)[i];
  }
  red_d[t] = md;
  red_i[t] = mi;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) { red_d[t] += red_d[t + o]; red_i[t] += red_i[t + o]; }
    __syncthreads();
  }
  for (int i = t; i < n; i += 256) {
    double mm, a, tot;
    if constexpr (BIN) {
      const long long* r = reinterpret_cast<const long long*>(red_v);
      mm = (double)r[i]; a = (double)r[n + i]; tot = (double)red_i[0];
    } else {
      const double* r = reinterpret_cast<const double*>(red_v);
      mm = r[i]; a = r[n + i]; tot = red_d[0];
    }
    const double ii = (mm > 0.0) ? a / ((double)n * mm) : 0.0;
    const double oo = (tot > 0.0) ? a / tot : 0.0;
    if (m_out) m_out[i] = mm;
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

// Optional tuning overrides, read once: PID_TUNE_MEAN_MPW (members per wave:
// 4, 8 or 16) and PID_TUNE_MEAN_TPW (tiles per workgroup, 1..64).  They
// change the launch geometry only, never what is computed.
static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  return v ? atoi(v) : dflt;
}

MeanPlan mean_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted) {
  static const int tune_mpw = env_int("PID_TUNE_MEAN_MPW", 0);
  static const int tune_tpw = env_int("PID_TUNE_MEAN_TPW", 16);
  MeanPlan p{};
  p.binary = is_binary(dtype, iso_kind, weighted) ? 1 : 0;
  const int eb = elem_bytes(dtype);
  const int ppl = 16 / eb;
  const int tp = 64 * ppl;
  // members per wave: the smallest slice that covers N with at most 8 waves;
  // FP32 soft input may use 16 waves of 16 members (N <= 256) within the
  // 128 registers a 1024-thread workgroup allows; beyond: two passes.
  int mpw = 4;
  if (n > 32) mpw = 8;
  if (n > 64) mpw = 16;
  if (tune_mpw == 4 || tune_mpw == 8 || tune_mpw == 16) mpw = tune_mpw;
  int nw = (int)((n + mpw - 1) / mpw);
  const int max_waves = (eb == 4 && !p.binary) ? 16 : 8;
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
  // at most 16 tiles per workgroup (short FP32 / INT32 lane sums), and at
  // least two workgroups per CU when there are enough tiles
  const int64_t cus = device_cu_count();
  const int64_t tpw = std::min(64, std::max(1, tune_tpw));
  int64_t g = std::max<int64_t>((p.ntiles + tpw - 1) / tpw, cus * 2);
  if (p.two_pass) g = std::max<int64_t>((p.ntiles + tpw - 1) / tpw, std::max<int64_t>(1, cus * 2 / p.groups));
  p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, g));
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
#define PM_LAUNCH(W, S)                                                                        \
  do {                                                                                           \
    if constexpr (sizeof(T) == 4) {                                                              \
      if (p.nwaves > 8) {                                                                        \
        hipLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, W, S, 16>), grid, block,          \
                           p.lds_bytes, st, U, e.ld, (int)e.n, e.m, e.weights, ex, p.ntiles,     \
                           sglob, part, vec ? 1 : 0);                                            \
        break;                                                                                   \
      }                                                                                          \
    }                                                                                            \
    hipLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, W, S, 8>), grid, block, p.lds_bytes,   \
                       st, U, e.ld, (int)e.n, e.m, e.weights, ex, p.ntiles, sglob, part,         \
                       vec ? 1 : 0);                                                             \
  } while (0)
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
#define PB_LAUNCH(S)                                                                          \
  hipLaunchKernelGGL((pidmean_bin_kernel<T, MODE, MPW, S, 8>), grid, block, p.lds_bytes, st, U,   \
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
  dim3 rgrid((unsigned)e.n, 2);
  if (p.binary) {
    hipLaunchKernelGGL(pidmean_reduce<true>, rgrid, 256, 0, st, part, p.grid, (int)e.n, red);
    hipLaunchKernelGGL(pidmean_ratios<true>, 1, 256, 0, st, red, (int)e.n, out.mass, out.in_in,
                       out.in_out, out.depth);
  } else {
    hipLaunchKernelGGL(pidmean_reduce<false>, rgrid, 256, 0, st, part, p.grid, (int)e.n, red);
    hipLaunchKernelGGL(pidmean_ratios<false>, 1, 256, 0, st, red, (int)e.n, out.mass, out.in_in,
                       out.in_out, out.depth);
  }
  return hipGetLastError();
}

}  // namespace pidk

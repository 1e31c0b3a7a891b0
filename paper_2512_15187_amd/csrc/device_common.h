// Device-side helpers shared by the PID kernels for gfx950 (CDNA4):
// element types, fuzzy extraction of membership probabilities (Sec. 3.5),
// vector loads and 64-lane wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "pid_internal.h"

namespace pidk {

typedef _Float16 f16;
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Stored bf16 is handled as raw 16-bit patterns.
struct bf16_t { uint16_t bits; };

// Parameters of the isovalue model, prepared on the host.
//   GAUSS: u = 0.5 * erfc((f - c) * a) with a = -side / (sigma * sqrt(2)),
//          i.e. u = Phi(side * (f - c) / sigma).
//   STEP:  u = [side * (f - c) > 0].  For values that widen exactly to float,
//          f > c  <=>  f > c_dn  (c_dn = largest float <= c) and
//          f < c  <=>  f < c_up  (c_up = smallest float >= c).
//   MODEL: with t = (f - c) * a,
//          RAMP    (isovalue uniform on [c - h, c + h], a = side / (2h)):  clamp(t + 1/2, 0, 1)
//          TENT    (level-centred map of width h, a = 1 / h):              max(0, 1 - |t|)
//          DENSITY (normalised density, c = 0 here, a = 1 / normaliser):   clamp(t, 0, 1)
struct Extract {
  int side;
  float cf, af;
  float c_dn, c_up;
  double cd, ad;
  int model;
};

__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(f16 v) { return (float)v; }
__device__ __forceinline__ float to_float(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
__device__ __forceinline__ float to_float(uint8_t v) { return (float)v; }
__device__ __forceinline__ float to_float(double v) { return (float)v; }

__device__ __forceinline__ double to_double(double v) { return v; }
template <typename T>
__device__ __forceinline__ double to_double(T v) { return (double)to_float(v); }

// erfc(z) / 2 in FP32 without a division, from the normal tail T(y) = 1 -
// Phi(y) at y = sqrt(2) z (the caller folds sqrt(2) into its scale factor).
// For y >= 0, T(y) = 2^(-1 - P(y)) with P(y) = a1 y + ... + a7 y^7: a
// weighted minimax fit of -log2(2 T(y)) on [0, 6] (weights T ln 2, so that
// the error is absolute; fit_normal_tail.py beside this file).  P(0) = 0 gives
// T(0) = 1/2 exactly; beyond 6 the argument is clamped (T(6) < 1e-9).  With
// FP32 rounding and the hardware 2^x the result is within 1.1e-7 of T and
// 1.4e-7 of 1 - T: one exponential and eight multiply-adds per value, far
// below the FP16 rounding of the values it feeds and the 1e-4 depth tolerance
// of the mixed-precision paths.  erfc(-z) / 2 = 1 - erfc(z) / 2.
constexpr float kSqrt2 = 1.41421356237309515f;

__device__ __forceinline__ float half_erfc_fast(float y) {
  const float x = fminf(fabsf(y), 6.0f);
  // -(1 + P(x)) in Horner form (the coefficients are -a_k)
  float q = 9.856917131e-06f;
  q = fmaf(x, q, -6.527679943e-05f);
  q = fmaf(x, q, -3.862405429e-04f);
  q = fmaf(x, q, 7.337194867e-03f);
  q = fmaf(x, q, -5.265045911e-02f);
  q = fmaf(x, q, -4.591701627e-01f);
  q = fmaf(x, q, -1.151107550e+00f);
  const float h = __builtin_amdgcn_exp2f(fmaf(x, q, -1.0f));   // T(|y|)
  return y >= 0.0f ? h : 1.0f - h;
}

// Lets a kernel take as dynamic LDS all of the CU's 160 KB that its static
// LDS leaves.  Called before a launch: the first call for a kernel sets the
// attribute and records the outcome, later calls for it return that outcome
// (a registry keyed by the kernel, so kernels of the same signature launched
// from one call site are each set).  A failure is returned and cleared, so
// that it does not surface at a later launch.
inline hipError_t allow_dynamic_lds(const void* k) {
  static std::mutex mu;
  static std::unordered_map<const void*, hipError_t> done;
  std::lock_guard<std::mutex> lk(mu);
  const auto it = done.find(k);
  if (it != done.end()) return it->second;
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, k);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(163840 - fa.sharedSizeBytes));
  if (e != hipSuccess) (void)hipGetLastError();
  done.emplace(k, e);
  return e;
}

// Membership probability in float from a stored value (all input types but
// double; doubles use extract_d).  FAST selects half_erfc_fast for the
// Gaussian model (the 16-bit MFMA Gram and PID-mean loaders); otherwise erfcf.
template <int MODE, typename T, bool FAST = false>
__device__ __forceinline__ float extract_f(T raw, const Extract& e) {
  float f = to_float(raw);
  if constexpr (MODE == MODE_NONE) {
    return f;
  } else if constexpr (MODE == MODE_GAUSS) {
    if constexpr (FAST) return half_erfc_fast((f - e.cf) * (e.af * kSqrt2));
    else return 0.5f * erfcf((f - e.cf) * e.af);
  } else if constexpr (MODE == MODE_MODEL) {
    const float t = (f - e.cf) * e.af;
    if (e.model == PID_ISO_TENT) return fmaxf(0.0f, 1.0f - fabsf(t));
    return fminf(fmaxf(e.model == PID_ISO_RAMP ? t + 0.5f : t, 0.0f), 1.0f);
  } else {
    return (e.side > 0) ? (f > e.c_dn ? 1.0f : 0.0f) : (f < e.c_up ? 1.0f : 0.0f);
  }
}

template <int MODE, typename T>
__device__ __forceinline__ double extract_d(T raw, const Extract& e) {
  double f = to_double(raw);
  if constexpr (MODE == MODE_NONE) {
    return f;
  } else if constexpr (MODE == MODE_GAUSS) {
    return 0.5 * erfc((f - e.cd) * e.ad);
  } else if constexpr (MODE == MODE_MODEL) {
    const double t = (f - e.cd) * e.ad;
    if (e.model == PID_ISO_TENT) return fmax(0.0, 1.0 - fabs(t));
    return fmin(fmax(e.model == PID_ISO_RAMP ? t + 0.5 : t, 0.0), 1.0);
  } else {
    return (e.side > 0) ? (f > e.cd ? 1.0 : 0.0) : (f < e.cd ? 1.0 : 0.0);
  }
}

// Binary decision as an integer (STEP on fields, or U8 masks with MODE_NONE).
template <int MODE, typename T>
__device__ __forceinline__ int extract_bit(T raw, const Extract& e) {
  if constexpr (MODE == MODE_STEP) {
    if constexpr (sizeof(T) == 8) {
      double f = to_double(raw);
      return (e.side > 0) ? (f > e.cd) : (f < e.cd);
    } else {
      float f = to_float(raw);
      return (e.side > 0) ? (f > e.c_dn) : (f < e.c_up);
    }
  } else {
    return (int)to_float(raw);
  }
}

// 16-byte vector of stored elements.
template <typename T>
struct Vec16 {
  static constexpr int N = 16 / sizeof(T);
  T v[N];
};

template <typename T>
__device__ __forceinline__ Vec16<T> load16(const T* p) {
  uint4 r = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(Vec16<T>, r);
}

template <typename T>
__device__ __forceinline__ Vec16<T> load16_nt(const T* p) {
  u32x4 r = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return __builtin_bit_cast(Vec16<T>, r);
}

// Vector of B (4, 8 or 16) bytes of stored elements, loaded non-temporally.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <typename T, int B>
struct VecB {
  static constexpr int N = B / sizeof(T);
  T v[N];
};

template <typename T, int B>
__device__ __forceinline__ VecB<T, B> loadB_nt(const T* p) {
  if constexpr (B == 16) {
    u32x4 r = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return __builtin_bit_cast(VecB<T, B>, r);
  } else {
    static_assert(B == 8, "8- or 16-byte vectors");
    u32x2 r = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    return __builtin_bit_cast(VecB<T, B>, r);
  }
}

// Raw buffer loads: one 128-bit resource per wave (base, byte extent) in
// scalar registers, a 32-bit per-lane byte offset and a wave-uniform scalar
// offset; cache policy "non-temporal".  Rows of a tile then share one offset
// register instead of holding a 64-bit address each.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T, int B>
__device__ __forceinline__ VecB<T, B> bufload_nt(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (B == 16) {
    intx4 r = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 2);
    return __builtin_bit_cast(VecB<T, B>, r);
  } else if constexpr (B == 4) {
    int r = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 2);
    return __builtin_bit_cast(VecB<T, B>, r);
  } else {
    typedef int intx2 __attribute__((ext_vector_type(2)));
    intx2 r = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 2);
    return __builtin_bit_cast(VecB<T, B>, r);
  }
}

// Direct load into LDS: every lane reads B (4 or 16) bytes at byte offset
// voff of the resource, and the wave's 64 results land in LDS contiguously
// from dst (lane l at dst + l * B), without passing through registers.  An
// offset at or past the resource's extent writes zeros and reads no memory.
// The instruction is written out (M0 = LDS address) rather than left to the
// compiler, which would otherwise wait for every such load before any LDS
// read it cannot prove disjoint; callers order LDS reads themselves with
// vm_wait<N>() (loads retire in order) and barriers.  It has no register
// results, and one call is exactly one instruction for the whole wave.
// The resource words must be wave-uniform.
typedef int intx4_t __attribute__((ext_vector_type(4)));
struct BufRes {
  intx4_t w;
};
__device__ __forceinline__ BufRes make_bufres(const void* base, uint32_t bytes) {
  const uint64_t a = (uint64_t)(uintptr_t)base;
  BufRes r;
  r.w[0] = (int)__builtin_amdgcn_readfirstlane((uint32_t)a);
  r.w[1] = (int)(__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) & 0xffffu);   // stride 0
  r.w[2] = (int)__builtin_amdgcn_readfirstlane(bytes);
  r.w[3] = 0x00020000;
  return r;
}
template <int B>
__device__ __forceinline__ void dma_to_lds(const BufRes& rs, const void* dst, uint32_t voff) {
  const uint32_t l = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
  asm volatile("" : "+v"(voff));   // keep a select of the offset a select
  if constexpr (B == 16) {
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds"
                 :: "s"(l), "v"(voff), "s"(rs.w) : "memory", "m0");
  } else {
    static_assert(B == 4, "4- or 16-byte lanes");
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, 0 offen lds"
                 :: "s"(l), "v"(voff), "s"(rs.w) : "memory", "m0");
  }
}
// The same with a wave-uniform byte offset `soff` added to every lane's
// (in a scalar register; voff + soff must stay below 2^32).
template <int B>
__device__ __forceinline__ void dma_to_lds(const BufRes& rs, const void* dst, uint32_t voff, uint32_t soff) {
  const uint32_t l = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
  const uint32_t so = __builtin_amdgcn_readfirstlane(soff);
  asm volatile("" : "+v"(voff));
  if constexpr (B == 16) {
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
                 :: "s"(l), "v"(voff), "s"(rs.w), "s"(so) : "memory", "m0");
  } else {
    static_assert(B == 4, "4- or 16-byte lanes");
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, %3 offen lds"
                 :: "s"(l), "v"(voff), "s"(rs.w), "s"(so) : "memory", "m0");
  }
}

// Wait until at most N vector memory operations of this wave are outstanding.
template <int N>
__device__ __forceinline__ void vm_wait() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Hide a register vector from common-subexpression elimination.
template <typename T, int B>
__device__ __forceinline__ void opaque(VecB<T, B>& v) {
  uint32_t q[B / 4];
  __builtin_memcpy(q, &v, B);
#pragma unroll
  for (int i = 0; i < B / 4; ++i) asm volatile("" : "+v"(q[i]));
  __builtin_memcpy(&v, q, B);
}

// Guarded form of loadB_nt for a ragged tile: entries at or past m read as
// zero; every access is in bounds (index clamped to m - 1).
template <typename T, int B>
__device__ __forceinline__ VecB<T, B> loadB_guarded(const T* row, int64_t x0, int64_t m) {
  using E = typename std::conditional<sizeof(T) == 8, uint64_t,
            typename std::conditional<sizeof(T) == 4, uint32_t,
            typename std::conditional<sizeof(T) == 2, uint16_t, uint8_t>::type>::type>::type;
  const E* rb = reinterpret_cast<const E*>(row);
  VecB<T, B> out;
#pragma unroll
  for (int p = 0; p < VecB<T, B>::N; ++p) {
    const int64_t x = x0 + p;
    const E v = rb[x < m ? x : m - 1];
    out.v[p] = __builtin_bit_cast(T, (E)(x < m ? v : (E)0));
  }
  return out;
}

// Element-wise guarded load of up to Vec16<T>::N values starting at index x0
// of a row with m >= 1 valid entries; missing entries read as zero.  Every
// load reads an in-bounds element (index clamped to m - 1) and the value is
// then selected, so no branch and no stack copy is needed.
template <typename T>
__device__ __forceinline__ Vec16<T> load16_guarded(const T* row, int64_t x0, int64_t m) {
  using B = typename std::conditional<sizeof(T) == 8, uint64_t,
            typename std::conditional<sizeof(T) == 4, uint32_t,
            typename std::conditional<sizeof(T) == 2, uint16_t, uint8_t>::type>::type>::type;
  const B* rb = reinterpret_cast<const B*>(row);
  Vec16<T> out;
#pragma unroll
  for (int p = 0; p < Vec16<T>::N; ++p) {
    const int64_t x = x0 + p;
    const B v = rb[x < m ? x : m - 1];
    out.v[p] = __builtin_bit_cast(T, (B)(x < m ? v : (B)0));
  }
  return out;
}

// Hide a 16-byte register vector from common-subexpression elimination, so
// that values derived from it are recomputed instead of kept live.
template <typename T>
__device__ __forceinline__ void opaque(Vec16<T>& v) {
  uint4 q = __builtin_bit_cast(uint4, v);
  asm volatile("" : "+v"(q.x), "+v"(q.y), "+v"(q.z), "+v"(q.w));
  v = __builtin_bit_cast(Vec16<T>, q);
}

// Workgroup barrier for LDS hand-offs only: waits for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads() it carries no memory
// fence, so global loads issued ahead (register prefetch) stay in flight
// across it.  Only LDS data may be exchanged through it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Round an FP32 value to FP16 as a separate step.  The value passes through
// an empty asm first, so the compiler cannot fuse the product that produced
// it with the conversion (a mixed-precision FMA rounds once, the two steps
// twice), and every kernel variant rounds the same way.
__device__ __forceinline__ _Float16 to_f16_rounded(float v) {
  asm volatile("" : "+v"(v));
  return (_Float16)v;
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---- wavefront (64-lane) sums; fixed butterfly order => deterministic ----
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---- sums across lanes without the LDS crossbar ----
// The gfx950 lane swaps (v_permlane16_swap / v_permlane32_swap) run in the
// vector ALU; every lane of the wave must be active.
// Lanes below 32 (resp. in even rows of 16) get x + x of the lane 32 (16)
// above; the others get y of the lane 32 (16) below + their own y.
__device__ __forceinline__ float fold32(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float fold16(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Sum over the lanes l, l ^ T, l ^ 2T, ... (T = 16 or 32; T = 64: the value
// itself), the same bits in all of them.
template <int T>
__device__ __forceinline__ float sum_from(float v) {
  static_assert(T == 16 || T == 32 || T == 64, "lane stride");
  if constexpr (T == 16) v = fold16(v, v);
  if constexpr (T <= 32) v = fold32(v, v);
  return v;
}

// ---- float -> 16-bit conversions (round to nearest even) ----
// (the hardware conversion, v_cvt_pk_bf16_f32: round to nearest even)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
// Two values in one conversion: a in the low half, b in the high half.
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f32x2_to_bf16x2_bits(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v{a, b}, bf16x2v));
}

}  // namespace pidk

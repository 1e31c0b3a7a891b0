// Gram kernel template for the all-pairs PID numerators (see k_gram.hip for
// the algorithm); included by the per-input-type translation units.
#pragma once
#include "device_common.h"
#include <hip/hip_ext.h>
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

namespace pidk {

template <int MT> struct MTraits;
template <> struct MTraits<MT_F16>   { using E = f16;      static constexpr int EB = 2; static constexpr int KK = 16; static constexpr int PLANES = 1; };
template <> struct MTraits<MT_BF16>  { using E = uint16_t; static constexpr int EB = 2; static constexpr int KK = 16; static constexpr int PLANES = 1; };
template <> struct MTraits<MT_BF16X3>{ using E = uint16_t; static constexpr int EB = 2; static constexpr int KK = 16; static constexpr int PLANES = 2; };
template <> struct MTraits<MT_I8>    { using E = int8_t;   static constexpr int EB = 1; static constexpr int KK = 32; static constexpr int PLANES = 1; };
template <> struct MTraits<MT_F32>   { using E = float;    static constexpr int EB = 4; static constexpr int KK = 4;  static constexpr int PLANES = 1; };
template <> struct MTraits<MT_F64>   { using E = double;   static constexpr int EB = 8; static constexpr int KK = 4;  static constexpr int PLANES = 1; };

// Store NB bytes (NB a multiple of 4, at least 4-byte aligned destination) to
// LDS with the widest aligned stores the size allows.
template <int NB>
__device__ __forceinline__ void store_lds(unsigned char* dst, const void* src) {
  const unsigned char* s8 = reinterpret_cast<const unsigned char*>(src);
  if constexpr (NB % 16 == 0) {
#pragma unroll
    for (int o = 0; o < NB; o += 16) {
      uint4 v;
      __builtin_memcpy(&v, s8 + o, 16);
      *reinterpret_cast<uint4*>(dst + o) = v;
    }
  } else if constexpr (NB % 8 == 0) {
#pragma unroll
    for (int o = 0; o < NB; o += 8) {
      uint2 v;
      __builtin_memcpy(&v, s8 + o, 8);
      *reinterpret_cast<uint2*>(dst + o) = v;
    }
  } else {
#pragma unroll
    for (int o = 0; o < NB; o += 4) {
      uint32_t v;
      __builtin_memcpy(&v, s8 + o, 4);
      *reinterpret_cast<uint32_t*>(dst + o) = v;
    }
  }
}

struct GramArgs {
  const void* U;
  int64_t ld;
  int n;
  int64_t m;
  const float* w;
  Extract ex;
  int nbt;             // 32-row blocks covering n
  int sb;              // row blocks per super-block (<= 8)
  int nsuper;          // super-blocks
  int ntiles_super;    // super-tiles
  int np;              // packed upper sub-tiles
  int nsplit;
  int64_t slabs;       // total slabs
  int vec;             // rows are 16-byte aligned
  void* part;          // [nsplit][np][1024] (float / int / double)
  double* part_mass;   // [nsplit][n] partial masses
};

// Super-tile index -> (I, J), I <= J, column-major over J.
__device__ __forceinline__ void super_ij(int t, int& I, int& J) {
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  J = j;
  I = t - j * (j + 1) / 2;
}

// Accumulator vector of one 32x32 sub-tile (int for INT8, float otherwise).
template <int MT>
using AccVec = typename std::conditional<MT == MT_I8, intx16, floatx16>::type;

// Multiply one LDS slab into the wave's sub-tiles: rows of block ir[t] times
// rows of block ic[t] (offset by jrow_base), KS points, row stride ROWB bytes,
// hi/lo planes PLANE bytes apart.  Per k-step the fragments of every
// sub-tile are read first (no data-dependent branch, so the reads are issued
// back to back and their latency is paid once), then the MFMAs follow.
template <int MT, int MAXT, int KS, int ROWB>
__device__ __forceinline__ void mfma_slab(const unsigned char* lbuf, int PLANE, int lane, int nt,
                                          const int* ir, const int* ic, int jrow_base, AccVec<MT>* acc) {
  using TR = MTraits<MT>;
  constexpr int KSTEPS = KS / TR::KK;
  constexpr int FE = 16 / TR::EB;   // elements per lane per fragment (16 bytes)
  constexpr int KUNR = KSTEPS > 2 ? 2 : KSTEPS;
#pragma unroll KUNR
  for (int kk = 0; kk < KSTEPS; ++kk) {
    const int koff = kk * TR::KK + (lane >> 5) * FE;   // element offset in the row
    uint4 fa[MAXT][TR::PLANES], fb[MAXT][TR::PLANES];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const unsigned char* pa = lbuf + (size_t)(ir[t] * 32 + (lane & 31)) * ROWB + koff * TR::EB;
      const unsigned char* pb = lbuf + (size_t)(jrow_base + ic[t] * 32 + (lane & 31)) * ROWB + koff * TR::EB;
      fa[t][0] = *reinterpret_cast<const uint4*>(pa);
      fb[t][0] = *reinterpret_cast<const uint4*>(pb);
      if constexpr (TR::PLANES == 2) {
        fa[t][1] = *reinterpret_cast<const uint4*>(pa + PLANE);
        fb[t][1] = *reinterpret_cast<const uint4*>(pb + PLANE);
      }
    }
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < nt) {
        if constexpr (MT == MT_F16) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, fa[t][0]),
                                                           __builtin_bit_cast(half8, fb[t][0]), acc[t], 0, 0, 0);
        } else if constexpr (MT == MT_BF16) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[t][0]),
                                                            __builtin_bit_cast(bf16x8, fb[t][0]), acc[t], 0, 0, 0);
        } else if constexpr (MT == MT_BF16X3) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[t][0]),
                                                            __builtin_bit_cast(bf16x8, fb[t][0]), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[t][0]),
                                                            __builtin_bit_cast(bf16x8, fb[t][1]), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[t][1]),
                                                            __builtin_bit_cast(bf16x8, fb[t][0]), acc[t], 0, 0, 0);
        } else {
          acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(intx4, fa[t][0]),
                                                          __builtin_bit_cast(intx4, fb[t][0]), acc[t], 0, 0, 0);
        }
      }
    }
  }
}

// acc += A B^T for one k-step of fragments (hi/lo planes for BF16x3).
template <int MT, int PL>
__device__ __forceinline__ void mfma_step(AccVec<MT>& acc, const uint4 (&fa)[PL], const uint4 (&fb)[PL]) {
  if constexpr (MT == MT_F16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, fa[0]), __builtin_bit_cast(half8, fb[0]),
                                                 acc, 0, 0, 0);
  } else if constexpr (MT == MT_BF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]), __builtin_bit_cast(bf16x8, fb[0]),
                                                  acc, 0, 0, 0);
  } else if constexpr (MT == MT_BF16X3) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]), __builtin_bit_cast(bf16x8, fb[0]),
                                                  acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]), __builtin_bit_cast(bf16x8, fb[1]),
                                                  acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[1]), __builtin_bit_cast(bf16x8, fb[0]),
                                                  acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(intx4, fa[0]), __builtin_bit_cast(intx4, fb[0]),
                                                acc, 0, 0, 0);
  }
}

// Grouped sub-tiles of one wave (rows r0 against r1 and r2, and r2 against
// itself when `three`): acc[0] += F(r0) F(r1)^T, acc[1] += F(r0) F(r2)^T,
// acc[2] += F(r2) F(r2)^T.  Three fragment reads per k-step.
template <int MT, int KS, int ROWB>
__device__ __forceinline__ void mfma_slab_g(const unsigned char* lbuf, int PLANE, int lane, bool three, int r0,
                                            int r1, int r2, AccVec<MT>* acc) {
  using TR = MTraits<MT>;
  constexpr int KSTEPS = KS / TR::KK;
  constexpr int FE = 16 / TR::EB;
  // k-steps whose fragments are read before their MFMAs (all reads issued
  // back to back, one wait): two, or one with hi/lo planes
  constexpr int KG = (TR::PLANES == 1 && KSTEPS % 2 == 0) ? 2 : 1;
  const unsigned char* p0 = lbuf + (size_t)(r0 * 32 + (lane & 31)) * ROWB + (lane >> 5) * FE * TR::EB;
  const unsigned char* p1 = lbuf + (size_t)(r1 * 32 + (lane & 31)) * ROWB + (lane >> 5) * FE * TR::EB;
  const unsigned char* p2 = lbuf + (size_t)(r2 * 32 + (lane & 31)) * ROWB + (lane >> 5) * FE * TR::EB;
#pragma unroll
  for (int k0 = 0; k0 < KSTEPS; k0 += KG) {
    uint4 f0[KG][TR::PLANES], f1[KG][TR::PLANES], f2[KG][TR::PLANES];
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      const int koff = (k0 + g) * TR::KK * TR::EB;
#pragma unroll
      for (int q = 0; q < TR::PLANES; ++q) {
        f0[g][q] = *reinterpret_cast<const uint4*>(p0 + koff + q * PLANE);
        f1[g][q] = *reinterpret_cast<const uint4*>(p1 + koff + q * PLANE);
        f2[g][q] = *reinterpret_cast<const uint4*>(p2 + koff + q * PLANE);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < KG; ++g) {
      mfma_step<MT>(acc[0], f0[g], f1[g]);
      mfma_step<MT>(acc[1], f0[g], f2[g]);
      if (three) mfma_step<MT>(acc[2], f2[g], f2[g]);
    }
  }
}

// The same with fragment reuse: a fragment is read once while consecutive
// sub-tiles share it (fewer registers; used where registers also hold the
// prefetched slab).
template <int MT, int MAXT, int KS, int ROWB>
__device__ __forceinline__ void mfma_slab_reuse(const unsigned char* lbuf, int PLANE, int lane, int nt,
                                                const int* ir, const int* ic, int jrow_base, AccVec<MT>* acc) {
  using TR = MTraits<MT>;
  constexpr int KSTEPS = KS / TR::KK;
  constexpr int FE = 16 / TR::EB;
  constexpr int KUNR = KSTEPS > 4 ? 4 : KSTEPS;
#pragma unroll KUNR
  for (int kk = 0; kk < KSTEPS; ++kk) {
    const int koff = kk * TR::KK + (lane >> 5) * FE;
    uint4 fa[TR::PLANES], fb[TR::PLANES];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < nt) {
        const bool newa = (t == 0) || (ir[t] != ir[t - 1]);
        const bool newb = (t == 0) || (ic[t] != ic[t - 1]);
        if (newa) {
          const unsigned char* pa = lbuf + (size_t)(ir[t] * 32 + (lane & 31)) * ROWB + koff * TR::EB;
          fa[0] = *reinterpret_cast<const uint4*>(pa);
          if constexpr (TR::PLANES == 2) fa[1] = *reinterpret_cast<const uint4*>(pa + PLANE);
        }
        if (newb) {
          const unsigned char* pb = lbuf + (size_t)(jrow_base + ic[t] * 32 + (lane & 31)) * ROWB + koff * TR::EB;
          fb[0] = *reinterpret_cast<const uint4*>(pb);
          if constexpr (TR::PLANES == 2) fb[1] = *reinterpret_cast<const uint4*>(pb + PLANE);
        }
        if constexpr (MT == MT_F16) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, fa[0]),
                                                           __builtin_bit_cast(half8, fb[0]), acc[t], 0, 0, 0);
        } else if constexpr (MT == MT_BF16) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]),
                                                            __builtin_bit_cast(bf16x8, fb[0]), acc[t], 0, 0, 0);
        } else if constexpr (MT == MT_BF16X3) {
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]),
                                                            __builtin_bit_cast(bf16x8, fb[0]), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[0]),
                                                            __builtin_bit_cast(bf16x8, fb[1]), acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, fa[1]),
                                                            __builtin_bit_cast(bf16x8, fb[0]), acc[t], 0, 0, 0);
        } else {
          acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(intx4, fa[0]),
                                                          __builtin_bit_cast(intx4, fb[0]), acc[t], 0, 0, 0);
        }
      }
    }
  }
}

template <typename Tin, int MT, int MODE, int MAXT, int CPR, int CH, bool WEIGHTED>
__global__ __launch_bounds__(512) void gram_kernel(GramArgs a) {
  const bool VEC = a.vec != 0;
  using TR = MTraits<MT>;
  using E = typename TR::E;
  constexpr int EPC = 16 / sizeof(Tin);          // elements per 16-byte chunk
  constexpr int KS = CPR * EPC;                  // points per slab
  constexpr int G4 = EPC < 4 ? EPC : 4;          // elements converted together
  constexpr int ROWB = KS * TR::EB + 16;         // LDS row stride in bytes (padded)
  constexpr bool IS_MFMA = (MT == MT_F16 || MT == MT_BF16 || MT == MT_BF16X3 || MT == MT_I8);
  constexpr bool BIN = (MT == MT_I8);
  using AccE = typename std::conditional<MT == MT_F64, double, float>::type;
  extern __shared__ __align__(16) unsigned char lds[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();

  // --- XCD-aware decode of the block index
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int q = b >> 3;
  const int st = q % a.ntiles_super;
  const int split = (q / a.ntiles_super) * 8 + xcd;
  int SI, SJ;
  super_ij(st, SI, SJ);
  const bool diag = (SI == SJ);
  const int na = min(a.sb, a.nbt - a.sb * SI);   // row blocks on the I side
  const int nb = min(a.sb, a.nbt - a.sb * SJ);   // row blocks on the J side
  const int rowsI = 32 * na;
  const int rows = diag ? rowsI : rowsI + 32 * nb;
  const int PLANE = rows * ROWB;                 // bytes of one LDS plane
  const int LBUF = TR::PLANES * PLANE;           // bytes of one LDS slab buffer

  // --- this wave's sub-tiles
  const int T = diag ? na * (na + 1) / 2 : na * nb;
  const int t0 = (wave * T) / 8, t1 = ((wave + 1) * T) / 8;
  const int nt = t1 - t0;
  int ir[MAXT], ic[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    int k = min(t0 + t, T - 1);
    if (diag) {
      int c = 0;
      while ((c + 1) * (c + 2) / 2 <= k) ++c;
      ic[t] = c;
      ir[t] = k - c * (c + 1) / 2;
    } else {
      ir[t] = k / nb;
      ic[t] = k % nb;
    }
  }

  // --- slabs of this split: split, split + nsplit, split + 2 nsplit, ...
  // (interleaved, so that at any time the workgroups read neighbouring slabs
  // of every row)
  const int64_t cnt = (a.slabs > split) ? (a.slabs - 1 - split) / a.nsplit + 1 : 0;
  auto slab = [&](int64_t j) -> int64_t { return split + j * a.nsplit; };

  // --- loader geometry: chunk q = tid + 512*ci -> row tid/CPR + (512/CPR)*ci, column tid%CPR
  const int ccol = tid % CPR;
  const int crow0 = tid / CPR;
  constexpr int RSTEP = 512 / CPR;
  const Tin* U = reinterpret_cast<const Tin*>(a.U);
  auto grow = [&](int lrow) -> int {
    return (lrow < rowsI) ? (32 * a.sb * SI + lrow) : (32 * a.sb * SJ + lrow - rowsI);
  };

  // Row of every chunk slot, clamped to a valid row so that the loads of full
  // slabs need no branches (slots outside the super-tile or past N are masked
  // when the slab is stored).
  int rowid[CH];
  unsigned rvalid_bits = 0;
#pragma unroll
  for (int ci = 0; ci < CH; ++ci) {
    const int lr = crow0 + RSTEP * ci;
    const int gr = grow(lr);
    const bool ok = (lr < rows) && (gr < a.n);
    rowid[ci] = ok ? gr : 0;
    rvalid_bits |= (ok ? 1u : 0u) << ci;
  }
  // two register buffers: slab s+1 stays in flight while slab s is stored,
  // and the loads for slab s+2 are issued as soon as slab s left its buffer
  Vec16<Tin> preA[CH], preB[CH];
  float wA[EPC], wB[EPC];   // weights of the slab's points (prefetched with it)
  auto load_full = [&](Vec16<Tin>* pre, float* wp, int64_t s) {   // every element in range, rows aligned
    const int64_t x0 = s * KS + (int64_t)ccol * EPC;
#pragma unroll
    for (int ci = 0; ci < CH; ++ci) pre[ci] = load16(U + (int64_t)rowid[ci] * a.ld + x0);
    if constexpr (WEIGHTED) {
#pragma unroll
      for (int e = 0; e < EPC; e += 4) {
        const float4 t = *reinterpret_cast<const float4*>(a.w + x0 + e);
        wp[e] = t.x;
        if (e + 1 < EPC) wp[e + 1] = t.y;
        if (e + 2 < EPC) wp[e + 2] = t.z;
        if (e + 3 < EPC) wp[e + 3] = t.w;
      }
    }
  };

  // masses (diagonal super-tiles only): per slab, the CPR lanes that share a
  // row add their chunk sums (fixed butterfly) and the first of them adds the
  // row sum to the row's FP64 accumulator in LDS, placed after the two slab
  // buffers.  Each row has one owner lane, which also clears it, so the order
  // is the slab order and no barrier is needed until the final read.
  double* lmass = reinterpret_cast<double*>(lds + 2 * LBUF);
#pragma unroll
  for (int ci = 0; ci < CH; ++ci) {
    const int lr = crow0 + RSTEP * ci;
    if (ccol == 0 && lr < rows) lmass[lr] = 0.0;
  }
  auto add_mass = [&](int ci, AccE v) {
#pragma unroll
    for (int o = CPR / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lr = crow0 + RSTEP * ci;
    if (ccol == 0) lmass[lr] += (double)v;
  };

  // Convert one slab from registers into the LDS tile, four elements at a
  // time (short live ranges), and add the masses.
  auto store_chunk = [&](int ci, const Vec16<Tin>& pv, const float* wv, int64_t s, unsigned char* lbuf) {
#pragma clang fp contract(off)   // the same rounding sequence as the LDS-staged kernel
    const int64_t x0 = s * KS + (int64_t)ccol * EPC;
    const bool full = (x0 + EPC <= a.m);
    {
      const int lr = crow0 + RSTEP * ci;
      if (lr >= rows) return;
      const bool rvalid = (rvalid_bits >> ci) & 1u;
      unsigned char* dst = lbuf + (size_t)lr * ROWB + (size_t)ccol * EPC * TR::EB;
      if constexpr (BIN && sizeof(Tin) == 1 && MODE == MODE_NONE) {
        // 0/1 bytes go to LDS as they are; ones counted four bytes at a time
        uint4 q = __builtin_bit_cast(uint4, pv);
        if (!rvalid) q = make_uint4(0u, 0u, 0u, 0u);
        if (!full) {
          uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int d = 0; d < 4; ++d) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (x0 + 4 * d + b >= a.m) w4[d] &= ~(0xffu << (8 * b));
          }
          q = make_uint4(w4[0], w4[1], w4[2], w4[3]);
        }
        const int cnt = (int)(((q.x * 0x01010101u) >> 24) + ((q.y * 0x01010101u) >> 24) +
                              ((q.z * 0x01010101u) >> 24) + ((q.w * 0x01010101u) >> 24));
        if (diag) add_mass(ci, (AccE)cnt);
        *reinterpret_cast<uint4*>(dst) = q;
      } else if constexpr (BIN) {
        int cnt = 0;
#pragma unroll
        for (int g = 0; g < EPC; g += 4) {
          int8_t o[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            int bit = rvalid ? extract_bit<MODE>(pv.v[g + e], a.ex) : 0;
            if (!full) bit = (x0 + g + e < a.m) ? bit : 0;
            o[e] = (int8_t)bit;
            cnt += bit;
          }
          store_lds<4>(dst + g, o);
        }
        if (diag) add_mass(ci, (AccE)cnt);
      } else {
        AccE msum = AccE(0);
#pragma unroll
        for (int g = 0; g < EPC; g += G4) {
          AccE uv[G4];
#pragma unroll
          for (int e = 0; e < G4; ++e) {
            AccE u;
            if constexpr (MT == MT_F64 || sizeof(Tin) == 8) u = (AccE)extract_d<MODE>(pv.v[g + e], a.ex);
            else u = (AccE)extract_f<MODE, Tin, MT != MT_F32>(pv.v[g + e], a.ex);
            if (!rvalid) u = AccE(0);
            if (!full) u = (x0 + g + e < a.m) ? u : AccE(0);
            if constexpr (WEIGHTED) {
              msum += (AccE)wv[g + e] * u;
              // sqrt(w) in the accumulation precision: an FP32 root would
              // carry its rounding into every FP64 product
              if constexpr (sizeof(AccE) == 8) uv[e] = sqrt((double)wv[g + e]) * u;
              else uv[e] = sqrtf(wv[g + e]) * u;
            }
            else { msum += u; uv[e] = u; }
          }
          unsigned char* d4 = dst + (size_t)g * TR::EB;
          if constexpr (MT == MT_F16) {
            f16 o[G4];
#pragma unroll
            for (int e = 0; e < G4; ++e) o[e] = to_f16_rounded((float)uv[e]);
            store_lds<2 * G4>(d4, o);
          } else if constexpr (MT == MT_BF16) {
            uint16_t o[G4];
#pragma unroll
            for (int e = 0; e < G4; ++e) o[e] = f32_to_bf16_bits((float)uv[e]);
            store_lds<2 * G4>(d4, o);
          } else if constexpr (MT == MT_BF16X3) {
            uint16_t hi[G4], lo[G4];
#pragma unroll
            for (int e = 0; e < G4; ++e) {
              const float v = (float)uv[e];
              hi[e] = f32_to_bf16_bits(v);
              lo[e] = f32_to_bf16_bits(v - bf16_bits_to_f32(hi[e]));
            }
            store_lds<2 * G4>(d4, hi);
            store_lds<2 * G4>(d4 + PLANE, lo);
          } else {
            store_lds<(int)sizeof(AccE) * G4>(d4, uv);
          }
        }
        if (diag) add_mass(ci, msum);
      }
    }
  };
  auto store_slab = [&](const Vec16<Tin>* pre, const float* wv, int64_t s, unsigned char* lbuf) {
#pragma unroll
    for (int ci = 0; ci < CH; ++ci) store_chunk(ci, pre[ci], wv, s, lbuf);
  };
  // Guarded path (ragged last slab, unaligned rows, single-buffer variants):
  // one chunk at a time, loaded by the compiler, straight into LDS.
  auto load_store_guarded = [&](int64_t s, unsigned char* lbuf) {
    const int64_t x0 = s * KS + (int64_t)ccol * EPC;
    float wt[EPC];
    if constexpr (WEIGHTED) {
#pragma unroll
      for (int e = 0; e < EPC; ++e) wt[e] = a.w[(x0 + e < a.m) ? x0 + e : a.m - 1] * ((x0 + e < a.m) ? 1.0f : 0.0f);
    }
#pragma unroll 1
    for (int ci = 0; ci < CH; ++ci) {
      Vec16<Tin> v{};
      if ((rvalid_bits >> ci) & 1u) v = load16_guarded(U + (int64_t)rowid[ci] * a.ld, x0, a.m);
      store_chunk(ci, v, wt, s, lbuf);
    }
  };

  // --- accumulators
  constexpr int ACCN = IS_MFMA ? 16 : 16;
  AccVec<MT> acc[MAXT];
  AccE vacc[IS_MFMA ? 1 : MAXT][IS_MFMA ? 1 : ACCN];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if constexpr (IS_MFMA) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][r] = 0;
    } else {
#pragma unroll
      for (int r = 0; r < ACCN; ++r) vacc[t][r] = AccE(0);
    }
  }

  const int jrow_base = diag ? 0 : rowsI;  // LDS row of J-side block 0

  auto compute_slab = [&](const unsigned char* lbuf) {
    if constexpr (IS_MFMA) {
      mfma_slab_reuse<MT, MAXT, KS, ROWB>(lbuf, PLANE, lane, nt, ir, ic, jrow_base, acc);
    } else {
      // Vector FMA: lane owns a 4x4 block of each 32x32 sub-tile
      // (rows 4*(lane/8) .. +3, cols 4*(lane%8) .. +3).
      const int rr = (lane >> 3) * 4, cc = (lane & 7) * 4;
#pragma unroll 1
      for (int k = 0; k < KS; k += 4) {
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
          if (t < nt) {
            AccE av[4][4], bv[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const AccE* pa = reinterpret_cast<const AccE*>(lbuf + (size_t)(ir[t] * 32 + rr + i) * ROWB) + k;
              const AccE* pb = reinterpret_cast<const AccE*>(lbuf + (size_t)(jrow_base + ic[t] * 32 + cc + i) * ROWB) + k;
#pragma unroll
              for (int kk = 0; kk < 4; ++kk) { av[i][kk] = pa[kk]; bv[i][kk] = pb[kk]; }
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
              for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) vacc[t][i * 4 + j] += av[i][kk] * bv[j][kk];
          }
        }
      }
    }
  };

  // --- main loop over pairs of full slabs of this split, over two register
  // and two LDS buffers.  Slab s goes to LDS buffer s&1; one barrier per slab
  // suffices because a wave can only overwrite a buffer after every wave has
  // passed the next barrier, i.e. after all of them finished multiplying the
  // slab it held (the barrier waits for each wave's LDS reads).  The loop body
  // has no branch around a memory load (the prefetch index is clamped, the
  // last prefetches re-read a slab and are not used), so the compiler's wait
  // counts stay exact: storing one buffer waits only for that buffer while
  // the other stays in flight.
  unsigned char* lds0 = lds;
  unsigned char* lds1 = lds + LBUF;
  const int64_t s_full = a.m / KS;                       // slabs [0, s_full) are full
  constexpr bool DB = IS_MFMA || MT == MT_F32;
  const int64_t nf_all = (s_full > split) ? (s_full - 1 - split) / a.nsplit + 1 : 0;
  const int64_t nfull = (DB && VEC) ? min(nf_all, cnt) : 0;   // full slabs come first
  const int64_t j_end = nfull & ~(int64_t)1;                   // an even number of them
  if (j_end > 0) {
    load_full(preA, wA, slab(0));
    // keep the two prologue slabs in issue order (A before B), as in the loop,
    // so that one wait count per chunk serves the first and later iterations
    __builtin_amdgcn_sched_barrier(0);
    load_full(preB, wB, slab(1));
    for (int64_t j = 0; j < j_end; j += 2) {
      store_slab(preA, wA, slab(j), lds0);
      lds_barrier();
      load_full(preA, wA, slab(min(j + 2, j_end - 1)));
      compute_slab(lds0);
      store_slab(preB, wB, slab(j + 1), lds1);
      lds_barrier();
      load_full(preB, wB, slab(min(j + 3, j_end - 1)));
      compute_slab(lds1);
    }
  }
  // ragged last slab, every slab when rows are not 16-byte aligned, and every
  // slab of the single-buffer variants
  if (j_end < cnt) {
    lds_barrier();
    for (int64_t j = j_end; j < cnt; ++j) {
      load_store_guarded(slab(j), lds0);
      lds_barrier();
      compute_slab(lds0);
      lds_barrier();
    }
  }

  // --- partial sub-tiles
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < nt) {
      const int R = a.sb * SI + ir[t], C = a.sb * SJ + ic[t];
      const size_t pidx = ((size_t)split * a.np + (size_t)(C * (C + 1) / 2 + R)) * 1024;
      if constexpr (IS_MFMA) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int j = lane & 31;
          if constexpr (BIN) reinterpret_cast<int*>(a.part)[pidx + i * 32 + j] = acc[t][r];
          else reinterpret_cast<float*>(a.part)[pidx + i * 32 + j] = acc[t][r];
        }
      } else {
        const int rr = (lane >> 3) * 4, cc = (lane & 7) * 4;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            reinterpret_cast<AccE*>(a.part)[pidx + (rr + i) * 32 + cc + j] = vacc[t][i * 4 + j];
      }
    }
  }

  // --- partial masses (rows of the I side of diagonal super-tiles)
  if (diag) {
    lds_barrier();
    for (int r = tid; r < rowsI; r += 512) {
      const int gr = 32 * a.sb * SI + r;
      if (gr < a.n) a.part_mass[(size_t)split * a.n + gr] = lmass[r];
    }
  }
}


// Launch one instantiation; the caller has checked that the combination is
// supported.  maxt: register tiles per wave (5 for one diagonal super-tile of
// 5..8 row blocks, else 2).
// LDS-staged Gram kernel (soft input, 16-bit MFMA types; rows 16-byte aligned
// and ending on a 16-byte boundary).  Super-tiles, splits, sub-tile runs, the
// MFMA loop and the outputs are those of gram_kernel; the loader differs.
// Each wave streams 32 rows of every slab (128 bytes per row) straight into a
// ring of NB LDS slots with loads to LDS, so NB - 1 slabs are in flight
// without holding registers.  Per slab, one pass converts the slot into the
// MFMA tile (isovalue model, sqrt(w), rounding) and adds the masses; the
// tile is then multiplied.  Rows past N, points past M and slabs past the
// split's share are read with an offset beyond the buffer's range: they land
// as zeros without a memory access, so no load sits under a branch that
// depends on the data and the wait counts are constants.
template <typename Tin, int MT, int MODE, int MAXT, bool WEIGHTED, int NB, int NT, int NW, bool GRP, int SEG>
// (at least 4 waves per SIMD: at most 128 VGPRs, so that two 8-wave
// workgroups can share a CU)
__global__ __launch_bounds__(64 * NW, 4) void gram_dma_kernel(GramArgs a) {
  using TR = MTraits<MT>;
  // SEG: bytes of a row per slab.  128 for up to 256 rows; 256 (FP32 input,
  // up to 128 rows) doubles the work between two barriers where the loader
  // evaluates a probability model on every value.
  static_assert(SEG == 128 || SEG == 256, "row segment");
  constexpr int EPC = 16 / (int)sizeof(Tin);  // elements per 16-byte chunk
  constexpr int KS = SEG / (int)sizeof(Tin);  // points per slab
  constexpr int ROWB = KS * TR::EB + 16;      // LDS tile row stride (padded)
  constexpr uint32_t OOB = 0x80000000u;
  constexpr int CPRW = SEG / 16;              // 16-byte chunks per row segment
  constexpr int RPI = 64 / CPRW;              // rows per load instruction (8 or 4)
  constexpr int RMAX = 256 * 128 / SEG;       // rows a workgroup stages at most
  constexpr int RW = RMAX / NW;               // staged rows per wave
  constexpr int LW = RW / RPI;                // row loads per slab and wave
  constexpr int NTH = 64 * NW;                // threads
  constexpr int DW = LW + (WEIGHTED ? 1 : 0); // loads per slab of wave 0 (rows, weights)
  static_assert(MT == MT_F16 || MT == MT_BF16 || MT == MT_BF16X3 || MT == MT_I8, "MFMA types");
  static_assert(MT != MT_I8 || (!WEIGHTED && MODE == MODE_STEP), "INT8: thresholded values, no weights");
  static_assert(KS % TR::KK == 0, "whole k-steps per slab");
  static_assert(KS <= 64, "weights of a slab: 64 per ring slot");
  static_assert(!GRP || SEG == 128, "grouped sub-tiles stage 256 rows");
  constexpr int CQ = (RMAX * CPRW + 64 * NW - 1) / (64 * NW);   // chunks per thread at most
  static_assert((NB - 2) * DW <= 63, "wait count");
  extern __shared__ __align__(16) unsigned char lds[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();

  // --- XCD-aware decode of the block index (as in gram_kernel)
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int q = b >> 3;
  const int st = q % a.ntiles_super;
  const int split = (q / a.ntiles_super) * 8 + xcd;
  int SI, SJ;
  super_ij(st, SI, SJ);
  const bool diag = GRP || (SI == SJ);   // (the grouped form has one, diagonal, super-tile)
  const int na = min(a.sb, a.nbt - a.sb * SI);
  const int nb = min(a.sb, a.nbt - a.sb * SJ);
  const int rowsI = 32 * na;
  const int rows = diag ? rowsI : rowsI + 32 * nb;
  const int PLANE = rows * ROWB;

  const int T = diag ? na * (na + 1) / 2 : na * nb;
  int nt;
  int ir[MAXT], ic[MAXT];
  // One diagonal super-tile of eight row blocks with 16 waves: groups of 2x2
  // blocks.  Wave g < 4 owns the diagonal group of blocks X = 2g, Y = X + 1
  // (sub-tiles XX, XY, YY); the two waves of an off-diagonal group (a, b),
  // a < b, own rows I = 2a + p against J = 2b and 2b + 1.  Either way the
  // wave's sub-tiles are (ir0, ic0), (ir0, ic1) [, (ic1, ic1)], so it reads
  // three fragments per k-step instead of two per sub-tile.
  // (GRP: the host has checked that the only super-tile is diagonal with
  // eight row blocks)
  static_assert(!GRP || (NW == 16 && MAXT >= 3), "grouped sub-tiles: 16 waves, 3 tiles");
  if constexpr (GRP) {
    if (wave < 4) {
      const int X = 2 * wave;
      ir[0] = X; ic[0] = X;
      ir[1] = X; ic[1] = X + 1;
      ir[2] = X + 1; ic[2] = X + 1;
      nt = 3;
    } else {
      const int o = (wave - 4) >> 1, p = (wave - 4) & 1;   // groups (0,1) (0,2) (1,2) (0,3) (1,3) (2,3)
      const int gb = (o >= 3) ? 3 : (o >= 1 ? 2 : 1);
      const int ga = o - gb * (gb - 1) / 2;
      const int I = 2 * ga + p;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) { ir[t] = I; ic[t] = 2 * gb + min(t, 1); }
      nt = 2;
    }
  } else {
    const int t0 = (wave * T) / NW, t1 = ((wave + 1) * T) / NW;
    nt = t1 - t0;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      int k = min(t0 + t, T - 1);
      if (diag) {
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= k) ++c;
        ic[t] = c;
        ir[t] = k - c * (c + 1) / 2;
      } else {
        ir[t] = k / nb;
        ic[t] = k % nb;
      }
    }
  }
  // slabs of this split (32-bit: the host keeps m * sizeof(Tin) below 2^31)
  const int cnt = (a.slabs > split) ? (int)((a.slabs - 1 - split) / a.nsplit + 1) : 0;
  auto grow = [&](int lrow) -> int {
    return (lrow < rowsI) ? (32 * a.sb * SI + lrow) : (32 * a.sb * SJ + lrow - rowsI);
  };

  // --- LDS: ring [NB][rows][SEG], NT tiles [PLANES][rows][ROWB], masses
  // [rows], weights [NB][64]
  unsigned char* stage = lds;
  unsigned char* tiles = stage + (size_t)NB * rows * SEG;
  auto tile_of = [&](int j) -> unsigned char* { return tiles + (size_t)(j % NT) * TR::PLANES * PLANE; };
  double* lmass = reinterpret_cast<double*>(tiles + (size_t)NT * TR::PLANES * PLANE);
  float* wsl = reinterpret_cast<float*>(lmass + rows);

  // --- loads: wave w streams staging rows [RW w, RW w + RW) (inside one
  // 32-row block, so all in the I or the J range), RPI rows per instruction
  const bool loader = RW * wave < rows;
  const int g0 = loader ? grow(RW * wave) : 0;            // first global row of the wave
  const int nvalid = loader ? max(0, min(RW, a.n - g0)) : 0;
  const Tin* Ub = reinterpret_cast<const Tin*>(a.U) + (int64_t)(nvalid > 0 ? g0 : 0) * a.ld;
  const BufRes rsU = make_bufres(Ub, (uint32_t)(((int64_t)max(nvalid - 1, 0) * a.ld + a.m) * (int64_t)sizeof(Tin)));
  const BufRes rsW = make_bufres(a.w, (uint32_t)(a.m * (int64_t)sizeof(float)));
  const uint32_t ldb = (uint32_t)(a.ld * (int64_t)sizeof(Tin));
  const int lr8 = lane / CPRW;               // row within an instruction
  const int lc = lane % CPRW;                // 16-byte chunk within the row segment
  // Per lane, fixed across slabs: the byte offset of its chunk within row
  // block i (OOB for rows past n) and the number of points left of its chunk.
  // Per slab, in scalar registers: the slab's byte offset in a row (the
  // loads' scalar offset) and its first point (past m for slabs beyond the
  // split's share).  All offsets stay below 2^32: OOB + slab offset < 2^31 +
  // m * sizeof(Tin) (the host keeps both below 2^31).
  uint32_t vrow[LW];
#pragma unroll
  for (int i = 0; i < LW; ++i) {
    const int r = RPI * i + lr8;
    vrow[i] = (r < nvalid) ? (uint32_t)r * ldb + (uint32_t)lc * 16u : OOB;
  }
  const int plim = (int)a.m - lc * EPC;      // chunk in range: first point of the slab < plim
  auto issue = [&](int j) {
    const int64_t s = split + (int64_t)j * a.nsplit;
    const bool ok = j < cnt;
    const uint32_t sbyte = ok ? (uint32_t)(s * SEG) : 0u;
    const int spt = ok ? (int)(s * KS) : INT_MAX;
    if (loader) {
      const bool pok = spt < plim;
#pragma unroll
      for (int i = 0; i < LW; ++i)
        dma_to_lds<16>(rsU, stage + ((size_t)(j % NB) * rows + RW * wave + RPI * i) * SEG, pok ? vrow[i] : OOB,
                       sbyte);
    }
    if constexpr (WEIGHTED) {
      if (wave == 0) {
        const bool wok = lane < KS && spt < (int)a.m - lane;
        dma_to_lds<4>(rsW, wsl + (size_t)(j % NB) * 64, wok ? (uint32_t)lane * 4u : OOB, sbyte / sizeof(Tin) * 4u);
      }
    }
  };
  // at most K slabs of this wave's loads still in flight
  auto wait_slab_n = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    if (WEIGHTED && wave == 0) vm_wait<K * DW>();
    else if (loader) vm_wait<K * LW>();
  };
  // the slab about to be used has landed (NB - 2 later ones may be in flight)
  auto wait_slab = [&]() { wait_slab_n(std::integral_constant<int, NB - 2>()); };

  // masses (diagonal super-tiles): a thread's chunks belong to the same rows
  // in every slab (row = (tid + NTH ci) / CPRW), so each lane adds its chunk
  // sum (FP32) to an FP64 register slab by slab; the CPRW lanes of a row are
  // added once at the end.
  double accm[CQ];
#pragma unroll
  for (int ci = 0; ci < CQ; ++ci) accm[ci] = 0.0;

  // Convert slot j (slab s) into its tile.  No contraction: sqrt(w) * u is
  // rounded to FP32 and then to the MFMA type in every kernel variant, so
  // results do not depend on which variant ran.
  auto convert = [&](int j) {
#pragma clang fp contract(off)
    const int64_t s = split + (int64_t)j * a.nsplit;
    const unsigned char* src = stage + (size_t)(j % NB) * rows * SEG;
    unsigned char* tile = tile_of(j);
    // every chunk of the thread is read before the first is converted, so
    // the LDS latency is paid once per slab
    Vec16<Tin> raws[CQ];
#pragma unroll
    for (int ci = 0; ci < CQ; ++ci) {
      // whole waves (rows * CPRW and NTH are multiples of 64): a scalar branch
      if (NTH * ci + 64 * wave < rows * CPRW) {
        const int qq = tid + NTH * ci;
        raws[ci] = *reinterpret_cast<const Vec16<Tin>*>(src + (size_t)(qq / CPRW) * SEG + (qq % CPRW) * 16);
      }
    }
#pragma unroll
    for (int ci = 0; ci < CQ; ++ci) {
      if (NTH * ci + 64 * wave >= rows * CPRW) break;
      const int qq = tid + NTH * ci;
      const int row = qq / CPRW, c = qq % CPRW;
      const Vec16<Tin>& raw = raws[ci];
      const int64_t x0 = s * KS + c * EPC;
      float msum = 0.f;
      float uv[EPC];
#pragma unroll
      for (int e = 0; e < EPC; ++e) uv[e] = extract_f<MODE, Tin, true>(raw.v[e], a.ex);
      if constexpr (MODE != MODE_NONE) {
        // the zeros read past the ends of the rows and of M went through the
        // model: cleared, in a wave-uniform branch that waves of inside
        // chunks skip (the empty asm keeps the compiler from turning it back
        // into selects on every value)
        const bool rv = grow(row) < a.n;
        const int lim = (int)min((int64_t)EPC, a.m - x0);   // points of the chunk inside M
        if (__builtin_amdgcn_ballot_w64(!(rv && lim == EPC)) != 0) {
          asm volatile("" ::: "memory");
#pragma unroll
          for (int e = 0; e < EPC; ++e) uv[e] = (rv && e < lim) ? uv[e] : 0.0f;
        }
      }
#pragma unroll
      for (int e = 0; e < EPC; ++e) {
        const float u = uv[e];
        if constexpr (WEIGHTED) {
          const float wv = wsl[(size_t)(j % NB) * 64 + c * EPC + e];
          msum = (e == 0) ? wv * u : msum + wv * u;
          uv[e] = sqrtf(wv) * u;
        } else {
          msum = (e == 0) ? u : msum + u;
          uv[e] = u;
        }
      }
      unsigned char* d = tile + (size_t)row * ROWB + (size_t)c * EPC * TR::EB;
      if constexpr (MT == MT_F16) {
        // a product is rounded to FP32 first (no fused convert); plain
        // values convert directly
        constexpr bool PRODUCT = WEIGHTED || MODE != MODE_NONE;
        f16 o[EPC];
#pragma unroll
        for (int e = 0; e < EPC; ++e) o[e] = PRODUCT ? to_f16_rounded(uv[e]) : (f16)uv[e];
        store_lds<2 * EPC>(d, o);
      } else if constexpr (MT == MT_BF16) {
        uint32_t o[EPC / 2];   // pairs of values, one conversion each
#pragma unroll
        for (int e = 0; e < EPC; e += 2) o[e / 2] = f32x2_to_bf16x2_bits(uv[e], uv[e + 1]);
        store_lds<2 * EPC>(d, o);
      } else if constexpr (MT == MT_I8) {
        int8_t o[EPC];   // the thresholded values are 0 or 1
#pragma unroll
        for (int e = 0; e < EPC; ++e) o[e] = (int8_t)(int)uv[e];
        store_lds<EPC>(d, o);
      } else {
        // pairs of values: hi rounded, the exact remainder rounded again
        uint32_t hi[EPC / 2], lo[EPC / 2];
#pragma unroll
        for (int e = 0; e < EPC; e += 2) {
          const uint32_t h = f32x2_to_bf16x2_bits(uv[e], uv[e + 1]);
          hi[e / 2] = h;
          lo[e / 2] = f32x2_to_bf16x2_bits(uv[e] - __uint_as_float(h << 16), uv[e + 1] - __uint_as_float(h & 0xffff0000u));
        }
        store_lds<2 * EPC>(d, hi);
        store_lds<2 * EPC>(d + PLANE, lo);
      }
      if (diag) accm[ci] += (double)msum;
    }
  };

  AccVec<MT> acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0;
  const int jrow_base = diag ? 0 : rowsI;
  auto multiply = [&](const unsigned char* tl) {
    if constexpr (GRP) mfma_slab_g<MT, KS, ROWB>(tl, PLANE, lane, nt == 3, ir[0], ic[0], ic[1], acc);
    else mfma_slab<MT, MAXT, KS, ROWB>(tl, PLANE, lane, nt, ir, ic, jrow_base, acc);
  };

  if constexpr (NT == 1) {
    // one tile: convert, barrier, multiply
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) issue(j);
    for (int j = 0; j < cnt; ++j) {
      wait_slab();
      lds_barrier();            // every wave's rows of slab j are in LDS; the tile is free
      issue(j + NB - 1);        // into the slot converted in the previous step
      convert(j);
      lds_barrier();            // the tile is complete
      multiply(tile_of(j));
    }
  } else {
    // two tiles: slab j + 1 is converted while slab j is multiplied, one
    // barrier per slab (it also separates the multiply of slab j - 1 from
    // the conversion that overwrites its tile)
#pragma unroll
    for (int j = 0; j < NB; ++j) issue(j);
    if (cnt > 0) {
      wait_slab_n(std::integral_constant<int, NB - 1>());
      lds_barrier();
      convert(0);
    }
    for (int j = 0; j < cnt; ++j) {
      wait_slab();              // slab j + 1
      lds_barrier();            // slab j + 1 is in LDS, tile j is complete, tile j + 1 is free
      issue(j + NB);            // into the slot of slab j, converted in the previous step
      if (j + 1 < cnt) convert(j + 1);
      multiply(tile_of(j));
    }
  }
  vm_wait<0>();               // no load into LDS outlives the workgroup
  // row sums to LDS: the CPRW lanes of a row (fixed butterfly), then lane c = 0
#pragma unroll
  for (int ci = 0; ci < CQ; ++ci) {
    if (NTH * ci + 64 * wave >= rows * CPRW) break;
    double t = accm[ci];
#pragma unroll
    for (int o = 1; o < CPRW; o <<= 1) t += __shfl_xor(t, o, 64);
    const int qq = tid + NTH * ci;
    if ((qq % CPRW) == 0) lmass[qq / CPRW] = t;
  }

  // --- partial sub-tiles
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    if (t < nt) {
      const int R = a.sb * SI + ir[t], C = a.sb * SJ + ic[t];
      const size_t pidx = ((size_t)split * a.np + (size_t)(C * (C + 1) / 2 + R)) * 1024;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int jj = lane & 31;
        if constexpr (MT == MT_I8) reinterpret_cast<int*>(a.part)[pidx + i * 32 + jj] = acc[t][r];
        else reinterpret_cast<float*>(a.part)[pidx + i * 32 + jj] = acc[t][r];
      }
    }
  }
  // --- partial masses (rows of the I side of diagonal super-tiles)
  if (diag) {
    lds_barrier();
    for (int r = tid; r < rowsI; r += NTH) {
      const int gr = 32 * a.sb * SI + r;
      if (gr < a.n) {
        a.part_mass[(size_t)split * a.n + gr] = lmass[r];
      }
    }
  }
}

// LDS bytes of gram_dma_kernel for a workgroup of `rows` staged rows.
template <typename Tin, int MT, int NT, int SEG>
constexpr int gram_dma_nb() {
  constexpr int KS = SEG / (int)sizeof(Tin);
  constexpr int ROWB = KS * MTraits<MT>::EB + 16;
  constexpr int RMAX = 256 * 128 / SEG;
  constexpr int fixed = NT * MTraits<MT>::PLANES * RMAX * ROWB + RMAX * 8 + 4 * 256;
  constexpr int nb = (163840 - fixed) / (RMAX * SEG + 256);
  return nb > 4 ? 4 : nb;
}
template <typename Tin, int MT, int NT, int SEG>
size_t gram_dma_lds(int rows, bool weighted) {
  constexpr int KS = SEG / (int)sizeof(Tin);
  constexpr int ROWB = KS * MTraits<MT>::EB + 16;
  constexpr int NB = gram_dma_nb<Tin, MT, NT, SEG>();
  return (size_t)NB * rows * SEG + (size_t)NT * MTraits<MT>::PLANES * rows * ROWB + (size_t)rows * 8 +
         (weighted ? (size_t)NB * 256 : 0);
}

// Launch the LDS-staged kernel when it applies (soft input in FP32, FP16 or
// BF16 with a 16-bit MFMA type, aligned rows ending on a 16-byte boundary,
// offsets within 2^31); returns false otherwise.
template <typename Tin, int MT, int MODE>
bool launch_gram_dma(const GramArgs& ga0, int maxt, int rows, int grid, hipStream_t st, const KernelTimer& tm) {
  if constexpr (!((MT == MT_F16 || MT == MT_BF16 || MT == MT_BF16X3 || (MT == MT_I8 && MODE == MODE_STEP)) &&
                  sizeof(Tin) <= 4 && sizeof(Tin) >= 2)) {
    return false;
  } else {
    constexpr int eb = sizeof(Tin);
    if (!ga0.vec || (ga0.m * eb) % 16 != 0) return false;
    if (((int64_t)31 * ga0.ld + ga0.m) * eb >= (INT64_C(1) << 31) || ga0.m * 4 >= (INT64_C(1) << 31)) return false;
    GramArgs ga = ga0;
    const bool w = ga.w != nullptr;
    auto go = [&](auto k, size_t lds, int threads) {
      (void)allow_dynamic_lds((const void*)k);   // set on the first launch of each kernel
      hipExtLaunchKernelGGL(k, dim3(grid), dim3(threads), (uint32_t)lds, st, tm.start(), tm.stop(), 0u, ga);
    };
    // 16 waves, one conversion tile, a ring of NB slabs; sub-tiles per wave:
    // at most 36 over 16 waves (3)
    constexpr int NT = 1;
    constexpr int NB = gram_dma_nb<Tin, MT, NT, 128>();
    static_assert(NB >= 2, "LDS ring");
    (void)maxt;
    ga.slabs = (ga0.m * eb + 127) / 128;   // 128-byte slabs of every row
    // launch with or without point weights (INT8 runs are unweighted: its
    // "weighted" kernel is the unweighted one, never launched as such)
    constexpr bool WW = MT != MT_I8;
    auto go_w = [&](auto kw, auto k, size_t lds, int threads) {
      if constexpr (MT == MT_I8) go(k, lds, threads);
      else if (w) go(kw, lds, threads);
      else go(k, lds, threads);
    };
    if constexpr (MODE == MODE_GAUSS && sizeof(Tin) == 4 && MT != MT_BF16X3) {
      // the Gaussian model on FP32 values, at most 128 rows: 8 waves and
      // about 76 KB of LDS, so that two workgroups share a CU (the plan
      // doubles the splits); each thread converts two chunks per slab.
      // (The BF16 split, with two tile planes, would not fit the 128
      // registers that this needs.)
      if (rows <= 128) {
        const size_t lds = gram_dma_lds<Tin, MT, NT, 128>(rows, w);
        go_w(gram_dma_kernel<Tin, MT, MODE, 3, WW, NB, NT, 8, false, 128>,
             gram_dma_kernel<Tin, MT, MODE, 3, false, NB, NT, 8, false, 128>, lds, 512);
        return true;
      }
    }
    if constexpr ((MODE == MODE_MODEL || MODE == MODE_STEP) && sizeof(Tin) == 4 && MT != MT_BF16X3) {
      // the piecewise-linear models or a threshold on FP32 values, at most
      // 128 rows: 256-byte row segments (twice the values between two
      // barriers; not for the BF16 split, whose two planes of a 64-point
      // tile would not fit the registers)
      if (rows <= 128) {
        constexpr int NB2 = gram_dma_nb<Tin, MT, NT, 256>();
        static_assert(NB2 >= 3, "LDS ring");
        ga.slabs = (ga0.m * eb + 255) / 256;
        const size_t lds = gram_dma_lds<Tin, MT, NT, 256>(rows, w);
        go_w(gram_dma_kernel<Tin, MT, MODE, 3, WW, NB2, NT, 16, false, 256>,
             gram_dma_kernel<Tin, MT, MODE, 3, false, NB2, NT, 16, false, 256>, lds, 1024);
        return true;
      }
    }
    // eight row blocks in one diagonal super-tile: grouped sub-tiles.  There
    // the BF16 split takes two conversion tiles (slab j + 1 is converted
    // while the three products of slab j run, one barrier per slab), which
    // leaves LDS for two ring slots: 64 against 74 us on 256 FP32 masks of
    // 512^2.  (The ungrouped kernels would spill with two tiles.)
    const bool grp = ga.nsuper == 1 && ga.nbt == 8;
    if (grp) {
      constexpr int NTG = (MT == MT_BF16X3) ? 2 : NT;
      constexpr int NBG = gram_dma_nb<Tin, MT, NTG, 128>();
      static_assert(NBG >= 2, "LDS ring");
      const size_t lds = gram_dma_lds<Tin, MT, NTG, 128>(rows, w);
      go_w(gram_dma_kernel<Tin, MT, MODE, 3, WW, NBG, NTG, 16, true, 128>,
           gram_dma_kernel<Tin, MT, MODE, 3, false, NBG, NTG, 16, true, 128>, lds, 1024);
    } else {
      const size_t lds = gram_dma_lds<Tin, MT, NT, 128>(rows, w);
      go_w(gram_dma_kernel<Tin, MT, MODE, 3, WW, NB, NT, 16, false, 128>,
           gram_dma_kernel<Tin, MT, MODE, 3, false, NB, NT, 16, false, 128>, lds, 1024);
    }
    return true;
  }
}

template <typename Tin, int MT, int MODE, bool W>
void launch_gram_w(const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st,
                   const KernelTimer& tm) {
  constexpr int EB = sizeof(Tin);
  constexpr int EPC = 16 / EB;
  constexpr int MB = (MT == MT_F16 || MT == MT_BF16 || MT == MT_BF16X3) ? 2 : (MT == MT_I8 ? 1 : (MT == MT_F32 ? 4 : 8));
  constexpr int CPR = (16 * EPC * MB <= 256) ? 16 : ((8 * EPC * MB <= 256) ? 8 : ((4 * EPC * MB <= 256) ? 4 : 2));
  constexpr int CH256 = (256 * CPR / 512) > 0 ? 256 * CPR / 512 : 1;   // chunk slots for 256 rows
  constexpr int CH128 = (128 * CPR / 512) > 0 ? 128 * CPR / 512 : 1;   // ... for 128 rows
  auto go = [&](auto k) {
    (void)allow_dynamic_lds((const void*)k);   // set on the first launch of each kernel
    hipExtLaunchKernelGGL(k, dim3(grid), dim3(512), (uint32_t)lds, st, tm.start(), tm.stop(), 0u, ga);
  };
  if (maxt > 2) go(gram_kernel<Tin, MT, MODE, 5, CPR, CH256, W>);
  else if (rows > 128) go(gram_kernel<Tin, MT, MODE, 2, CPR, CH256, W>);
  else go(gram_kernel<Tin, MT, MODE, 2, CPR, CH128, W>);
}

// Launch one instantiation; the caller has checked that the combination is
// supported.  maxt: register tiles per wave (5 for one diagonal super-tile of
// 5..8 row blocks, else 2).  INT8 runs are unweighted.
template <typename Tin, int MT, int MODE>
void launch_gram_t(const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st) {
  KernelTimer tm("gram", st, /*by_launch=*/true);
  if (launch_gram_dma<Tin, MT, MODE>(ga, maxt, rows, grid, st, tm)) return;
  if constexpr (MT == MT_I8) launch_gram_w<Tin, MT, MODE, false>(ga, maxt, rows, grid, lds, st, tm);
  else if (ga.w != nullptr) launch_gram_w<Tin, MT, MODE, true>(ga, maxt, rows, grid, lds, st, tm);
  else launch_gram_w<Tin, MT, MODE, false>(ga, maxt, rows, grid, lds, st, tm);
}

// Per-input-type dispatchers (one translation unit each); return false when
// the (MFMA type, extraction mode) combination is not provided.
bool gram_dispatch_f32(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_f16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_bf16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_f64(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_u8(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_model(int dtype, int mt, const GramArgs& ga, int maxt, int rows, int grid, size_t lds,
                         hipStream_t st);
}  // namespace pidk

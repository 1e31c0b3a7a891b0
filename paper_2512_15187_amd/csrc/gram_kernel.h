// Gram kernel template for the all-pairs PID numerators (see k_gram.hip for
// the algorithm); included by the per-input-type translation units.
#pragma once
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <type_traits>

namespace pidk {

// MFMA input flavours
enum MType { MT_F16 = 0, MT_BF16 = 1, MT_BF16X3 = 2, MT_I8 = 3, MT_F32 = 4, MT_F64 = 5 };

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
  double* part_mass;   // [nsplit][n]
};

// Super-tile index -> (I, J), I <= J, column-major over J.
__device__ __forceinline__ void super_ij(int t, int& I, int& J) {
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  J = j;
  I = t - j * (j + 1) / 2;
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
            else u = (AccE)extract_f<MODE>(pv.v[g + e], a.ex);
            if (!rvalid) u = AccE(0);
            if (!full) u = (x0 + g + e < a.m) ? u : AccE(0);
            if constexpr (WEIGHTED) { msum += (AccE)wv[g + e] * u; uv[e] = (AccE)sqrtf(wv[g + e]) * u; }
            else { msum += u; uv[e] = u; }
          }
          unsigned char* d4 = dst + (size_t)g * TR::EB;
          if constexpr (MT == MT_F16) {
            f16 o[G4];
#pragma unroll
            for (int e = 0; e < G4; ++e) o[e] = (f16)uv[e];
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
  using AccV = typename std::conditional<BIN, intx16, floatx16>::type;
  AccV acc[MAXT];
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
      constexpr int KSTEPS = KS / TR::KK;
      constexpr int FE = 16 / TR::EB;   // elements per lane per fragment (16 bytes)
      constexpr int KUNR = KSTEPS > 4 ? 4 : KSTEPS;   // bounded unroll: fragments stay few
#pragma unroll KUNR
      for (int kk = 0; kk < KSTEPS; ++kk) {
        const int koff = kk * TR::KK + (lane >> 5) * FE;   // element offset in the row
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
template <typename Tin, int MT, int MODE, bool W>
void launch_gram_w(const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st) {
  constexpr int EB = sizeof(Tin);
  constexpr int EPC = 16 / EB;
  constexpr int MB = (MT == MT_F16 || MT == MT_BF16 || MT == MT_BF16X3) ? 2 : (MT == MT_I8 ? 1 : (MT == MT_F32 ? 4 : 8));
  constexpr int CPR = (16 * EPC * MB <= 256) ? 16 : ((8 * EPC * MB <= 256) ? 8 : ((4 * EPC * MB <= 256) ? 4 : 2));
  constexpr int CH256 = (256 * CPR / 512) > 0 ? 256 * CPR / 512 : 1;   // chunk slots for 256 rows
  constexpr int CH128 = (128 * CPR / 512) > 0 ? 128 * CPR / 512 : 1;   // ... for 128 rows
  auto go = [&](auto k) {
    // allow up to 160 KB of LDS, once per kernel
    static const bool attr = (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  163840) == hipSuccess);
    (void)attr;
    hipLaunchKernelGGL(k, grid, 512, lds, st, ga);
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
  KernelTimer tm("gram", st);
  if constexpr (MT == MT_I8) launch_gram_w<Tin, MT, MODE, false>(ga, maxt, rows, grid, lds, st);
  else if (ga.w != nullptr) launch_gram_w<Tin, MT, MODE, true>(ga, maxt, rows, grid, lds, st);
  else launch_gram_w<Tin, MT, MODE, false>(ga, maxt, rows, grid, lds, st);
}

// Per-input-type dispatchers (one translation unit each); return false when
// the (MFMA type, extraction mode) combination is not provided.
bool gram_dispatch_f32(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_f16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_bf16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_f64(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_dispatch_u8(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st);
bool gram_supported(int dtype, int mt, int mode);

}  // namespace pidk

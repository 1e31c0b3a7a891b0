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
// Per tile the sums are FP32 (FP64 for FP64 input), across tiles FP64.
// Per-workgroup partials are reduced in a fixed order by pidmean_reduce, and
// pidmean_ratios forms the depths.  Binary input (U8 masks, thresholded
// values) takes the exact popcount passes of k_bits.hip instead.
#include "device_common.h"
#include <hip/hip_ext.h>
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

namespace pidk {

template <typename T>
using ComputeT = typename std::conditional<sizeof(T) == 8, double, float>::type;

// The piecewise-linear models (ramp, tent, density) are built for FP64, FP32
// and FP16 fields.
template <typename T>
constexpr bool has_models() {
  return std::is_same<T, double>::value || std::is_same<T, float>::value || std::is_same<T, f16>::value;
}

template <typename CT, typename T>
__device__ __forceinline__ CT to_ct(T raw) {
  if constexpr (std::is_same<CT, double>::value) return to_double(raw);
  else return to_float(raw);
}

template <int MODE, typename T, typename CT>
__device__ __forceinline__ CT extract_ct(T raw, const Extract& e) {
  if constexpr (std::is_same<CT, double>::value) return extract_d<MODE>(raw, e);
  else return extract_f<MODE, T, true>(raw, e);
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
    // A tile inside M on aligned rows (the same for the whole wave): every
    // member's load is unconditional, so that they are all in flight
    // together (a load under a branch of its own is waited for before the
    // next one is issued); rows past n re-read row n - 1 and stay out of
    // the sums.  Other tiles take guarded loads.
    const bool fast = VEC && (tile + 1) * TP <= m;
    Vec16<T> vv[MPW];
    if (fast) {
#pragma unroll
      for (int r = 0; r < MPW; ++r) vv[r] = load16_nt(U + (int64_t)min(mbase + r, n - 1) * ld + x0);
    } else {
#pragma unroll
      for (int r = 0; r < MPW; ++r) {
        Vec16<T> v{};
        if (mbase + r < n) v = load16_guarded(U + (int64_t)(mbase + r) * ld, x0, m);
        vv[r] = v;
      }
    }
    Vec16<T> raw[KEEP_RAW ? MPW : 1];
    CT u[KEEP_RAW ? 1 : MPW][PPL];
    CT sp[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) sp[p] = CT(0);
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const bool rv = mbase + r < n;   // (rows past n: their sums are never written)
      if constexpr (KEEP_RAW) {
        raw[r] = vv[r];
        if (rv) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) sp[p] += extract_ct<MODE, T, CT>(vv[r].v[p], ex);
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          CT val = rv ? extract_ct<MODE, T, CT>(vv[r].v[p], ex) : CT(0);
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
      if (fast) {   // PPL values, a multiple of 16 bytes at a 16-byte boundary
        static_assert((PPL * sizeof(CT)) % 16 == 0, "whole 16-byte loads");
#pragma unroll
        for (int q = 0; q < (int)(PPL * sizeof(CT) / 16); ++q) {
          const uint4 t = *reinterpret_cast<const uint4*>(sg + x0 + q * (16 / sizeof(CT)));
          __builtin_memcpy(&s[q * (16 / sizeof(CT))], &t, 16);
        }
      } else {
#pragma unroll
        for (int p = 0; p < PPL; ++p) s[p] = (x0 + p < m) ? sg[x0 + p] : CT(0);
      }
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
// Pipelined soft path (rows aligned to LB bytes, N <= NWMAX * MPW): the same sums
// as pidmean_soft_kernel, with a register double buffer.  Workgroup b takes
// the full tiles b, b + G, b + 2G, ... (G = grid); while one tile's column
// sums go through LDS and its members' sums are accumulated, the loads of
// the next tile are in flight.  The loop runs over pairs of tiles with no
// branch around a load, so the compiler's wait counts keep the other buffer
// outstanding: a tile past the workgroup's last one is read with an offset
// beyond the buffer's range, which the hardware answers with zeros and no
// memory access, and it adds nothing.  Rows past n re-read the wave's last
// row, and their copies are taken off the column sum.  The ragged last tile
// is taken afterwards, with guarded loads, by the workgroup it falls to.
// Soft masks keep the raw vectors and widen them twice; fields keep the
// extracted probabilities.
// part layout: [2][n][grid] doubles (m, then A).
template <typename T, int MODE, int MPW, int LB, bool WEIGHTED, int NWMAX>
__global__ __launch_bounds__(64 * NWMAX) void pidmean_pipe_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, const float* __restrict__ w,
    Extract ex, double* __restrict__ part) {
  using CT = ComputeT<T>;
  using V = VecB<T, LB>;
  constexpr int PPL = V::N;
  constexpr int TP = 64 * PPL;
  constexpr bool KEEP_RAW = (MODE == MODE_NONE);
  constexpr uint32_t OOB = 0x80000000u;   // beyond every buffer range used here
  extern __shared__ __align__(16) unsigned char smem_raw[];
  CT* sbuf = reinterpret_cast<CT*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int nw = blockDim.x >> 6;
  const int mbase = wave * MPW;
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int64_t nfull = m / TP;
  const int64_t K = (nfull > b) ? (nfull - 1 - b) / G + 1 : 0;   // full tiles of this workgroup

  // One buffer resource per wave, based at its first row; row r sits at
  // scalar offset min(r, rl) * ld, the points at a 32-bit per-lane offset.
  // The host has checked that every offset fits in 31 bits.
  const int rl = min(n - 1, mbase + MPW - 1) - mbase;            // last valid row of the wave
  const CT dup = (CT)(MPW - 1 - rl);                               // copies of row rl beyond it
  const __amdgpu_buffer_rsrc_t rsU = buffer_rsrc(
      U + (int64_t)mbase * ld, (uint32_t)(((int64_t)rl * ld + m) * (int64_t)sizeof(T)));
  const __amdgpu_buffer_rsrc_t rsW = buffer_rsrc(w, (uint32_t)(m * (int64_t)sizeof(float)));
  const uint32_t ldb0 = (uint32_t)(ld * (int64_t)sizeof(T));     // row stride in bytes
  const uint32_t xb = (uint32_t)b * TP + (uint32_t)(lane * PPL);
  const uint32_t xg = (uint32_t)G * TP;

  V bufA[MPW], bufB[MPW];
  float wA[WEIGHTED ? PPL : 1], wB[WEIGHTED ? PPL : 1];
  auto load_tile = [&](V* buf, float* wb, int64_t k) {
    const bool ok = k < K;
    const uint32_t x = xb + (uint32_t)k * xg;
    const uint32_t vo = ok ? x * (uint32_t)sizeof(T) : OOB;
    // row offsets recomputed per tile (a scalar multiply each) rather than
    // kept in scalar registers across the loop
    uint32_t ldb = ldb0;
    asm volatile("" : "+s"(ldb));
#pragma unroll
    for (int r = 0; r < MPW; ++r) buf[r] = bufload_nt<T, LB>(rsU, vo, (uint32_t)min(r, rl) * ldb);
    if constexpr (WEIGHTED) {
      // wave 0 reads the tile's weights (shared through LDS); the other
      // waves issue the same loads past the buffer's end (no memory access,
      // the same instructions, so the wait counts stay the same)
      constexpr int WB = PPL * 4 < 16 ? PPL * 4 : 16;   // bytes per weight load
      const uint32_t wo = (ok && wave == 0) ? x * 4u : OOB;
#pragma unroll
      for (int o = 0; o < PPL; o += WB / 4) {
        const VecB<float, WB> t = bufload_nt<float, WB>(rsW, wo + 4u * o, 0u);
#pragma unroll
        for (int p = 0; p < WB / 4; ++p) wb[o + p] = t.v[p];
      }
    }
  };

  // Per-lane sums run over at most 16 tiles; then each wave folds them
  // (fixed butterfly) into FP64 accumulators of its members in LDS, placed
  // after the two column-sum halves.  Lane 0 owns the wave's accumulators.
  CT accm[MPW], acca[MPW];
#pragma unroll
  for (int r = 0; r < MPW; ++r) { accm[r] = CT(0); acca[r] = CT(0); }
  double* lacc = reinterpret_cast<double*>(sbuf + (size_t)2 * nw * TP) + (size_t)wave * MPW * 2;
  float* wsh = reinterpret_cast<float*>(reinterpret_cast<double*>(sbuf + (size_t)2 * nw * TP) + (size_t)nw * MPW * 2);
                                                          // [2][TP] weights of the tile (wave 0's loads)
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < 2 * MPW; ++r) lacc[r] = 0.0;
  }
  auto fold = [&]() {
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const CT a = wave_sum(accm[r]);
      const CT c = wave_sum(acca[r]);
      if (lane == 0) { lacc[2 * r] += (double)a; lacc[2 * r + 1] += (double)c; }
      accm[r] = CT(0);
      acca[r] = CT(0);
    }
  };

  // One tile: column sums of the wave's members -> LDS half `parity`; after
  // the barrier every lane adds the NW partials for its points (fixed order)
  // and accumulates m_i and A_i of its members.  tv[p] = 0 marks a point past
  // the end (its raw value reads as zero; fields would turn it into
  // Phi(-c/sigma)); soft masks need no factor.
  auto process = [&](V* buf, const float* wb, int parity, const CT* tv) {
    CT u[KEEP_RAW ? 1 : MPW][PPL];
    CT sp[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) sp[p] = CT(0);
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        CT val = extract_ct<MODE, T, CT>(buf[r].v[p], ex);
        if constexpr (!KEEP_RAW) { val *= tv[p]; u[r][p] = val; }
        sp[p] += val;
      }
    }
    // take off the copies of row rl read for rows past n
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      CT last;
      if constexpr (KEEP_RAW) last = extract_ct<MODE, T, CT>(buf[MPW - 1].v[p], ex);
      else last = u[MPW - 1][p];
      sp[p] -= dup * last;
    }
    if constexpr (KEEP_RAW) {
#pragma unroll
      for (int r = 0; r < MPW; ++r) opaque(buf[r]);   // widen again below
    }
    CT* sb = sbuf + (size_t)parity * nw * TP;
#pragma unroll
    for (int p = 0; p < PPL; ++p) sb[wave * TP + lane * PPL + p] = sp[p];
    if constexpr (WEIGHTED) {
      if (wave == 0) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) wsh[(size_t)parity * TP + lane * PPL + p] = wb[p];
      }
    }
    lds_barrier();
    float wl[WEIGHTED ? PPL : 1];
    if constexpr (WEIGHTED) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) wl[p] = wsh[(size_t)parity * TP + lane * PPL + p];
    }
    CT s[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) s[p] = CT(0);
    for (int q = 0; q < nw; ++q) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] += sb[q * TP + lane * PPL + p];
    }
    if constexpr (WEIGHTED) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) s[p] *= (CT)wl[p];   // s now holds w * s
    }
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      CT tm = CT(0), ta = CT(0);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        CT uv;
        if constexpr (KEEP_RAW) uv = extract_ct<MODE, T, CT>(buf[r].v[p], ex);
        else uv = u[r][p];
        if constexpr (WEIGHTED) tm += (CT)wl[p] * uv;
        else tm += uv;
        ta += s[p] * uv;
      }
      accm[r] += tm;
      acca[r] += ta;
    }
  };

  // pairs of tiles; when K is odd the second tile of the last pair is past
  // the end and adds zeros
  load_tile(bufA, wA, 0);
  __builtin_amdgcn_sched_barrier(0);   // prologue loads in the loop's order (A, then B)
  load_tile(bufB, wB, 1);
  for (int64_t k = 0; k < K; k += 2) {
    CT one[PPL], second[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) { one[p] = CT(1); second[p] = (k + 1 < K) ? CT(1) : CT(0); }
    process(bufA, wA, 0, one);
    load_tile(bufA, wA, k + 2);
    process(bufB, wB, 1, second);
    load_tile(bufB, wB, k + 3);
    if ((k & 15) == 14 && k + 2 < K) fold();   // every 16 tiles, if more follow
  }
  // ragged last tile (LDS half 0 follows the loop's last tile, which used 1)
  if ((m % TP) != 0 && b == (int)(nfull % G)) {
    const int64_t x0 = nfull * TP + (int64_t)lane * PPL;
#pragma unroll
    for (int r = 0; r < MPW; ++r)
      bufA[r] = loadB_guarded<T, LB>(U + (int64_t)(mbase + min(r, rl)) * ld, x0, m);
    if constexpr (WEIGHTED) {
#pragma unroll
      for (int p = 0; p < PPL; ++p) wA[p] = w[(x0 + p < m) ? x0 + p : m - 1] * ((x0 + p < m) ? 1.0f : 0.0f);
    }
    CT pf[PPL];   // entries past m add nothing (fields would map 0 to Phi(-c/sigma))
#pragma unroll
    for (int p = 0; p < PPL; ++p) pf[p] = (x0 + p < m) ? CT(1) : CT(0);
    process(bufA, wA, 0, pf);
  }

  fold();
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < MPW; ++r) {
      const int i = mbase + r;
      if (i < n) {
        part[(size_t)i * G + b] = lacc[2 * r];
        part[((size_t)n + i) * G + b] = lacc[2 * r + 1];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// DMA-staged soft path (soft masks; rows 16-byte aligned, M * sizeof(T) a
// multiple of 16, N <= 8 * RPW).  Tiles hold TPP = 128 / sizeof(T) points of
// every row.  Each wave owns RPW rows and streams its 128-byte row segments of
// each tile straight into a ring of NBUF LDS slots (16 bytes per lane, eight
// rows per instruction), so NBUF - 1 tiles are in flight without holding
// registers, and no other wave reads them.  Per tile, a lane reads its point
// of the wave's rows from LDS for the wave's column sums, which go through
// LDS (one barrier), and again for m_i and A_i.  Loads of tiles past the
// workgroup's share, of rows past N and of points past M use an offset
// beyond the buffer's range: they write zeros and read no memory, so the
// loop has no branch around a load and the wait counts are constants.
// Lane sums run over at most 16 tiles and are then folded (fixed butterfly)
// into FP64 accumulators in LDS.  part layout: [2][n][grid] doubles.
template <typename T, bool WEIGHTED, int RPW, int NBUF>
__global__ __launch_bounds__(512) void pidmean_dma_kernel(
    const T* __restrict__ U, int64_t ld, int n, int64_t m, const float* __restrict__ w,
    double* __restrict__ part) {
  using CT = ComputeT<T>;
  constexpr int SEG = 128;                  // bytes of a row per tile
  constexpr int TPP = SEG / (int)sizeof(T); // points per tile
  constexpr int LPP = 64 / TPP;             // lanes per point
  constexpr int RPL = RPW / LPP;            // rows per lane
  constexpr int RPI = 64 * 16 / SEG;        // rows per load instruction (8)
  constexpr int DPT = RPW / RPI + (WEIGHTED ? 1 : 0);   // load instructions per tile and wave
  constexpr uint32_t OOB = 0x80000000u;
  static_assert(RPW % RPI == 0 && RPW % LPP == 0, "row split");
  static_assert((NBUF - 2) * DPT <= 63, "wait count");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int nw = blockDim.x >> 6;
  const int mbase = wave * RPW;
  const int nrows = min(RPW, n - mbase);    // valid rows of this wave (>= 1)
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int64_t ntiles = (m + TPP - 1) / TPP;
  const int64_t K = (ntiles > b) ? (ntiles - 1 - b) / G + 1 : 0;

  // LDS: raw ring [NBUF][nw][RPW][SEG], weights [NBUF][nw][64] floats,
  // column-sum partials [2][nw][TPP], FP64 accumulators [nw][RPW][2]
  unsigned char* raw = smem_raw;
  float* wts = reinterpret_cast<float*>(raw + (size_t)NBUF * nw * RPW * SEG);
  CT* psum = reinterpret_cast<CT*>(wts + (WEIGHTED ? (size_t)NBUF * nw * 64 : 0));
  double* lacc = reinterpret_cast<double*>(psum + (size_t)2 * nw * TPP) + (size_t)wave * RPW * 2;
  auto slot_raw = [&](int64_t k) -> unsigned char* {
    return raw + ((size_t)(k % NBUF) * nw + wave) * RPW * SEG;
  };
  auto slot_w = [&](int64_t k) -> float* { return wts + ((size_t)(k % NBUF) * nw + wave) * 64; };

  // resources based at the wave's first row; the host has checked that all
  // offsets stay below 2^31
  const BufRes rsU = make_bufres(U + (int64_t)mbase * ld, (uint32_t)(((int64_t)(nrows - 1) * ld + m) * (int64_t)sizeof(T)));
  const BufRes rsW = make_bufres(w, (uint32_t)(m * (int64_t)sizeof(float)));
  const uint32_t ldb = (uint32_t)(ld * (int64_t)sizeof(T));
  const int lrow = lane >> 3;               // row within a load instruction
  const uint32_t lbyte = (uint32_t)(lane & 7) * 16u;

  auto issue = [&](int64_t k) {
    const int64_t t = b + k * G;
    const bool tok = k < K;
    const uint32_t xb = (uint32_t)(t * SEG) + lbyte;                  // byte of the point in a row
    const bool pok = tok && (int64_t)(t * TPP) + (lane & 7) * (16 / (int)sizeof(T)) < m;
    unsigned char* dst = slot_raw(k);
#pragma unroll
    for (int j = 0; j < RPW / RPI; ++j) {
      const int r = j * RPI + lrow;
      const uint32_t vo = (pok && r < nrows) ? (uint32_t)r * ldb + xb : OOB;
      dma_to_lds<16>(rsU, dst + (size_t)j * RPI * SEG, vo);
    }
    if constexpr (WEIGHTED) {
      const int64_t x = t * TPP + lane;
      const uint32_t vo = (tok && lane < TPP && x < m) ? (uint32_t)(x * 4) : OOB;
      dma_to_lds<4>(rsW, slot_w(k), vo);
    }
  };

  CT accm[RPL], acca[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) { accm[i] = CT(0); acca[i] = CT(0); }
  if (lane == 0) {
    for (int r = 0; r < 2 * RPW; ++r) lacc[r] = 0.0;
  }
  const int pt = lane % TPP;                // this lane's point in a tile
  const int hr = lane / TPP;                // and its first row
  // members of a lane: rows hr + LPP * i; fold the TPP lanes of each row
  auto fold = [&]() {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      CT a = accm[i], c = acca[i];
#pragma unroll
      for (int o = TPP / 2; o >= 1; o >>= 1) { a += __shfl_xor(a, o, 64); c += __shfl_xor(c, o, 64); }
      if (pt == 0) {
        const int r = hr + LPP * i;
        lacc[2 * r] += (double)a;
        lacc[2 * r + 1] += (double)c;
      }
      accm[i] = CT(0);
      acca[i] = CT(0);
    }
  };

#pragma unroll
  for (int k = 0; k < NBUF - 1; ++k) issue(k);
  for (int64_t k = 0; k < K; ++k) {
    vm_wait<(NBUF - 2) * DPT>();            // this wave's loads of tile k have landed
    const unsigned char* rt = slot_raw(k);
    const int64_t x = (b + k * G) * TPP + pt;
    const bool pv = x < m;
    CT sp = CT(0);
#pragma unroll
    for (int i = 0; i < RPL; ++i)
      sp += to_ct<CT>(*reinterpret_cast<const T*>(rt + (size_t)(hr + LPP * i) * SEG + (size_t)pt * sizeof(T)));
    // the wave's rows (lanes pt, pt + TPP, ...)
    if constexpr (std::is_same<CT, float>::value) {
      sp = sum_from<TPP>(sp);
    } else {
#pragma unroll
      for (int o = TPP; o < 64; o <<= 1) sp += __shfl_xor(sp, o, 64);
    }
    CT* ps = psum + (size_t)(k & 1) * nw * TPP;
    if (hr == 0) ps[wave * TPP + pt] = pv ? sp : CT(0);
    lds_barrier();
    issue(k + NBUF - 1);                    // into the slot this wave finished with
    CT s = CT(0);
    for (int q = 0; q < nw; ++q) s += ps[q * TPP + pt];
    CT wv = CT(1);
    if constexpr (WEIGHTED) { wv = pv ? (CT)slot_w(k)[pt] : CT(0); s *= wv; }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      CT u = to_ct<CT>(*reinterpret_cast<const T*>(rt + (size_t)(hr + LPP * i) * SEG + (size_t)pt * sizeof(T)));
      u = pv ? u : CT(0);
      accm[i] += WEIGHTED ? wv * u : u;
      acca[i] += s * u;
    }
    if ((k & 15) == 15 && k + 1 < K) fold();
  }
  fold();
  vm_wait<0>();                             // no load into LDS outlives the workgroup
  if (lane == 0) {
    for (int r = 0; r < nrows; ++r) {
      part[(size_t)(mbase + r) * G + b] = lacc[2 * r];
      part[((size_t)n + mbase + r) * G + b] = lacc[2 * r + 1];
    }
  }
}

// ---------------------------------------------------------------------------
// 16 bytes of stored elements from an address that is 8-byte but not
// necessarily 16-byte aligned (rows whose byte length is a multiple of 8
// only): two 8-byte non-temporal loads.
template <typename T>
__device__ __forceinline__ Vec16<T> load16_nt8(const T* p) {
  struct Two { VecB<T, 8> a, b; };
  const Two t{loadB_nt<T, 8>(p), loadB_nt<T, 8>(p + 8 / sizeof(T))};
  return __builtin_bit_cast(Vec16<T>, t);
}

// ---------------------------------------------------------------------------
// Column sums over the members for the two-pass cases: s(x) = sum_j u_j(x)
// and, for all-pairs depths without the matrix, t(x) = sum_j coef_j u_j(x).
// Block (bx, g) owns 64 * PPL points (16 bytes of every row per lane) and the
// members [g chunk, (g + 1) chunk); its 4 waves take the members q, q + 4, ...
// of that range in ascending order, four rows in flight, and add their sums
// in order q = 0..3; the member groups' sums are added in order g = 0, 1, ...
// by colsum_combine.
template <typename T, int MODE, bool SCALED>
__global__ __launch_bounds__(256) void colsum_part_kernel(const T* __restrict__ U, int64_t ld, int n, int64_t m,
                                                          Extract ex, const ComputeT<T>* __restrict__ coef,
                                                          int chunk, void* __restrict__ part_v, int vec) {
  using CT = ComputeT<T>;
  using AT = CT;
  constexpr int PPL = Vec16<T>::N;
  __shared__ AT part[4][64 * PPL];
  const int lane = threadIdx.x & 63;
  const int q = threadIdx.x >> 6;
  const int64_t x0 = (int64_t)blockIdx.x * (64 * PPL) + (int64_t)lane * PPL;
  const bool full = vec == 2 && x0 + PPL <= m;   // rows 16-byte aligned
  const bool half = vec == 1 && x0 + PPL <= m;   // rows 8-byte aligned
  const int i0 = blockIdx.y * chunk, i1 = min(n, i0 + chunk);
  AT t[PPL];
#pragma unroll
  for (int p = 0; p < PPL; ++p) t[p] = AT(0);
  auto row = [&](int i) -> Vec16<T> {
    const T* r = U + (int64_t)i * ld;
    return full ? load16_nt(r + x0) : (half ? load16_nt8(r + x0) : load16_guarded(r, x0, m));
  };
  auto add = [&](int i, const Vec16<T>& v) {
    const CT c = SCALED ? coef[i] : CT(1);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const CT u = extract_ct<MODE, T, CT>(v.v[p], ex);
      t[p] += SCALED ? c * u : u;
    }
  };
  // vector loads of four rows in flight; element loads (unaligned rows, the
  // ragged end of a row) one row at a time
  auto rowv = [&](int i) -> Vec16<T> {
    const T* r = U + (int64_t)i * ld;
    return full ? load16_nt(r + x0) : load16_nt8(r + x0);
  };
  int i = i0 + q;
  if (full || half) {
    for (; i + 12 < i1; i += 16) {
      const Vec16<T> a0 = rowv(i), a1 = rowv(i + 4), a2 = rowv(i + 8), a3 = rowv(i + 12);
      add(i, a0); add(i + 4, a1); add(i + 8, a2); add(i + 12, a3);
    }
  }
  for (; i < i1; i += 4) add(i, row(i));
#pragma unroll
  for (int p = 0; p < PPL; ++p) part[q][lane * PPL + p] = t[p];
  __syncthreads();
  AT* out = reinterpret_cast<AT*>(part_v) + (size_t)blockIdx.y * m;
  for (int e = threadIdx.x; e < 64 * PPL; e += 256) {
    const int64_t x = (int64_t)blockIdx.x * (64 * PPL) + e;
    if (x < m) out[x] = ((part[0][e] + part[1][e]) + part[2][e]) + part[3][e];
  }
}

template <typename AT>
__global__ __launch_bounds__(256) void colsum_combine(const AT* __restrict__ part, int groups, int64_t m,
                                                      AT* __restrict__ out) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < m; x += (int64_t)gridDim.x * blockDim.x) {
    AT s = part[x];
    for (int g = 1; g < groups; ++g) s += part[(size_t)g * m + x];
    out[x] = s;
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reduction of the per-workgroup partials: one block per member
// and quantity (grid.y = 2: m, then A); thread t sums the partials
// t, t+256, ... in ascending order, then a fixed tree over the 256 threads.
__global__ __launch_bounds__(256) void pidmean_reduce(const double* __restrict__ part, int nparts, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x, q = blockIdx.y, t = threadIdx.x;
  const size_t base = ((size_t)q * n + i) * nparts;
  double s = 0.0;
  for (int b = t; b < nparts; b += 256) s += part[base + b];
  red[t] = s;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) out[(size_t)q * n + i] = red[0];
}

// One block per 256 members: every block forms the total mass with the
// same fixed tree (the same value in each), then the ratios of Sec. 4.1 and
// the depth of its members.
__global__ __launch_bounds__(256) void pidmean_ratios(const double* __restrict__ red_v, int n,
                                                      double* __restrict__ m_out,
                                                      double* __restrict__ in_in,
                                                      double* __restrict__ in_out,
                                                      double* __restrict__ depth) {
#pragma clang fp contract(off)
  __shared__ double red[256];
  const int t = threadIdx.x;
  double md = 0.0;
  for (int i = t; i < n; i += 256) md += red_v[i];
  red[t] = md;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const int i = blockIdx.x * 256 + t;
  if (i < n) {
    const double mm = red_v[i], a = red_v[n + i], tot = red[0];
    const double ii = (mm > 0.0) ? a / ((double)n * mm) : 0.0;
    const double oo = (tot > 0.0) ? a / tot : 0.0;
    if (m_out) m_out[i] = mm;
    if (in_in) in_in[i] = ii;
    if (in_out) in_out[i] = oo;
    if (depth) depth[i] = ii < oo ? ii : oo;
  }
}

// ---------------------------------------------------------------------------
// All-pairs depths in O(N M) (no inclusion matrix).  With G_ji = sum_x w u_j u_i
// (Sec. 3.2 / 3.4),
//   IN_out(i) = (1/N) sum_j G_ji / m_j = (1/N) sum_x w u_i(x) t(x),
//   t(x) = sum_j u_j(x) / m_j   (terms with m_j = 0 are 0),
// so IN_out needs one column sum weighted by the inverse masses and one row
// dot product; IN_in(i) = S_i / (N m_i) is the PID-mean IN_in (Sec. 4.1).

// Inverse masses (0 for m = 0) in the compute type of the passes.
template <typename CT>
__global__ __launch_bounds__(256) void inv_mass_kernel(const double* __restrict__ mass, int n,
                                                       CT* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) coef[i] = mass[i] > 0.0 ? (CT)(1.0 / mass[i]) : CT(0);
}

// red = [m (n), B (n)] with B_i = sum_x w u_i t; in_in from the PID-mean pass.
__global__ __launch_bounds__(256) void pairs_linear_ratios(const double* __restrict__ red,
                                                           const double* __restrict__ in_in_pm, int n,
                                                           double* __restrict__ m_out, double* __restrict__ in_in,
                                                           double* __restrict__ in_out, double* __restrict__ depth) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ii = in_in_pm[i];
  const double oo = red[n + i] / (double)n;
  if (m_out) m_out[i] = red[i];
  if (in_in) in_in[i] = ii;
  if (in_out) in_out[i] = oo;
  if (depth) depth[i] = ii < oo ? ii : oo;
}

// ---------------------------------------------------------------------------
// Host side: plan, workspace and launch.

template <typename T, int MODE, int MPW, bool W, int NWMAX>
static void launch_soft_one(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                            int nwaves, const void* sglob, double* part, hipStream_t st, const KernelTimer& tm) {
  const size_t lds = (size_t)2 * nwaves * (64 * Vec16<T>::N) * sizeof(ComputeT<T>);
  hipExtLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, W, false, NWMAX>), dim3(p.grid), dim3(64 * nwaves),
                        (uint32_t)lds, st, tm.start(), tm.stop(), 0u, reinterpret_cast<const T*>(e.data), e.ld, (int)e.n, e.m, e.weights, ex,
                     p.ntiles, sglob, part, vec ? 1 : 0);
}

template <typename T, int MODE, int MPW>
static void launch_soft_t(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                          const void* sglob, double* part, hipStream_t st) {
  const T* U = reinterpret_cast<const T*>(e.data);
  const bool wtd = e.weights != nullptr;
  KernelTimer tm("pidmean", st, /*by_launch=*/true);   // one kernel per call
  if (p.pipe_lb) {   // the plan picks the pipelined kernel only where it is instantiated
    if constexpr (MODE != MODE_STEP && !std::is_same<T, uint8_t>::value && !(sizeof(T) == 8 && MPW == 32) &&
                  !(sizeof(T) == 2 && (MODE == MODE_GAUSS || MODE == MODE_MODEL)) && MPW != 16) {
      constexpr int LB = (MPW == 4) ? 16 : (MPW == 8 ? 8 : 4);
      constexpr int NWM = (MPW == 32) ? 8 : 16;
      if (wtd)
        hipExtLaunchKernelGGL((pidmean_pipe_kernel<T, MODE, MPW, LB, true, NWM>), dim3(p.pipe_grid),
                              dim3(64 * p.nwaves), (uint32_t)p.lds_bytes, st, tm.start(), tm.stop(), 0u, U, e.ld, (int)e.n, e.m, e.weights, ex, part);
      else
        hipExtLaunchKernelGGL((pidmean_pipe_kernel<T, MODE, MPW, LB, false, NWM>), dim3(p.pipe_grid),
                              dim3(64 * p.nwaves), (uint32_t)p.lds_bytes, st, tm.start(), tm.stop(), 0u, U, e.ld, (int)e.n, e.m, e.weights, ex, part);
    }
    return;
  }
  if constexpr (MPW != 32) {
    dim3 grid(p.grid, p.two_pass ? p.groups : 1);
    dim3 block(64 * p.nwaves);
    if (p.two_pass) {
      if (wtd)
        hipExtLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, true, true, 8>), grid, block, 0u, st, tm.start(), tm.stop(), 0u, U,
                           e.ld, (int)e.n, e.m, e.weights, ex, p.ntiles, sglob, part, vec ? 1 : 0);
      else
        hipExtLaunchKernelGGL((pidmean_soft_kernel<T, MODE, MPW, false, true, 8>), grid, block, 0u, st, tm.start(), tm.stop(), 0u, U,
                           e.ld, (int)e.n, e.m, e.weights, ex, p.ntiles, sglob, part, vec ? 1 : 0);
      return;
    }
    // single pass; 16 waves only where N needs them.  The plan gives U8 and
    // FP64 input at most 8 waves, so their 16-wave variants are not built (a
    // larger block would fail at launch, reported by the caller's check).
    if constexpr (sizeof(T) == 4 || sizeof(T) == 2) {
      if (p.nwaves > 8) {
        if (wtd) launch_soft_one<T, MODE, MPW, true, 16>(p, e, ex, vec, p.nwaves, sglob, part, st, tm);
        else launch_soft_one<T, MODE, MPW, false, 16>(p, e, ex, vec, p.nwaves, sglob, part, st, tm);
        return;
      }
    }
    if (wtd) launch_soft_one<T, MODE, MPW, true, 8>(p, e, ex, vec, p.nwaves, sglob, part, st, tm);
    else launch_soft_one<T, MODE, MPW, false, 8>(p, e, ex, vec, p.nwaves, sglob, part, st, tm);
  }
}

// Row alignment for the loads of the column-sum kernel: 2 when
// every row is 16-byte aligned (vec), 1 when 8-byte aligned, else 0.
template <typename T>
static int row_align(const pid_ensemble& e, bool vec) {
  if (vec) return 2;
  return ((reinterpret_cast<uintptr_t>(e.data) & 7) == 0 && (e.ld * (int64_t)sizeof(T)) % 8 == 0) ? 1 : 0;
}

template <typename T, int MODE>
static void dispatch_mpw(const MeanPlan& p, const pid_ensemble& e, const Extract& ex, bool vec,
                         const void* sglob, void* part, hipStream_t st) {
  switch (p.mpw) {
    case 4: launch_soft_t<T, MODE, 4>(p, e, ex, vec, sglob, (double*)part, st); break;
    case 8: launch_soft_t<T, MODE, 8>(p, e, ex, vec, sglob, (double*)part, st); break;
    case 32: launch_soft_t<T, MODE, 32>(p, e, ex, vec, sglob, (double*)part, st); break;
    default: launch_soft_t<T, MODE, 16>(p, e, ex, vec, sglob, (double*)part, st); break;
  }
}

template <typename T>
static void dispatch_mode(const MeanPlan& p, const pid_ensemble& e, int iso_kind, const Extract& ex,
                          bool vec, const void* sglob, void* part, hipStream_t st) {
  switch (iso_kind) {
    case PID_ISO_GAUSSIAN: dispatch_mpw<T, MODE_GAUSS>(p, e, ex, vec, sglob, part, st); break;
    case PID_ISO_STEP: dispatch_mpw<T, MODE_STEP>(p, e, ex, vec, sglob, part, st); break;
    case PID_ISO_RAMP: case PID_ISO_TENT: case PID_ISO_DENSITY:
      if constexpr (has_models<T>()) dispatch_mpw<T, MODE_MODEL>(p, e, ex, vec, sglob, part, st);
      break;
    default: dispatch_mpw<T, MODE_NONE>(p, e, ex, vec, sglob, part, st); break;
  }
}

template <typename T, int MODE, bool SCALED>
static void launch_colsum_g(const pid_ensemble& e, const Extract& ex, int groups, const void* coef, void* gpart,
                            void* sout, bool vec, hipStream_t st) {
  using CT = ComputeT<T>;
  using AT = CT;
  constexpr int PPL = Vec16<T>::N;
  const T* U = reinterpret_cast<const T*>(e.data);
  const dim3 grid((unsigned)((e.m + 64 * PPL - 1) / (64 * PPL)), (unsigned)groups);
  const int chunk = (int)((e.n + groups - 1) / groups);
  KernelTimer tm("pidmean_colsum", st);
  void* dst = groups > 1 ? gpart : sout;
  hipLaunchKernelGGL((colsum_part_kernel<T, MODE, SCALED>), grid, 256, 0, st, U, e.ld, (int)e.n, e.m, ex,
                     (const CT*)coef, chunk, dst, row_align<T>(e, vec));
  if (groups > 1) {
    const int cgrid = (int)std::min<int64_t>((e.m + 255) / 256, device_cu_count() * 8);
    hipLaunchKernelGGL(colsum_combine<AT>, cgrid, 256, 0, st, (const AT*)gpart, groups, e.m, (AT*)sout);
  }
}

template <typename T>
static void launch_colsum(const MeanPlan& p, const pid_ensemble& e, int iso_kind, const Extract& ex,
                          void* sout, void* gpart, bool vec, hipStream_t st) {
  const int g = p.colsum_groups;
  if (iso_kind == PID_ISO_GAUSSIAN) {
    launch_colsum_g<T, MODE_GAUSS, false>(e, ex, g, nullptr, gpart, sout, vec, st);
  } else if (iso_mode(iso_kind) == MODE_MODEL) {
    if constexpr (has_models<T>()) launch_colsum_g<T, MODE_MODEL, false>(e, ex, g, nullptr, gpart, sout, vec, st);
  } else if (iso_kind == PID_ISO_STEP) {
    launch_colsum_g<T, MODE_STEP, false>(e, ex, g, nullptr, gpart, sout, vec, st);
  } else {
    launch_colsum_g<T, MODE_NONE, false>(e, ex, g, nullptr, gpart, sout, vec, st);
  }
}

static hipError_t launch_mean_finalize(const MeanPlan& p, const pid_ensemble& e, void* part, void* red,
                                       int nparts, const pid_out& out, hipStream_t st) {
  KernelTimer tm("pidmean_finalize", st);
  dim3 rgrid((unsigned)e.n, 2);
  hipLaunchKernelGGL(pidmean_reduce, rgrid, 256, 0, st, (const double*)part, nparts, (int)e.n, (double*)red);
  hipLaunchKernelGGL(pidmean_ratios, (int)((e.n + 255) / 256), 256, 0, st, (const double*)red, (int)e.n, out.mass, out.in_in, out.in_out,
                     out.depth);
  return hipGetLastError();
}

template <typename T>
static void launch_dma(const MeanPlan& p, const pid_ensemble& e, double* part, hipStream_t st) {
  const T* U = reinterpret_cast<const T*>(e.data);
  KernelTimer tm("pidmean", st, /*by_launch=*/true);
  auto go = [&](auto kern) {
    (void)allow_dynamic_lds((const void*)kern);   // set on the first launch of each kernel
    hipExtLaunchKernelGGL(kern, dim3(p.dma_grid), dim3(64 * p.dma_nwaves), (uint32_t)p.dma_lds, st, tm.start(),
                          tm.stop(), 0u, U, e.ld, (int)e.n, e.m,
                       e.weights, part);
  };
  const bool wtd = e.weights != nullptr;
  if (wtd) go(pidmean_dma_kernel<T, true, 32, 4>);
  else go(pidmean_dma_kernel<T, false, 32, 4>);
}

hipError_t launch_pid_mean(const MeanPlan& plan, const pid_ensemble& e, int iso_kind,
                           const ExtractHost& exh, const pid_out& out, void* ws, hipStream_t st) {
  if (plan.bits) return launch_mask_bits_mean(e, iso_kind, exh, out, ws, st);
  Extract ex = __builtin_bit_cast(Extract, exh);
  Carve c(ws);
  void* part = c.take<double>((size_t)std::max(std::max(plan.grid, plan.pipe_grid), plan.dma_grid) * 2 * e.n);
  void* red = c.take<double>((size_t)2 * e.n);
  void* sbuf = plan.two_pass ? (void*)c.take<double>((size_t)e.m) : nullptr;
  void* gpart = plan.two_pass ? (void*)c.take<double>((size_t)e.m * (size_t)plan.colsum_groups) : nullptr;
  const int eb = elem_bytes_of(e.dtype);
  const bool vec = ((reinterpret_cast<uintptr_t>(e.data) & 15) == 0) && ((e.ld * eb) % 16 == 0) &&
                   (e.weights == nullptr || (reinterpret_cast<uintptr_t>(e.weights) & 15) == 0);
  // the pipelined kernel needs aligned rows and buffer offsets (one wave's
  // rows, the weights) below 2^31; otherwise the unpipelined kernel runs
  MeanPlan p = plan;
  if (p.dma_rpw) {
    const bool fits = ((int64_t)(p.dma_rpw - 1) * e.ld + e.m) * eb < (INT64_C(1) << 31) &&
                      e.m * (int64_t)sizeof(float) < (INT64_C(1) << 31);
    if (vec && fits) {
      switch (e.dtype) {
        case PID_F64: launch_dma<double>(p, e, (double*)part, st); break;
        case PID_F32: launch_dma<float>(p, e, (double*)part, st); break;
        case PID_F16: launch_dma<f16>(p, e, (double*)part, st); break;
        default: launch_dma<bf16_t>(p, e, (double*)part, st); break;
      }
      hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
      return launch_mean_finalize(p, e, part, red, p.dma_grid, out, st);
    }
  }
  if (p.pipe_lb) {
    const bool fits = ((int64_t)(p.mpw - 1) * e.ld + e.m) * eb < (INT64_C(1) << 31) &&
                      e.m * (int64_t)sizeof(float) < (INT64_C(1) << 31);
    if (!(vec && fits)) { p.pipe_lb = 0; p.mpw = p.fb_mpw; p.nwaves = p.fb_nwaves; }
  }
  const int nparts = p.pipe_lb ? p.pipe_grid : p.grid;
  switch (e.dtype) {
    case PID_F64:
      if (p.two_pass) launch_colsum<double>(p, e, iso_kind, ex, sbuf, gpart, vec, st);
      dispatch_mode<double>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_F32:
      if (p.two_pass) launch_colsum<float>(p, e, iso_kind, ex, sbuf, gpart, vec, st);
      dispatch_mode<float>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_F16:
      if (p.two_pass) launch_colsum<f16>(p, e, iso_kind, ex, sbuf, gpart, vec, st);
      dispatch_mode<f16>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    case PID_BF16:
      if (p.two_pass) launch_colsum<bf16_t>(p, e, iso_kind, ex, sbuf, gpart, vec, st);
      dispatch_mode<bf16_t>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
    default:
      if (p.two_pass) launch_colsum<uint8_t>(p, e, iso_kind, ex, sbuf, gpart, vec, st);
      dispatch_mode<uint8_t>(p, e, iso_kind, ex, vec, sbuf, part, st); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_mean_finalize(p, e, part, red, nparts, out, st);
}


// ---------------------------------------------------------------------------
// All-pairs depths without the inclusion matrix: the PID-mean pass (masses,
// IN_in), then t = sum_j u_j / m_j into memory, then B_i = sum_x w u_i t with
// the two-pass row kernel (soft arithmetic, also for binary input).
template <typename T>
static void launch_linear_t(const pid_ensemble& e, int iso_kind, const Extract& ex, bool vec, const MeanPlan& p3,
                            void* coef, int tg, void* tpart, void* tbuf, double* part, hipStream_t st) {
  if (iso_kind == PID_ISO_GAUSSIAN) launch_colsum_g<T, MODE_GAUSS, true>(e, ex, tg, coef, tpart, tbuf, vec, st);
  else if (iso_kind == PID_ISO_STEP) launch_colsum_g<T, MODE_STEP, true>(e, ex, tg, coef, tpart, tbuf, vec, st);
  else if (iso_mode(iso_kind) == MODE_MODEL) {
    if constexpr (has_models<T>()) launch_colsum_g<T, MODE_MODEL, true>(e, ex, tg, coef, tpart, tbuf, vec, st);
  } else launch_colsum_g<T, MODE_NONE, true>(e, ex, tg, coef, tpart, tbuf, vec, st);
  if (iso_kind == PID_ISO_GAUSSIAN) dispatch_mpw<T, MODE_GAUSS>(p3, e, ex, vec, tbuf, part, st);
  else if (iso_kind == PID_ISO_STEP) dispatch_mpw<T, MODE_STEP>(p3, e, ex, vec, tbuf, part, st);
  else if (iso_mode(iso_kind) == MODE_MODEL) {
    if constexpr (has_models<T>()) dispatch_mpw<T, MODE_MODEL>(p3, e, ex, vec, tbuf, part, st);
  } else dispatch_mpw<T, MODE_NONE>(p3, e, ex, vec, tbuf, part, st);
}

hipError_t launch_pairs_linear(const pid_ensemble& e, int iso_kind, const ExtractHost& exh, const pid_out& out,
                               void* ws, hipStream_t st) {
  const MeanPlan p1 = mean_plan(e.n, e.m, e.dtype, iso_kind, e.weights != nullptr);
  const MeanPlan p3 = rows_plan(e.n, e.m, e.dtype);
  Carve c(ws);
  void* ws1 = c.take<char>(mean_workspace(p1, e.n, e.m));
  double* mass = c.take<double>((size_t)e.n);
  double* inin = c.take<double>((size_t)e.n);
  void* coef = c.take<double>((size_t)e.n);
  void* tbuf = c.take<double>((size_t)e.m);
  const int tg = colsum_groups(e.n, e.m, elem_bytes_of(e.dtype));
  void* tpart = c.take<double>((size_t)e.m * (size_t)tg);
  double* part = c.take<double>((size_t)p3.grid * 2 * e.n);
  double* red = c.take<double>((size_t)2 * e.n);
  // pass 1: masses and IN_in
  pid_out o1{};
  o1.mass = mass;
  o1.in_in = inin;
  hipError_t err = launch_pid_mean(p1, e, iso_kind, exh, o1, ws1, st);
  if (err != hipSuccess) return err;
  // coefficients 1 / m_j
  const bool dbl = e.dtype == PID_F64;
  if (dbl)
    hipLaunchKernelGGL(inv_mass_kernel<double>, (int)((e.n + 255) / 256), 256, 0, st, mass, (int)e.n, (double*)coef);
  else
    hipLaunchKernelGGL(inv_mass_kernel<float>, (int)((e.n + 255) / 256), 256, 0, st, mass, (int)e.n, (float*)coef);
  // passes 2 and 3: t, then B
  Extract ex = __builtin_bit_cast(Extract, exh);
  const int eb = elem_bytes_of(e.dtype);
  const bool vec = ((reinterpret_cast<uintptr_t>(e.data) & 15) == 0) && ((e.ld * eb) % 16 == 0) &&
                   (e.weights == nullptr || (reinterpret_cast<uintptr_t>(e.weights) & 15) == 0);
  switch (e.dtype) {
    case PID_F64: launch_linear_t<double>(e, iso_kind, ex, vec, p3, coef, tg, tpart, tbuf, part, st); break;
    case PID_F32: launch_linear_t<float>(e, iso_kind, ex, vec, p3, coef, tg, tpart, tbuf, part, st); break;
    case PID_F16: launch_linear_t<f16>(e, iso_kind, ex, vec, p3, coef, tg, tpart, tbuf, part, st); break;
    case PID_BF16: launch_linear_t<bf16_t>(e, iso_kind, ex, vec, p3, coef, tg, tpart, tbuf, part, st); break;
    default: launch_linear_t<uint8_t>(e, iso_kind, ex, vec, p3, coef, tg, tpart, tbuf, part, st); break;
  }
  err = hipGetLastError();
  if (err != hipSuccess) return err;
  KernelTimer tm("pidmean_finalize", st);
  dim3 rgrid((unsigned)e.n, 2);
  hipLaunchKernelGGL(pidmean_reduce, rgrid, 256, 0, st, part, p3.grid, (int)e.n, red);
  hipLaunchKernelGGL(pairs_linear_ratios, (int)((e.n + 255) / 256), 256, 0, st, red, inin, (int)e.n, out.mass,
                     out.in_in, out.in_out, out.depth);
  return hipGetLastError();
}

}  // namespace pidk

namespace pidk {

// ---------------------------------------------------------------------------
// PID-mean against a reliability-weighted mean contour (Sec. 4.1, the
// optional weighting of the point-wise mean):
//   ubar = s_r / R,  s_r(x) = sum_j r_j u_j(x),  R = sum_j r_j,
//   A_i = sum_x w u_i(x) s_r(x)  =>  u_i <_p ubar = A_i / (R m_i),
//   m(ubar) = sum_j r_j m_j / R  =>  ubar <_p u_i = A_i / sum_j r_j m_j.
// Two streaming passes: s_r into the workspace (the column-sum kernel with
// the weights as coefficients), then m_i and A_i by the two-pass row kernel.

template <typename CT>
__global__ __launch_bounds__(256) void member_coef_kernel(const double* __restrict__ r, int n, CT* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = (CT)r[i];
}

// One block: R and sum_j r_j m_j by a fixed tree, then the ratios.  R <= 0
// (no positive weight) gives zero depths.
__global__ __launch_bounds__(256) void pidmean_weighted_ratios(const double* __restrict__ red,
                                                               const double* __restrict__ r, int n,
                                                               double* __restrict__ m_out,
                                                               double* __restrict__ in_in,
                                                               double* __restrict__ in_out,
                                                               double* __restrict__ depth) {
#pragma clang fp contract(off)
  __shared__ double sr[256], sm[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int i = t; i < n; i += 256) {
    a += r[i];
    b += r[i] * red[i];
  }
  sr[t] = a;
  sm[t] = b;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (t < o) { sr[t] += sr[t + o]; sm[t] += sm[t + o]; }
    __syncthreads();
  }
  const double R = sr[0], Mq = sm[0];
  for (int i = t; i < n; i += 256) {
    const double mm = red[i], A = red[n + i];
    const double ii = (mm > 0.0 && R > 0.0) ? A / (R * mm) : 0.0;
    const double oo = (Mq > 0.0 && R > 0.0) ? A / Mq : 0.0;
    if (m_out) m_out[i] = mm;
    if (in_in) in_in[i] = ii;
    if (in_out) in_out[i] = oo;
    if (depth) depth[i] = ii < oo ? ii : oo;
  }
}

template <typename T>
static void launch_weighted_t(const pid_ensemble& e, int iso_kind, const Extract& ex, bool vec, const MeanPlan& p3,
                              const void* coef, int tg, void* tpart, void* sbuf, double* part, hipStream_t st) {
  if (iso_kind == PID_ISO_GAUSSIAN) launch_colsum_g<T, MODE_GAUSS, true>(e, ex, tg, coef, tpart, sbuf, vec, st);
  else if (iso_kind == PID_ISO_STEP) launch_colsum_g<T, MODE_STEP, true>(e, ex, tg, coef, tpart, sbuf, vec, st);
  else if (iso_mode(iso_kind) == MODE_MODEL) {
    if constexpr (has_models<T>()) launch_colsum_g<T, MODE_MODEL, true>(e, ex, tg, coef, tpart, sbuf, vec, st);
  } else launch_colsum_g<T, MODE_NONE, true>(e, ex, tg, coef, tpart, sbuf, vec, st);
  if (iso_kind == PID_ISO_GAUSSIAN) dispatch_mpw<T, MODE_GAUSS>(p3, e, ex, vec, sbuf, part, st);
  else if (iso_kind == PID_ISO_STEP) dispatch_mpw<T, MODE_STEP>(p3, e, ex, vec, sbuf, part, st);
  else if (iso_mode(iso_kind) == MODE_MODEL) {
    if constexpr (has_models<T>()) dispatch_mpw<T, MODE_MODEL>(p3, e, ex, vec, sbuf, part, st);
  } else dispatch_mpw<T, MODE_NONE>(p3, e, ex, vec, sbuf, part, st);
}

hipError_t launch_pid_mean_weighted(const pid_ensemble& e, int iso_kind, const ExtractHost& exh,
                                    const double* member_w, const pid_out& out, void* ws, hipStream_t st) {
  const MeanPlan p3 = rows_plan(e.n, e.m, e.dtype);
  Carve c(ws);
  void* coef = c.take<double>((size_t)e.n);
  void* sbuf = c.take<double>((size_t)e.m);
  const int tg = colsum_groups(e.n, e.m, elem_bytes_of(e.dtype));
  void* tpart = c.take<double>((size_t)e.m * (size_t)tg);
  double* part = c.take<double>((size_t)p3.grid * 2 * e.n);
  double* red = c.take<double>((size_t)2 * e.n);
  const int cg = (int)((e.n + 255) / 256);
  if (e.dtype == PID_F64) hipLaunchKernelGGL(member_coef_kernel<double>, cg, 256, 0, st, member_w, (int)e.n, (double*)coef);
  else hipLaunchKernelGGL(member_coef_kernel<float>, cg, 256, 0, st, member_w, (int)e.n, (float*)coef);
  Extract ex = __builtin_bit_cast(Extract, exh);
  const int eb = elem_bytes_of(e.dtype);
  const bool vec = ((reinterpret_cast<uintptr_t>(e.data) & 15) == 0) && ((e.ld * eb) % 16 == 0) &&
                   (e.weights == nullptr || (reinterpret_cast<uintptr_t>(e.weights) & 15) == 0);
  switch (e.dtype) {
    case PID_F64: launch_weighted_t<double>(e, iso_kind, ex, vec, p3, coef, tg, tpart, sbuf, part, st); break;
    case PID_F32: launch_weighted_t<float>(e, iso_kind, ex, vec, p3, coef, tg, tpart, sbuf, part, st); break;
    case PID_F16: launch_weighted_t<f16>(e, iso_kind, ex, vec, p3, coef, tg, tpart, sbuf, part, st); break;
    case PID_BF16: launch_weighted_t<bf16_t>(e, iso_kind, ex, vec, p3, coef, tg, tpart, sbuf, part, st); break;
    default: launch_weighted_t<uint8_t>(e, iso_kind, ex, vec, p3, coef, tg, tpart, sbuf, part, st); break;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  KernelTimer tm("pidmean_finalize", st);
  dim3 rgrid((unsigned)e.n, 2);
  hipLaunchKernelGGL(pidmean_reduce, rgrid, 256, 0, st, part, p3.grid, (int)e.n, red);
  hipLaunchKernelGGL(pidmean_weighted_ratios, 1, 256, 0, st, red, member_w, (int)e.n, out.mass, out.in_in,
                     out.in_out, out.depth);
  return hipGetLastError();
}

}  // namespace pidk

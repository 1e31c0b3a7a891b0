// Bit-packed binary masks: one bit per grid point, 32 points per 32-bit word
// (point x of a row is bit x mod 32 of word x / 32, little-endian bytes, so
// bit x mod 8 of byte x / 8).  PID-mean of binary masks (Sec. 4.1 with the
// binary reduction of Sec. 3.2) in exact integers, from popcounts:
//   m_i = sum_x b_i(x),   s(x) = sum_j b_j(x),   S_i = sum_x b_i(x) s(x),
//   IN_in = S_i / (N m_i),  IN_out = S_i / sum_k m_k,
// so the results are bitwise those of the oracle's exact integer form.  Two
// streaming passes over the bits:
//   1. column counts: for every word, the members are added bit-sliced (a
//      vertical counter: plane k holds bit k of the 32 points' counts), up to
//      255 members per group into 8 planes; the groups' planes are then added
//      with a bit-sliced ripple-carry adder into KT planes of the count s;
//   2. row sums: S_i = sum_w sum_k 2^k popcount(b_i(w) & P_k(w)) and
//      m_i = sum_w popcount(b_i(w)), per lane in registers, per wave by a fixed
//      butterfly, per tile into int64 partials reduced in a fixed order.
// U8 0/1 masks and thresholded fields (the sharp isovalue, Sec. 3.1 Eq. 2)
// take the same path: their first pass reads the stored values once, turns
// them into bits, packs them into a workspace copy and counts them, and the
// row pass reads the packed copy.  The packing kernel writes the packed
// layout from U8 masks for callers that keep them packed.
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <type_traits>

namespace pidk {

// ---------------------------------------------------------------- U8 -> bits
// Bit k of the result: the lowest bit of byte k of x (k < 4); shifts by 7,
// 14 and 21 bring the lowest bits of bytes 1, 2 and 3 to bits 1, 2 and 3.
// FOLD first ORs each byte's bits into its lowest one (a nonzero byte counts
// as 1); without it the bytes must be 0 or 1.
template <bool FOLD>
__device__ __forceinline__ uint32_t nz4(uint32_t x) {
  if constexpr (FOLD) {
    x |= x >> 4;
    x |= x >> 2;
    x |= x >> 1;
  }
  const uint32_t y = x & 0x01010101u;
  return (y | (y >> 7) | (y >> 14) | (y >> 21)) & 0xfu;
}

template <bool FOLD>
__device__ __forceinline__ uint32_t nz16(uint4 v) {
  return nz4<FOLD>(v.x) | (nz4<FOLD>(v.y) << 4) | (nz4<FOLD>(v.z) << 8) | (nz4<FOLD>(v.w) << 12);
}

// A chunk of 2048 points of a row is 64 words; lane l holds word l / 2
// (even l) or 32 + l / 2 (odd l) of it.
__device__ __forceinline__ int chunk_word(int lane) { return (lane & 1) ? 32 + (lane >> 1) : (lane >> 1); }

// The lane's word of chunk c of a U8 row, for any row alignment.  The wave
// reads the chunk as 16-byte blocks aligned down from its first byte (a
// misalignment of a bytes): lane l loads blocks l and 64 + l, and lane 63
// also block 128 when a > 0; block k holds points 16k - a .. 16k - a + 15 of
// the chunk.  A block is loaded only if it holds a point of the row below m,
// so no load leaves the 16-byte block (and page) of a valid byte; points
// outside the chunk or at or past m are shifted or masked out.  Lane l's 16
// points from 16l are the top 16 - a bits of its block's bits and the low a
// bits of its right neighbour's; likewise from 1024 + 16l.  Neighbouring
// lanes then swap one half-word.  Wave-uniform call.
// Lane l's word from its two pieces hA, hB (blocks l and 64 + l of the
// aligned-down run) and, when the chunk is not 16-byte aligned (a != 0, the
// same for the whole wave), the neighbours' low bits shifted in; lane 63
// takes them from hC (block 128).
template <bool FOLD>
__device__ __forceinline__ uint32_t u8_assemble(uint32_t hA, uint32_t hB, uint32_t hC, int a, int64_t rem, int lane) {
  uint32_t lo = hA, hi = hB;
  if (a != 0) {   // wave-uniform: shift in the neighbours' low bits
    uint32_t nA = (uint32_t)__shfl_down((int)hA, 1, 64);
    uint32_t nB = (uint32_t)__shfl_down((int)hB, 1, 64);
    const uint32_t b0 = (uint32_t)__shfl((int)hB, 0, 64);
    if (lane == 63) {
      nA = b0;
      nB = hC;
    }
    lo = ((hA >> a) | (nA << (16 - a))) & 0xffffu;
    hi = ((hB >> a) | (nB << (16 - a))) & 0xffffu;
  }
  const uint32_t r = (uint32_t)__shfl_xor((int)((lane & 1) ? lo : hi), 1, 64);
  uint32_t wd = (lane & 1) ? (r | (hi << 16)) : (lo | (r << 16));
  const int64_t left = rem - 32 * (int64_t)chunk_word(lane);   // points of the word below m
  if (left < 32) wd = left <= 0 ? 0u : (wd & ((1u << left) - 1u));
  return wd;
}

template <bool FOLD>
__device__ __forceinline__ uint32_t chunk_word_u8(const uint8_t* row, int64_t c, int64_t m, int lane) {
  const uint8_t* cp = row + c * 2048;
  const int a = (int)(reinterpret_cast<uintptr_t>(cp) & 15);
  const uint4* bp = reinterpret_cast<const uint4*>(cp - a);
  const int64_t rem = m - c * 2048;   // points of the row from the chunk's first one
  uint32_t hA, hB;
  if (rem >= 2048) {   // a full chunk (wave-uniform): no guards on the loads
    hA = nz16<FOLD>(bp[lane]);
    hB = nz16<FOLD>(bp[64 + lane]);
  } else {
    hA = (16 * lane - a < rem) ? nz16<FOLD>(bp[lane]) : 0u;
    hB = (16 * (64 + lane) - a < rem) ? nz16<FOLD>(bp[64 + lane]) : 0u;
  }
  const uint32_t hC = (a != 0 && lane == 63 && 16 * 128 - a < rem) ? nz16<FOLD>(bp[128]) : 0u;
  return u8_assemble<FOLD>(hA, hB, hC, a, rem, lane);
}

// A chunk inside the row (m - 2048 c >= 2048): the three blocks a lane needs,
// loaded without a branch, so that several rows' loads can be in flight
// together.  Block 128 is one address for the whole wave (only lane 63 uses
// it, and only when a != 0, where it holds a byte of the chunk); when the
// chunk is aligned and ends the row it would lie past the row, and block 127
// is read instead (unused).
struct U8Blocks {
  uint4 a, b, c;
};
__device__ __forceinline__ U8Blocks chunk_blocks_u8_full(const uint8_t* row, int64_t c, int64_t m, int lane) {
  const uint8_t* cp = row + c * 2048;
  const int a = (int)(reinterpret_cast<uintptr_t>(cp) & 15);
  const uint4* bp = reinterpret_cast<const uint4*>(cp - a);
  U8Blocks r;
  r.a = bp[lane];
  r.b = bp[64 + lane];
  r.c = bp[(a != 0 || m - c * 2048 > 2048) ? 128 : 127];
  return r;
}
template <bool FOLD>
__device__ __forceinline__ uint32_t chunk_word_u8_full(const U8Blocks& k, const uint8_t* row, int64_t c, int64_t m,
                                                       int lane) {
  const int a = (int)(reinterpret_cast<uintptr_t>(row + c * 2048) & 15);
  return u8_assemble<FOLD>(nz16<FOLD>(k.a), nz16<FOLD>(k.b), nz16<FOLD>(k.c), a, m - c * 2048, lane);
}

// Adds one bit per point to an 8-plane vertical counter.
__device__ __forceinline__ void count_add(uint32_t (&P)[8], uint32_t c) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t t = P[k] & c;
    P[k] ^= c;
    c = t;
  }
}

// OR of v over groups of L consecutive lanes (L = 2, 4, 8 or 16) by DPP
// moves: pairs, quads, half rows, rows.
template <int L>
__device__ __forceinline__ uint32_t group_or(uint32_t v) {
  int x = (int)v;
  x |= __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);                       // quad_perm [1,0,3,2]
  if constexpr (L >= 4) x |= __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  if constexpr (L >= 8) x |= __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
  if constexpr (L >= 16) x |= __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false); // row_mirror
  return (uint32_t)x;
}

// The lane's word of chunk c (2048 points) of a row of stored values of T
// under the sharp isovalue, rows 16-byte aligned.  A 16-byte block holds
// P = 16 / sizeof(T) points and a word L = 32 / P blocks; the wave reads the
// chunk in L fully coalesced loads (lane l takes block 64k + l in load k), so
// that in load k the L lanes of group j hold the P-bit pieces of word
// 64k / L + j: an OR over the group (DPP) gives every lane of it that word,
// and lane l keeps the one of load k = l mod L, i.e. word
// (64 / L)(l mod L) + l / L of the chunk.  Blocks wholly past m are not
// loaded; points past m are masked.  Wave-uniform calls.
template <typename T>
__device__ __forceinline__ int chunk_word_step_index(int lane) {
  constexpr int L = 2 * (int)sizeof(T);
  return (64 / L) * (lane % L) + lane / L;
}

// The L blocks of a chunk that lane `lane` reads (zeros for blocks wholly
// past m; a full chunk loads without guards, a wave-uniform branch).
template <typename T>
struct StepBlocks {
  Vec16<T> v[2 * sizeof(T)];
};

template <typename T>
__device__ __forceinline__ StepBlocks<T> chunk_load_step(const T* row, int64_t c, int64_t m, int lane) {
  constexpr int P = 16 / (int)sizeof(T);
  constexpr int L = 32 / P;
  const Vec16<T>* cp = reinterpret_cast<const Vec16<T>*>(row + c * 2048);
  const int64_t rem = m - c * 2048;
  StepBlocks<T> r;
  if (rem >= 2048) {
#pragma unroll
    for (int k = 0; k < L; ++k) r.v[k] = cp[64 * k + lane];
  } else {
#pragma unroll
    for (int k = 0; k < L; ++k) r.v[k] = ((int64_t)(64 * k + lane) * P < rem) ? cp[64 * k + lane] : Vec16<T>{};
  }
  return r;
}

template <typename T>
__device__ __forceinline__ uint32_t chunk_word_step(const StepBlocks<T>& blk, int64_t c, int64_t m, int lane,
                                                    const Extract& ex) {
  constexpr int P = 16 / (int)sizeof(T);
  constexpr int L = 32 / P;
  const int64_t rem = m - c * 2048;
  uint32_t mine = 0u;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int64_t x0 = (int64_t)(64 * k + lane) * P;
    uint32_t piece = 0u;
#pragma unroll
    for (int p = 0; p < P; ++p) piece |= (uint32_t)(extract_bit<MODE_STEP>(blk.v[k].v[p], ex) != 0) << p;
    if (rem < 2048) piece &= (x0 >= rem) ? 0u : (rem - x0 >= P ? 0xffffffffu : ((1u << (rem - x0)) - 1u));
    const uint32_t w = group_or<L>(piece << (P * (lane % L)));
    if (lane % L == k) mine = w;
  }
  return mine;
}

// Word wi of a row from single values under the sharp isovalue (rows of any
// alignment; points at or past m read as 0).
template <typename T>
__device__ __forceinline__ uint32_t word_elems_step(const T* row, int64_t m, int64_t wi, const Extract& ex) {
  const int64_t p0 = wi * 32;
  const int cnt = (int)max((int64_t)0, min((int64_t)32, m - p0));
  uint32_t b = 0u;
  for (int k = 0; k < cnt; ++k) b |= (uint32_t)(extract_bit<MODE_STEP>(row[p0 + k], ex) != 0) << k;
  return b;
}

// ---------------------------------------------------------------- packing
// Wave per (chunk of 2048 points, 16 rows): grid.x covers four chunks per
// block, grid.y 16 rows per block.
__global__ __launch_bounds__(256) void pack_bits_kernel(const uint8_t* __restrict__ U, int64_t ld, int n, int64_t m,
                                                        uint32_t* __restrict__ out, int64_t ldw) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t W = (m + 31) / 32;
  if (c * 64 >= W) return;   // whole wave
  const int64_t wi = c * 64 + chunk_word(lane);
  const int i1 = min(n, (int)blockIdx.y * 16 + 16);
  int i = blockIdx.y * 16;
  if (m - c * 2048 >= 2048) {   // the chunk lies inside every row: four rows' blocks loaded first
    for (; i + 3 < i1; i += 4) {
      U8Blocks k[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) k[q] = chunk_blocks_u8_full(U + (int64_t)(i + q) * ld, c, m, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        out[(int64_t)(i + q) * ldw + wi] = chunk_word_u8_full<true>(k[q], U + (int64_t)(i + q) * ld, c, m, lane);
    }
  }
  for (; i + 3 < i1; i += 4) {   // four rows in flight
    uint32_t wd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wd[q] = chunk_word_u8<true>(U + (int64_t)(i + q) * ld, c, m, lane);
    if (wi < W) {
#pragma unroll
      for (int q = 0; q < 4; ++q) out[(int64_t)(i + q) * ldw + wi] = wd[q];
    }
  }
  for (; i < i1; ++i) {
    const uint32_t wd = chunk_word_u8<true>(U + (int64_t)i * ld, c, m, lane);
    if (wi < W) out[(int64_t)i * ldw + wi] = wd;
  }
}

// ---------------------------------------------------------------- pass 1
constexpr int kB1Group = 255;   // members per group of the column counts (8 planes)

// U8 input (values 0 or 1).  Block = four waves on one chunk (blockIdx.x)
// and one member group (blockIdx.y): wave q packs the group's rows q, q + 4,
// ... of the chunk into pk and counts them (at most 64: 7 bits of its 8
// planes); waves 1-3 pass their planes through LDS and wave 0 adds them
// (bit-sliced ripple-carry, in wave order) into gpart[g][k][w] (row stride
// Wp).
__global__ __launch_bounds__(256) void u8_count_pack_kernel(const uint8_t* __restrict__ U, int64_t ld, int n,
                                                            int64_t m, int chunk, uint32_t* __restrict__ pk,
                                                            int64_t ldp, int64_t Wp, uint32_t* __restrict__ gpart) {
  __shared__ uint32_t red[3][8][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = blockIdx.x;
  const int g = blockIdx.y;
  const int64_t W = (m + 31) / 32;
  const int64_t wi = c * 64 + chunk_word(lane);
  const int i0 = g * chunk, i1 = min(n, i0 + chunk);
  uint32_t P[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) P[k] = 0u;
  int i = i0 + wave;
  if (m - c * 2048 >= 2048) {   // the chunk lies inside every row: four rows' blocks loaded first
    for (; i + 12 < i1; i += 16) {
      U8Blocks k[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) k[q] = chunk_blocks_u8_full(U + (int64_t)(i + 4 * q) * ld, c, m, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t wd = chunk_word_u8_full<false>(k[q], U + (int64_t)(i + 4 * q) * ld, c, m, lane);
        count_add(P, wd);
        pk[(int64_t)(i + 4 * q) * ldp + wi] = wd;
      }
    }
  }
  for (; i + 12 < i1; i += 16) {   // four rows in flight
    uint32_t wd[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) wd[q] = chunk_word_u8<false>(U + (int64_t)(i + 4 * q) * ld, c, m, lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) count_add(P, wd[q]);
    if (wi < W) {
#pragma unroll
      for (int q = 0; q < 4; ++q) pk[(int64_t)(i + 4 * q) * ldp + wi] = wd[q];
    }
  }
  for (; i < i1; i += 4) {
    const uint32_t w0 = chunk_word_u8<false>(U + (int64_t)i * ld, c, m, lane);
    count_add(P, w0);
    if (wi < W) pk[(int64_t)i * ldp + wi] = w0;
  }
  if (wave > 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) red[wave - 1][k][lane] = P[k];
  }
  __syncthreads();
  if (wave != 0 || wi >= W) return;
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    uint32_t cy = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {   // counts of at most 255 in all: 8 planes
      const uint32_t a = red[w][k][lane];
      const uint32_t x = P[k] ^ a;
      const uint32_t sum = x ^ cy;
      cy = (P[k] & a) | (cy & x);
      P[k] = sum;
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) gpart[((int64_t)g * 8 + k) * Wp + wi] = P[k];
}

// Thresholded fields: packs and counts as u8_count_pack_kernel did with one
// wave per block (the wave takes all rows of the group), with the words
// formed by chunk_word_step (ALIGNED: rows 16-byte aligned) or element by
// element.
template <typename T, bool ALIGNED>
__global__ __launch_bounds__(64) void step_count_pack_kernel(const T* __restrict__ U, int64_t ld, int n, int64_t m,
                                                             Extract ex, int chunk, uint32_t* __restrict__ pk,
                                                             int64_t ldp, int64_t Wp, uint32_t* __restrict__ gpart) {
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int g = blockIdx.y;
  const int64_t W = (m + 31) / 32;
  const int64_t wi = c * 64 + (ALIGNED ? chunk_word_step_index<T>(lane) : lane);
  const int i0 = g * chunk, i1 = min(n, i0 + chunk);
  uint32_t P[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) P[k] = 0u;
  auto word = [&](int i) -> uint32_t {
    const T* row = U + (int64_t)i * ld;
    if constexpr (ALIGNED) return chunk_word_step<T>(chunk_load_step<T>(row, c, m, lane), c, m, lane, ex);
    else return word_elems_step<T>(row, m, wi, ex);
  };
  int i = i0;
  for (; i + 1 < i1; i += 2) {   // two rows in flight
    uint32_t w0, w1;
    if constexpr (ALIGNED) {
      const StepBlocks<T> b0 = chunk_load_step<T>(U + (int64_t)i * ld, c, m, lane);
      const StepBlocks<T> b1 = chunk_load_step<T>(U + (int64_t)(i + 1) * ld, c, m, lane);
      w0 = chunk_word_step<T>(b0, c, m, lane, ex);
      w1 = chunk_word_step<T>(b1, c, m, lane, ex);
    } else {
      w0 = word(i);
      w1 = word(i + 1);
    }
    count_add(P, w0);
    count_add(P, w1);
    if (wi < W) {
      pk[(int64_t)i * ldp + wi] = w0;
      pk[(int64_t)(i + 1) * ldp + wi] = w1;
    }
  }
  if (i < i1) {
    const uint32_t w0 = word(i);
    count_add(P, w0);
    if (wi < W) pk[(int64_t)i * ldp + wi] = w0;
  }
  if (wi < W) {
#pragma unroll
    for (int k = 0; k < 8; ++k) gpart[((int64_t)g * 8 + k) * Wp + wi] = P[k];
  }
}

// V consecutive words of a row from word w0 (vector load when all V lie
// below W; words at or past W read as 0).  VEC loads need the row 4V-byte
// aligned.
template <int V>
struct Words {
  uint32_t v[V];
};

template <int V>
__device__ __forceinline__ Words<V> load_words(const uint32_t* row, int64_t w0, int64_t W) {
  Words<V> r;
  if constexpr (V == 4) {
    if (w0 + 4 <= W) {
      const uint4 t = *reinterpret_cast<const uint4*>(row + w0);
      r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
      return r;
    }
  } else if constexpr (V == 2) {
    if (w0 + 2 <= W) {
      const uint2 t = *reinterpret_cast<const uint2*>(row + w0);
      r.v[0] = t.x; r.v[1] = t.y;
      return r;
    }
  }
#pragma unroll
  for (int q = 0; q < V; ++q) r.v[q] = (w0 + q < W) ? row[w0 + q] : 0u;
  return r;
}

// Packed input.  Block = four waves on V consecutive words per lane from
// (blockIdx.x * 64 + lane) * V and member group blockIdx.y: wave q counts
// the group's rows q, q + 4, ... (at most 64, so 7 bits of its 8 planes),
// waves 1-3 pass their planes through LDS and wave 0 adds them (bit-sliced
// ripple-carry, in wave order).  Bits past m in the last word are masked off.
template <int V>
__global__ __launch_bounds__(256) void b1_count_kernel(const uint32_t* __restrict__ U, int64_t ldw, int n, int64_t W,
                                                       uint32_t lastmask, int chunk, int64_t Wp,
                                                       uint32_t* __restrict__ gpart) {
  __shared__ uint32_t red[3][8][64 * V];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t w0 = ((int64_t)blockIdx.x * 64 + lane) * V;
  const bool live = w0 < W;   // (no early return: a barrier follows)
  const int g = blockIdx.y;
  const int i0 = g * chunk, i1 = min(n, i0 + chunk);
  uint32_t mask[V];
#pragma unroll
  for (int q = 0; q < V; ++q) mask[q] = (w0 + q == W - 1) ? lastmask : 0xffffffffu;
  uint32_t P[V][8];
#pragma unroll
  for (int q = 0; q < V; ++q)
#pragma unroll
    for (int k = 0; k < 8; ++k) P[q][k] = 0u;
  if (live) {
    int i = i0 + wave;
    for (; i + 12 < i1; i += 16) {   // four rows in flight
      Words<V> a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = load_words<V>(U + (int64_t)(i + 4 * r) * ldw, w0, W);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < V; ++q) count_add(P[q], a[r].v[q] & mask[q]);
    }
    for (; i < i1; i += 4) {
      const Words<V> a = load_words<V>(U + (int64_t)i * ldw, w0, W);
#pragma unroll
      for (int q = 0; q < V; ++q) count_add(P[q], a.v[q] & mask[q]);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int q = 0; q < V; ++q)
#pragma unroll
      for (int k = 0; k < 8; ++k) red[wave - 1][k][lane * V + q] = P[q][k];
  }
  __syncthreads();
  if (wave != 0 || !live) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int q = 0; q < V; ++q) {
      uint32_t c = 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k) {   // counts of at most 255 in all: 8 planes
        const uint32_t a = red[w][k][lane * V + q];
        const uint32_t x = P[q][k] ^ a;
        const uint32_t sum = x ^ c;
        c = (P[q][k] & a) | (c & x);
        P[q][k] = sum;
      }
    }
#pragma unroll
  for (int q = 0; q < V; ++q)
    if (w0 + q < W) {
#pragma unroll
      for (int k = 0; k < 8; ++k) gpart[((int64_t)g * 8 + k) * Wp + w0 + q] = P[q][k];
    }
}

// Block of 256 / SL words x SL group slices: thread (word w, slice q) adds
// the 8-plane counts of groups q, q + SL, ... with a bit-sliced ripple-carry
// adder; slice 0 then adds the SL partial counts (integers, so the order of
// the additions does not change them) and writes the KT planes of the count
// s.  Words W..Wp-1 are padding, set to 0.  SL = 16 when there are many
// groups, else 1.

__device__ __forceinline__ void ripple_add(uint32_t (&S)[32], const uint32_t* a, int na) {
  uint32_t c = 0u;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const uint32_t x = (k < na) ? a[k] : 0u;
    const uint32_t y = S[k] ^ x;
    const uint32_t s = y ^ c;
    c = (S[k] & x) | (c & y);
    S[k] = s;
  }
}

template <int SL>
__global__ __launch_bounds__(256) void b1_combine_kernel(const uint32_t* __restrict__ gpart, int groups, int64_t W,
                                                         int64_t Wp, int KT, uint32_t* __restrict__ planes) {
  constexpr int WB = 256 / SL;   // words per block
  __shared__ uint32_t lds[SL > 1 ? SL : 1][32][SL > 1 ? WB + 1 : 1];
  const int wl = threadIdx.x % WB, q = threadIdx.x / WB;
  const int64_t w = (int64_t)blockIdx.x * WB + wl;
  uint32_t S[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) S[k] = 0u;
  if (w < W) {
    for (int g = q; g < groups; g += SL) {
      uint32_t a[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = gpart[((int64_t)g * 8 + k) * Wp + w];
      ripple_add(S, a, 8);
    }
  }
  if constexpr (SL > 1) {
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < KT) lds[q][k][wl] = S[k];
    __syncthreads();
  }
  if (q == 0 && w < Wp) {
    for (int r = 1; r < SL; ++r) {
      uint32_t a[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) a[k] = (k < KT) ? lds[r][k][wl] : 0u;
      ripple_add(S, a, KT);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k)
      if (k < KT) planes[(int64_t)k * Wp + w] = S[k];
  }
}

// ---------------------------------------------------------------- pass 2
// Sum of a non-negative 32-bit integer over the wave, exact while every row
// of 16 lanes sums below 2^31: pairs, quads, half rows and rows by DPP moves,
// then the four row totals added as 64-bit scalars.
__device__ __forceinline__ long long wave_sum_rows(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);   // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);   // row_mirror
  return (long long)__builtin_amdgcn_readlane(v, 0) + (long long)__builtin_amdgcn_readlane(v, 16) +
         (long long)__builtin_amdgcn_readlane(v, 32) + (long long)__builtin_amdgcn_readlane(v, 48);
}

constexpr int kB1Members = 64;   // members per block (16 per wave)

// Most row tiles one block may take: the per-lane sums of S stay below
// 2^27, so that 16 lanes sum below 2^31 (a lane's S per tile is below
// V * 32 * 2^KT <= 2^23).  32 planes keep 64-bit sums, one tile per block.
template <int KT>
constexpr int b1_rows_max_tiles() { return KT == 8 ? 2048 : (KT == 16 ? 16 : 1); }

// Block (tiles [bx * T, bx * T + T), member group of 64): lane l holds the
// count planes of the V words from t * 64V + lV of tile t and runs over its
// wave's 16 members, eight rows in flight, adding m and S per member in its
// registers across the block's tiles; then per member the lanes' sums meet
// (a fixed DPP tree, or a butterfly for 64-bit sums) and lane 0 writes the
// block's partials part[0][i][bx] = m, part[1][i][bx] = S (int64, row length
// nblk).
template <int KT, int V>
__global__ __launch_bounds__(256) void b1_rows_kernel(const uint32_t* __restrict__ U, int64_t ldw, int n, int64_t W,
                                                      uint32_t lastmask, const uint32_t* __restrict__ planes,
                                                      int64_t Wp, int ntiles, int T, int nblk,
                                                      long long* __restrict__ part) {
  constexpr bool WIDE = KT > 16;   // 64-bit per-lane sums
  using SumT = typename std::conditional<WIDE, unsigned long long, uint32_t>::type;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i0 = blockIdx.y * kB1Members + wave;   // the wave's members i0 + 4t, t < 16
  uint32_t am[16];
  SumT as[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    am[t] = 0u;
    as[t] = 0;
  }
  const int tt1 = min(ntiles, (int)blockIdx.x * T + T);
  for (int tt = blockIdx.x * T; tt < tt1; ++tt) {
    const int64_t w0 = (int64_t)tt * (64 * V) + (int64_t)lane * V;
    const bool live = w0 < W;   // then w0 + V <= Wp (Wp is a multiple of 4)
    uint32_t P[KT][V];
    uint32_t mask[V];
#pragma unroll
    for (int q = 0; q < V; ++q) mask[q] = (w0 + q < W) ? ((w0 + q == W - 1) ? lastmask : 0xffffffffu) : 0u;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const Words<V> pw = live ? load_words<V>(planes + (int64_t)k * Wp, w0, Wp) : Words<V>{};
#pragma unroll
      for (int q = 0; q < V; ++q) P[k][q] = live ? pw.v[q] : 0u;
    }
#pragma unroll
    for (int t0 = 0; t0 < 16; t0 += 8) {
      if (i0 + 4 * t0 >= n) break;   // whole wave
      Words<V> b[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int i = i0 + 4 * (t0 + t);
        b[t] = (live && i < n) ? load_words<V>(U + (int64_t)i * ldw, w0, W) : Words<V>{};
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        uint32_t cm = 0u, ck[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) ck[k] = 0u;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          const uint32_t x = b[t].v[q] & mask[q];
          cm += __popc(x);
#pragma unroll
          for (int k = 0; k < KT; ++k) ck[k] += __popc(x & P[k][q]);
        }
        SumT sv = 0;
#pragma unroll
        for (int k = 0; k < KT; ++k) sv += (SumT)ck[k] << k;
        am[t0 + t] += cm;
        as[t0 + t] += sv;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int i = i0 + 4 * t;
    if (i >= n) break;   // whole wave
    long long ms, ss;
    if constexpr (WIDE) {
      ms = (long long)am[t];
      ss = (long long)as[t];
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        ms += __shfl_xor(ms, o, 64);
        ss += __shfl_xor(ss, o, 64);
      }
    } else {
      ms = wave_sum_rows((int)am[t]);
      ss = wave_sum_rows((int)as[t]);
    }
    if (lane == 0) {
      part[(size_t)i * nblk + blockIdx.x] = ms;
      part[((size_t)n + i) * nblk + blockIdx.x] = ss;
    }
  }
}

// ---------------------------------------------------------------- finalize
// Wave per (quantity q, member i): the tile partials part[q][i][*] summed
// (int64, so exactly), into red[q][i].
__global__ __launch_bounds__(256) void b1_reduce_kernel(const long long* __restrict__ part, int nparts, int n,
                                                        long long* __restrict__ red) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= 2 * (int64_t)n) return;   // whole wave
  const long long* p = part + row * nparts;
  long long s = 0;
  for (int b = lane; b < nparts; b += 64) s += p[b];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) red[row] = s;
}

// One block: tot = sum_k m_k (int64, exact), into red[2n].
__global__ __launch_bounds__(1024) void b1_total_kernel(long long* __restrict__ red, int n) {
  __shared__ long long acc[16];
  long long s = 0;
  for (int i = threadIdx.x; i < n; i += 1024) s += red[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) acc[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int k = 0; k < 16; ++k) t += acc[k];
    red[2 * (int64_t)n] = t;
  }
}

// Thread per member: m_i, IN_in = S_i / (N m_i), IN_out = S_i / tot and the
// depth, each ratio one FP64 division of exact integers (0 when the divisor
// is 0).
__global__ __launch_bounds__(256) void b1_ratios_kernel(const long long* __restrict__ red, int n,
                                                        double* __restrict__ m_out, double* __restrict__ in_in,
                                                        double* __restrict__ in_out, double* __restrict__ depth) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double mm = (double)red[i], a = (double)red[n + i], tot = (double)red[2 * (int64_t)n];
  const double ii = (mm > 0.0) ? a / ((double)n * mm) : 0.0;
  const double oo = (tot > 0.0) ? a / tot : 0.0;
  if (m_out) m_out[i] = mm;
  if (in_in) in_in[i] = ii;
  if (in_out) in_out[i] = oo;
  if (depth) depth[i] = ii < oo ? ii : oo;
}

// ---------------------------------------------------------------- host side
namespace {

// Pass 2 and the finalize, on packed rows U (row stride ldw words, vector
// loads when `aligned`).
hipError_t b1_rows_finalize(const B1Plan& p, const uint32_t* U, int64_t ldw, bool aligned, int64_t n, int64_t m,
                            const uint32_t* planes, long long* part, long long* red, const pid_out& out,
                            hipStream_t st) {
  const int rem = (int)(m % 32);
  const uint32_t lastmask = rem ? ((1u << rem) - 1u) : 0xffffffffu;
  const int v = aligned ? (p.kt <= 16 ? 4 : 2) : 1;
  const int ntiles = (int)((p.W + 64 * v - 1) / (64 * v));
  // tiles per block: enough blocks to fill the GPU (about 2048), within the
  // range of the per-lane sums
  const int tmax = p.kt == 8 ? b1_rows_max_tiles<8>() : (p.kt == 16 ? b1_rows_max_tiles<16>() : 1);
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>(tmax, (int64_t)ntiles * p.mgroups / 2048));
  const int nblk = (ntiles + T - 1) / T;
  {
    KernelTimer tm("pidmean", st);
    const dim3 grid((unsigned)nblk, (unsigned)p.mgroups);
#define PID_B1_ROWS(KT, V)                                                                                    \
  hipLaunchKernelGGL((b1_rows_kernel<KT, V>), grid, 256, 0, st, U, ldw, (int)n, p.W, lastmask, planes, p.Wp, \
                     ntiles, T, nblk, part)
    if (p.kt == 8) {
      if (v == 4) PID_B1_ROWS(8, 4); else PID_B1_ROWS(8, 1);
    } else if (p.kt == 16) {
      if (v == 4) PID_B1_ROWS(16, 4); else PID_B1_ROWS(16, 1);
    } else {
      if (v == 2) PID_B1_ROWS(32, 2); else PID_B1_ROWS(32, 1);
    }
#undef PID_B1_ROWS
  }
  KernelTimer tm("pidmean_finalize", st);
  hipLaunchKernelGGL(b1_reduce_kernel, dim3((unsigned)((2 * n + 3) / 4)), 256, 0, st, part, nblk, (int)n, red);
  hipLaunchKernelGGL(b1_total_kernel, 1, 1024, 0, st, red, (int)n);
  hipLaunchKernelGGL(b1_ratios_kernel, dim3((unsigned)((n + 255) / 256)), 256, 0, st, red, (int)n, out.mass,
                     out.in_in, out.in_out, out.depth);
  return hipGetLastError();
}

hipError_t b1_combine(const B1Plan& p, const uint32_t* gpart, uint32_t* planes, hipStream_t st) {
  if (p.groups >= 32)
    hipLaunchKernelGGL((b1_combine_kernel<16>), dim3((unsigned)((p.Wp + 15) / 16)), 256, 0, st, gpart, p.groups,
                       p.W, p.Wp, p.kt, planes);
  else
    hipLaunchKernelGGL((b1_combine_kernel<1>), dim3((unsigned)((p.Wp + 255) / 256)), 256, 0, st, gpart, p.groups,
                       p.W, p.Wp, p.kt, planes);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_b1_mean(const pid_ensemble& e, const pid_out& out, void* ws, hipStream_t st) {
  const B1Plan p = b1_plan(e.n, e.m);
  Carve c(ws);
  uint32_t* gpart = c.take<uint32_t>((size_t)p.groups * 8 * p.Wp);
  uint32_t* planes = c.take<uint32_t>((size_t)p.kt * p.Wp);
  long long* part = c.take<long long>((size_t)2 * e.n * p.ntiles);
  long long* red = c.take<long long>((size_t)2 * e.n + 1);
  const uint32_t* U = reinterpret_cast<const uint32_t*>(e.data);
  const int64_t ldw = e.ld / 32;
  const int rem = (int)(e.m % 32);
  const uint32_t lastmask = rem ? ((1u << rem) - 1u) : 0xffffffffu;
  const bool aligned = (reinterpret_cast<uintptr_t>(e.data) & 15) == 0 && ldw % 4 == 0;
  {
    KernelTimer tm("pidmean_colsum", st);
    if (aligned)
      hipLaunchKernelGGL((b1_count_kernel<4>), dim3((unsigned)((p.W + 255) / 256), (unsigned)p.groups), 256, 0, st,
                         U, ldw, (int)e.n, p.W, lastmask, p.chunk, p.Wp, gpart);
    else
      hipLaunchKernelGGL((b1_count_kernel<1>), dim3((unsigned)((p.W + 63) / 64), (unsigned)p.groups), 256, 0, st,
                         U, ldw, (int)e.n, p.W, lastmask, p.chunk, p.Wp, gpart);
    hipError_t err = b1_combine(p, gpart, planes, st);
    if (err != hipSuccess) return err;
  }
  return b1_rows_finalize(p, U, ldw, aligned, e.n, e.m, planes, part, red, out, st);
}

template <typename T>
static void launch_step_count(const pid_ensemble& e, const Extract& ex, const B1Plan& p, uint32_t* pk,
                              uint32_t* gpart, hipStream_t st) {
  const T* U = reinterpret_cast<const T*>(e.data);
  const dim3 grid((unsigned)((e.m + 2047) / 2048), (unsigned)p.groups);
  const bool aligned = (reinterpret_cast<uintptr_t>(e.data) & 15) == 0 && (e.ld * (int64_t)sizeof(T)) % 16 == 0;
  if (aligned)
    hipLaunchKernelGGL((step_count_pack_kernel<T, true>), grid, 64, 0, st, U, e.ld, (int)e.n, e.m, ex, p.chunk, pk,
                       p.Wp, p.Wp, gpart);
  else
    hipLaunchKernelGGL((step_count_pack_kernel<T, false>), grid, 64, 0, st, U, e.ld, (int)e.n, e.m, ex, p.chunk, pk,
                       p.Wp, p.Wp, gpart);
}

hipError_t launch_mask_bits_mean(const pid_ensemble& e, int iso_kind, const ExtractHost& exh, const pid_out& out,
                                 void* ws, hipStream_t st) {
  const B1Plan p = b1_plan(e.n, e.m);
  Carve c(ws);
  uint32_t* gpart = c.take<uint32_t>((size_t)p.groups * 8 * p.Wp);
  uint32_t* planes = c.take<uint32_t>((size_t)p.kt * p.Wp);
  long long* part = c.take<long long>((size_t)2 * e.n * p.ntiles);
  long long* red = c.take<long long>((size_t)2 * e.n + 1);
  uint32_t* pk = c.take<uint32_t>((size_t)e.n * p.Wp);
  {
    KernelTimer tm("pidmean_colsum", st);
    if (iso_kind == PID_ISO_NONE) {   // U8 0/1 masks
      const dim3 grid((unsigned)((e.m + 2047) / 2048), (unsigned)p.groups);
      hipLaunchKernelGGL(u8_count_pack_kernel, grid, 256, 0, st, reinterpret_cast<const uint8_t*>(e.data), e.ld,
                         (int)e.n, e.m, p.chunk, pk, p.Wp, p.Wp, gpart);
    } else {                          // the sharp isovalue on stored values
      const Extract ex = __builtin_bit_cast(Extract, exh);
      switch (e.dtype) {
        case PID_F64: launch_step_count<double>(e, ex, p, pk, gpart, st); break;
        case PID_F32: launch_step_count<float>(e, ex, p, pk, gpart, st); break;
        case PID_F16: launch_step_count<f16>(e, ex, p, pk, gpart, st); break;
        case PID_BF16: launch_step_count<bf16_t>(e, ex, p, pk, gpart, st); break;
        default: launch_step_count<uint8_t>(e, ex, p, pk, gpart, st); break;
      }
    }
    hipError_t err = b1_combine(p, gpart, planes, st);
    if (err != hipSuccess) return err;
  }
  return b1_rows_finalize(p, pk, p.Wp, true, e.n, e.m, planes, part, red, out, st);
}

hipError_t launch_pack_bits(const pid_ensemble& e, uint32_t* out, int64_t out_ldw, hipStream_t st) {
  const int64_t chunks = (e.m + 2047) / 2048;
  const dim3 grid((unsigned)((chunks + 3) / 4), (unsigned)((e.n + 15) / 16));
  hipLaunchKernelGGL(pack_bits_kernel, grid, 256, 0, st, reinterpret_cast<const uint8_t*>(e.data), e.ld, (int)e.n,
                     e.m, out, out_ldw);
  return hipGetLastError();
}

}  // namespace pidk

// Bit-packed binary masks (PID_B1): one bit per grid point, 32 points per
// 32-bit word (point x of a row is bit x mod 32 of word x / 32, little-endian
// bytes, so bit x mod 8 of byte x / 8).  PID-mean of binary masks (Sec. 4.1
// with the binary reduction of Sec. 3.2) in exact integers, from popcounts:
//   m_i = sum_x b_i(x),   s(x) = sum_j b_j(x),   S_i = sum_x b_i(x) s(x),
//   IN_in = S_i / (N m_i),  IN_out = S_i / sum_k m_k,
// so the results are bitwise those of the U8 path and of the oracle's exact
// integer form.  Two streaming passes over the bits:
//   1. column counts: for every word, the members are added bit-sliced (a
//      vertical counter: plane k holds bit k of the 32 points' counts), 255
//      members per group into 8 planes; the groups' planes are added with a
//      bit-sliced ripple-carry adder into KT planes of the total count s;
//   2. row sums: S_i = sum_w sum_k 2^k popcount(b_i(w) & P_k(w)) and
//      m_i = sum_w popcount(b_i(w)), per lane in registers, per wave by a fixed
//      butterfly, per tile into int64 partials reduced in a fixed order.
// The packing kernel writes this layout from U8 0/1 masks.
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>

namespace pidk {

// ---------------------------------------------------------------- packing
// Thread per output word: 32 bytes of a U8 row (points past m read as 0).
__global__ __launch_bounds__(256) void pack_bits_kernel(const uint8_t* __restrict__ U, int64_t ld, int n, int64_t m,
                                                        uint32_t* __restrict__ out, int64_t ldw) {
  const int64_t W = (m + 31) / 32;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * W) return;
  const int64_t i = e / W, w = e - i * W;
  const uint8_t* row = U + i * ld + w * 32;
  const int cnt = (int)min((int64_t)32, m - w * 32);
  uint32_t b = 0u;
  for (int k = 0; k < cnt; ++k) b |= (row[k] ? 1u : 0u) << k;
  out[i * ldw + w] = b;
}

// ---------------------------------------------------------------- pass 1
constexpr int kB1Group = 255;   // members per group of the column counts (8 planes)

// Block (word tile of 256, member group g): the 8 count planes of the
// group's members for each word, into part[g][k][w].
__global__ __launch_bounds__(256) void b1_count_kernel(const uint32_t* __restrict__ U, int64_t ldw, int n, int64_t W,
                                                       uint32_t lastmask, int chunk, uint32_t* __restrict__ part) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= W) return;   // (no barrier in this kernel)
  const uint32_t mask = (w == W - 1) ? lastmask : 0xffffffffu;
  const int g = blockIdx.y;
  const int i0 = g * chunk, i1 = min(n, i0 + chunk);
  uint32_t P[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) P[k] = 0u;
  auto add = [&](uint32_t c) {   // add one bit per point (a vertical counter)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t t = P[k] & c;
      P[k] ^= c;
      c = t;
    }
  };
  const uint32_t* col = U + w;
  int i = i0;
  for (; i + 3 < i1; i += 4) {   // four rows in flight
    const uint32_t a0 = col[(int64_t)i * ldw], a1 = col[(int64_t)(i + 1) * ldw];
    const uint32_t a2 = col[(int64_t)(i + 2) * ldw], a3 = col[(int64_t)(i + 3) * ldw];
    add(a0 & mask); add(a1 & mask); add(a2 & mask); add(a3 & mask);
  }
  for (; i < i1; ++i) add(col[(int64_t)i * ldw] & mask);
#pragma unroll
  for (int k = 0; k < 8; ++k) part[((int64_t)g * 8 + k) * W + w] = P[k];
}

// Thread per word: the groups' 8-plane counts added (in group order) into
// the KT planes of the total count s.
__global__ __launch_bounds__(256) void b1_combine_kernel(const uint32_t* __restrict__ part, int groups, int64_t W,
                                                         int KT, uint32_t* __restrict__ planes) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= W) return;
  uint32_t S[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) S[k] = 0u;
  for (int g = 0; g < groups; ++g) {
    uint32_t c = 0u;
#pragma unroll
    for (int k = 0; k < 32; ++k) {   // ripple-carry add of an 8-plane number
      const uint32_t a = (k < 8) ? part[((int64_t)g * 8 + k) * W + w] : 0u;
      const uint32_t x = S[k] ^ a;
      const uint32_t s = x ^ c;
      c = (S[k] & a) | (c & x);
      S[k] = s;
    }
  }
  for (int k = 0; k < KT; ++k) planes[(int64_t)k * W + w] = S[k];
}

// ---------------------------------------------------------------- pass 2
constexpr int kB1Members = 64; // members per block (16 per wave)

// Block (row tile t, member group): lane l holds the count planes of words
// t*64*WPL + l + 64 q (q < WPL) and runs over the wave's members; per member
// the lanes' sums meet in a fixed butterfly and lane 0 writes the tile's
// partials part[0][i][t] = m, part[1][i][t] = S (int64).
template <int KT, int kB1Wpl>
__global__ __launch_bounds__(256) void b1_rows_kernel(const uint32_t* __restrict__ U, int64_t ldw, int n, int64_t W,
                                                      uint32_t lastmask, const uint32_t* __restrict__ planes,
                                                      int ntiles, long long* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tile = blockIdx.x;
  uint32_t P[KT][kB1Wpl];
  uint32_t mask[kB1Wpl];
  int64_t wq[kB1Wpl];
#pragma unroll
  for (int q = 0; q < kB1Wpl; ++q) {
    const int64_t w = (int64_t)tile * (64 * kB1Wpl) + lane + 64 * q;
    wq[q] = w < W ? w : W - 1;                   // in bounds; masked to zero below
    mask[q] = w < W ? (w == W - 1 ? lastmask : 0xffffffffu) : 0u;
#pragma unroll
    for (int k = 0; k < KT; ++k) P[k][q] = planes[(int64_t)k * W + wq[q]];
  }
  const int i0 = blockIdx.y * kB1Members;
  for (int r = wave; r < kB1Members; r += 4) {
    const int i = i0 + r;
    if (i >= n) break;   // whole wave
    const uint32_t* row = U + (int64_t)i * ldw;
    uint32_t b[kB1Wpl];
#pragma unroll
    for (int q = 0; q < kB1Wpl; ++q) b[q] = row[wq[q]] & mask[q];
    uint32_t cm = 0u, ck[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) ck[k] = 0u;
#pragma unroll
    for (int q = 0; q < kB1Wpl; ++q) {
      cm += __popc(b[q]);
#pragma unroll
      for (int k = 0; k < KT; ++k) ck[k] += __popc(b[q] & P[k][q]);
    }
    unsigned long long s = 0ull;
#pragma unroll
    for (int k = 0; k < KT; ++k) s += (unsigned long long)ck[k] << k;
    long long ms = (long long)cm, ss = (long long)s;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      ms += __shfl_xor(ms, o, 64);
      ss += __shfl_xor(ss, o, 64);
    }
    if (lane == 0) {
      part[(size_t)i * ntiles + tile] = ms;
      part[((size_t)n + i) * ntiles + tile] = ss;
    }
  }
}

// ---------------------------------------------------------------- host side
hipError_t launch_b1_mean(const pid_ensemble& e, const pid_out& out, void* ws, hipStream_t st) {
  const B1Plan p = b1_plan(e.n, e.m);
  Carve c(ws);
  uint32_t* gpart = c.take<uint32_t>((size_t)p.groups * 8 * p.W);
  uint32_t* planes = c.take<uint32_t>((size_t)p.kt * p.W);   // 8, 16 or 32 planes, as the row kernel reads
  long long* part = c.take<long long>((size_t)2 * e.n * p.ntiles);
  long long* red = c.take<long long>((size_t)2 * e.n);
  const uint32_t* U = reinterpret_cast<const uint32_t*>(e.data);
  const int64_t ldw = e.ld / 32;
  const int rem = (int)(e.m % 32);
  const uint32_t lastmask = rem ? ((1u << rem) - 1u) : 0xffffffffu;
  {
    KernelTimer tm("pidmean_colsum", st);
    hipLaunchKernelGGL(b1_count_kernel, dim3((unsigned)((p.W + 255) / 256), (unsigned)p.groups), 256, 0, st, U, ldw,
                       (int)e.n, p.W, lastmask, p.chunk, gpart);
    hipLaunchKernelGGL(b1_combine_kernel, dim3((unsigned)((p.W + 255) / 256)), 256, 0, st, gpart, p.groups, p.W,
                       p.kt, planes);
  }
  {
    KernelTimer tm("pidmean", st);
    const dim3 grid((unsigned)p.ntiles, (unsigned)p.mgroups);
    if (p.kt == 8)   // (the plan's words per lane: 4 up to 16 planes, 2 beyond)
      hipLaunchKernelGGL((b1_rows_kernel<8, 4>), grid, 256, 0, st, U, ldw, (int)e.n, p.W, lastmask, planes, p.ntiles, part);
    else if (p.kt == 16)
      hipLaunchKernelGGL((b1_rows_kernel<16, 4>), grid, 256, 0, st, U, ldw, (int)e.n, p.W, lastmask, planes, p.ntiles, part);
    else
      hipLaunchKernelGGL((b1_rows_kernel<32, 2>), grid, 256, 0, st, U, ldw, (int)e.n, p.W, lastmask, planes, p.ntiles, part);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return launch_binary_finalize(part, red, p.ntiles, e.n, out, st);
}

hipError_t launch_pack_bits(const pid_ensemble& e, uint32_t* out, int64_t out_ldw, hipStream_t st) {
  const int64_t W = (e.m + 31) / 32;
  const int64_t tot = e.n * W;
  hipLaunchKernelGGL(pack_bits_kernel, dim3((unsigned)((tot + 255) / 256)), 256, 0, st,
                     reinterpret_cast<const uint8_t*>(e.data), e.ld, (int)e.n, e.m, out, out_ldw);
  return hipGetLastError();
}

}  // namespace pidk

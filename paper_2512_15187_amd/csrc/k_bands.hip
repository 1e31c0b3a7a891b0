// Contour-boxplot bands of a ranked ensemble (the pipeline of Sec. 1 and the
// boxplot views of Sec. 6 / 6.1): members binarised at a threshold; the
// median is the deepest member; the band of the k deepest members is bounded
// by the per-point union and intersection of their binarised masks.
//
// One streaming pass over the rows of the k_outer deepest members (gathered
// through `order`), HBM-bound: each lane owns one 16-byte chunk of points
// and keeps, per point, one bit in each of five 32-bit masks.  The decision
// u >= threshold is taken in FP64 on the extracted value (exact for stored
// values and STEP isovalues).
#include "device_common.h"
#include "pid_internal.h"
#include "pid_timing.h"

#include <type_traits>

namespace pidk {

struct BandArgs {
  const void* U;
  int64_t ld;
  int n;
  int64_t m;
  const int32_t* order;
  int k_inner, k_outer;
  double thr;
  int vec;                // rows 16-byte aligned: vector loads
  uint8_t* out;
};

// members whose chunks are loaded together (fewer for 1- and 2-byte input,
// whose chunks carry more points to decide)
template <typename T>
constexpr int band_unr() { return sizeof(T) >= 4 ? 16 : 8; }

// A block covers the points of 64 lanes; its four waves take interleaved
// rounds of members (wave w: members 4r*UNR + w*UNR ... of round r) and meet
// in LDS, where the masks combine by OR / AND (exact, order-free).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void bands_kernel(BandArgs a, Extract ex) {
  constexpr int P = 16 / (int)sizeof(T);   // points per lane
  constexpr int UNR = band_unr<T>();
  constexpr uint32_t ALL = (1u << P) - 1u;
  __shared__ uint32_t sh[4][6][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t x0 = ((int64_t)blockIdx.x * 64 + lane) * P;
  const bool active = x0 < a.m;            // no early return: every wave reaches the barrier
  const int cnt = active ? (int)min((int64_t)P, a.m - x0) : 0;
  const bool full = a.vec && cnt == P;
  const T* __restrict__ U = reinterpret_cast<const T*>(a.U);
  uint32_t med = 0, ui = 0, ii = ALL, uo = 0, io = ALL, bad = 0;
  for (int j0 = wv * UNR; j0 < a.k_outer; j0 += 4 * UNR) {
    Vec16<T> v[UNR];
    bool use[UNR];
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const int j = j0 + q;
      const int idx = (j < a.k_outer) ? a.order[j] : -1;
      use[q] = j < a.k_outer && (unsigned)idx < (unsigned)a.n;
      if (j < a.k_outer && !use[q]) bad = 1;   // an index outside 0..n-1 is never read
      if (use[q] && active) {
        const T* row = U + (int64_t)idx * a.ld + x0;
        if (full) {
          v[q] = load16(row);
        } else {
#pragma unroll
          for (int p = 0; p < P; ++p) v[q].v[p] = (p < cnt) ? row[p] : T{};
        }
      }
    }
    if (!active) continue;
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      if (!use[q]) continue;
      const int j = j0 + q;
      uint32_t b = 0;
#pragma unroll
      for (int p = 0; p < P; ++p) b |= (extract_d<MODE>(v[q].v[p], ex) >= a.thr ? 1u : 0u) << p;
      if (j == 0) med = b;
      if (j < a.k_inner) { ui |= b; ii &= b; }
      uo |= b;
      io &= b;
    }
  }
  sh[wv][0][lane] = med;
  sh[wv][1][lane] = ui;
  sh[wv][2][lane] = ii;
  sh[wv][3][lane] = uo;
  sh[wv][4][lane] = io;
  sh[wv][5][lane] = bad;
  __syncthreads();
  if (wv != 0 || !active) return;
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    med |= sh[w][0][lane];
    ui |= sh[w][1][lane];
    ii &= sh[w][2][lane];
    uo |= sh[w][3][lane];
    io &= sh[w][4][lane];
    bad |= sh[w][5][lane];
  }
  for (int p = 0; p < cnt; ++p) {
    const uint32_t c = ((med >> p) & 1u) | (((ui >> p) & 1u) << 1) | (((ii >> p) & 1u) << 2) |
                       (((uo >> p) & 1u) << 3) | (((io >> p) & 1u) << 4) | (bad ? 128u : 0u);
    a.out[x0 + p] = (uint8_t)c;
  }
}

template <typename T>
static void launch_bands_t(const BandArgs& a, int kind, const Extract& ex, hipStream_t st) {
  constexpr int P = 16 / (int)sizeof(T);
  const int64_t lanes = (a.m + P - 1) / P;
  const unsigned grid = (unsigned)((lanes + 63) / 64);
  switch (kind) {
    case PID_ISO_GAUSSIAN: hipLaunchKernelGGL((bands_kernel<T, MODE_GAUSS>), grid, 256, 0, st, a, ex); break;
    case PID_ISO_STEP: hipLaunchKernelGGL((bands_kernel<T, MODE_STEP>), grid, 256, 0, st, a, ex); break;
    case PID_ISO_RAMP: case PID_ISO_TENT: case PID_ISO_DENSITY:
      if constexpr (sizeof(T) >= 2 && !std::is_same<T, bf16_t>::value)
        hipLaunchKernelGGL((bands_kernel<T, MODE_MODEL>), grid, 256, 0, st, a, ex);
      break;
    default: hipLaunchKernelGGL((bands_kernel<T, MODE_NONE>), grid, 256, 0, st, a, ex); break;
  }
}

hipError_t launch_bands(const pid_ensemble& e, int iso_kind, const ExtractHost& exh, const int32_t* order,
                        int64_t k_inner, int64_t k_outer, double threshold, uint8_t* out, hipStream_t st) {
  const Extract ex = __builtin_bit_cast(Extract, exh);
  const int eb = (e.dtype == PID_F64) ? 8 : (e.dtype == PID_F32) ? 4 : (e.dtype == PID_U8) ? 1 : 2;
  BandArgs a{};
  a.U = e.data;
  a.ld = e.ld;
  a.n = (int)e.n;
  a.m = e.m;
  a.order = order;
  a.k_inner = (int)k_inner;
  a.k_outer = (int)k_outer;
  a.thr = threshold;
  a.vec = ((reinterpret_cast<uintptr_t>(e.data) & 15) == 0 && (e.ld * eb) % 16 == 0) ? 1 : 0;
  a.out = out;
  KernelTimer tm("bands", st);
  switch (e.dtype) {
    case PID_F64: launch_bands_t<double>(a, iso_kind, ex, st); break;
    case PID_F32: launch_bands_t<float>(a, iso_kind, ex, st); break;
    case PID_F16: launch_bands_t<f16>(a, iso_kind, ex, st); break;
    case PID_BF16: launch_bands_t<bf16_t>(a, iso_kind, ex, st); break;
    default: launch_bands_t<uint8_t>(a, iso_kind, ex, st); break;
  }
  return hipGetLastError();
}

}  // namespace pidk

// Standalone extraction (Sec. 3.5), ranks by depth (Sec. 5.1) and the opt-in
// value-range check of the inputs.
#include "device_common.h"

#include <climits>
#include "pid_internal.h"
#include "pid_timing.h"

#include <algorithm>
#include <type_traits>

namespace pidk {

template <typename T, int MODE, typename OT>
__global__ __launch_bounds__(256) void extract_kernel(const T* __restrict__ U, int64_t ld, int64_t n,
                                                      int64_t m, Extract ex, OT* __restrict__ out) {
  const int64_t tot = n * m;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / m, x = e - i * m;
    const T v = U[i * ld + x];
    if constexpr (sizeof(OT) == 8) out[e] = extract_d<MODE>(v, ex);
    else if constexpr (sizeof(T) == 8) out[e] = (float)extract_d<MODE>(v, ex);
    else out[e] = extract_f<MODE>(v, ex);
  }
}

template <typename T, int MODE>
static void launch_extract_t(const pid_ensemble& e, const Extract& ex, void* out, int odt, hipStream_t st) {
  const int64_t tot = e.n * e.m;
  const int grid = (int)std::min<int64_t>((tot + 255) / 256, 65536);
  const T* U = reinterpret_cast<const T*>(e.data);
  if (odt == PID_F64)
    hipLaunchKernelGGL((extract_kernel<T, MODE, double>), grid, 256, 0, st, U, e.ld, e.n, e.m, ex, (double*)out);
  else
    hipLaunchKernelGGL((extract_kernel<T, MODE, float>), grid, 256, 0, st, U, e.ld, e.n, e.m, ex, (float*)out);
}

template <typename T>
static void launch_extract_m(const pid_ensemble& e, int kind, const Extract& ex, void* out, int odt, hipStream_t st) {
  switch (kind) {
    case PID_ISO_GAUSSIAN: launch_extract_t<T, MODE_GAUSS>(e, ex, out, odt, st); break;
    case PID_ISO_STEP: launch_extract_t<T, MODE_STEP>(e, ex, out, odt, st); break;
    case PID_ISO_RAMP: case PID_ISO_TENT: case PID_ISO_DENSITY:
      if constexpr (sizeof(T) >= 2 && !std::is_same<T, bf16_t>::value) launch_extract_t<T, MODE_MODEL>(e, ex, out, odt, st);
      break;
    default: launch_extract_t<T, MODE_NONE>(e, ex, out, odt, st); break;
  }
}

hipError_t launch_extract(const pid_ensemble& e, int iso_kind, const ExtractHost& exh, void* u_out,
                          int out_dtype, hipStream_t st) {
  Extract ex = __builtin_bit_cast(Extract, exh);
  KernelTimer tm("extract", st);
  switch (e.dtype) {
    case PID_F64: launch_extract_m<double>(e, iso_kind, ex, u_out, out_dtype, st); break;
    case PID_F32: launch_extract_m<float>(e, iso_kind, ex, u_out, out_dtype, st); break;
    case PID_F16: launch_extract_m<f16>(e, iso_kind, ex, u_out, out_dtype, st); break;
    case PID_BF16: launch_extract_m<bf16_t>(e, iso_kind, ex, u_out, out_dtype, st); break;
    default: launch_extract_m<uint8_t>(e, iso_kind, ex, u_out, out_dtype, st); break;
  }
  return hipGetLastError();
}

// Largest stored value of the ensemble (NaN values skipped), e.g. the
// normalising density of PID_ISO_DENSITY.  Doubles are mapped to unsigned
// keys that order like the values, so one integer atomicMax per wave finds
// the maximum (an order-independent, exact result); the key is decoded in
// place at the end.
__device__ __forceinline__ unsigned long long max_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void field_max_init(unsigned long long* key) { *key = 0ull; }

template <typename T>
__global__ __launch_bounds__(256) void field_max_kernel(const T* __restrict__ U, int64_t ld, int64_t n, int64_t m,
                                                        unsigned long long* __restrict__ key) {
  const int64_t tot = n * m;
  unsigned long long k = 0ull;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / m, x = e - i * m;
    const double v = to_double(U[i * ld + x]);
    if (v == v) k = max(k, max_key(v));
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) k = max(k, (unsigned long long)__shfl_xor(k, o, 64));
  if ((threadIdx.x & 63) == 0 && k) atomicMax(key, k);
}

__global__ void field_max_final(unsigned long long* key) {
  const unsigned long long k = *key;
  double v = __longlong_as_double(0x7ff8000000000000ll);   // NaN: no value that is not NaN
  if (k) v = __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffull) : ~k));
  *reinterpret_cast<double*>(key) = v;
}

hipError_t launch_field_max(const pid_ensemble& e, double* out, hipStream_t st) {
  unsigned long long* key = reinterpret_cast<unsigned long long*>(out);
  hipLaunchKernelGGL(field_max_init, 1, 1, 0, st, key);
  const int64_t tot = e.n * e.m;
  const int grid = (int)std::min<int64_t>((tot + 255) / 256, (int64_t)device_cu_count() * 16);
  switch (e.dtype) {
    case PID_F64: hipLaunchKernelGGL(field_max_kernel<double>, grid, 256, 0, st, (const double*)e.data, e.ld, e.n, e.m, key); break;
    case PID_F32: hipLaunchKernelGGL(field_max_kernel<float>, grid, 256, 0, st, (const float*)e.data, e.ld, e.n, e.m, key); break;
    case PID_F16: hipLaunchKernelGGL(field_max_kernel<f16>, grid, 256, 0, st, (const f16*)e.data, e.ld, e.n, e.m, key); break;
    case PID_BF16: hipLaunchKernelGGL(field_max_kernel<bf16_t>, grid, 256, 0, st, (const bf16_t*)e.data, e.ld, e.n, e.m, key); break;
    default: hipLaunchKernelGGL(field_max_kernel<uint8_t>, grid, 256, 0, st, (const uint8_t*)e.data, e.ld, e.n, e.m, key); break;
  }
  hipLaunchKernelGGL(field_max_final, 1, 1, 0, st, key);
  return hipGetLastError();
}

// rank[i] = #{ j : d_j > d_i  or  (d_j == d_i and j < i) };  order[rank[i]] = i.
// One wave per member: lanes compare strided j against the member,
// popcounts of the ballots give the count (an exact integer, so the result
// does not depend on the order of the comparisons).
// blockIdx.y selects one of two depth arrays (the second may be absent).
struct RankArgs {
  const double* d[2];
  int32_t* rank[2];
  int32_t* order[2];
};

__global__ __launch_bounds__(256) void rank_kernel(RankArgs ra, int n) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const double* __restrict__ d = ra.d[blockIdx.y];
  int32_t* __restrict__ rank = ra.rank[blockIdx.y];
  int32_t* __restrict__ order = ra.order[blockIdx.y];
  if (i >= n) return;                       // whole wave leaves together
  const double di = d[i];
  int r = 0;
  // four 64-member chunks per round: their loads are issued together
  for (int j0 = 0; j0 < n; j0 += 256) {
    double dj[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + 64 * c + lane;
      dj[c] = j < n ? d[j] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = j0 + 64 * c + lane;
      const bool before = j < n && ((dj[c] > di) || (dj[c] == di && j < i));
      r += __popcll(__ballot(before));
    }
  }
  if (lane == 0) {
    if (rank) rank[i] = r;
    if (order) order[r] = i;
  }
}

// Large ensembles: a block of four waves ranks 64 consecutive members (16
// per wave) against tiles of 2048 depths staged in LDS.  For a chunk of 64 j
// entirely below the wave's members, "before" is d_j >= d_i; entirely above,
// d_j > d_i; only the chunk that holds the members themselves needs the
// index test.  Padding past n is NaN, which compares false.
constexpr int kRankTile = 2048;

__global__ __launch_bounds__(256) void rank_lds_kernel(RankArgs ra, int n) {
  __shared__ double tile[kRankTile];
  const int lane = threadIdx.x & 63;
  const int i0 = blockIdx.x * 64 + (threadIdx.x >> 6) * 16;   // the wave's first member
  const double* __restrict__ d = ra.d[blockIdx.y];
  double di[16];
  int r[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    di[q] = (i0 + q < n) ? d[i0 + q] : 0.0;
    r[q] = 0;
  }
  for (int t0 = 0; t0 < n; t0 += kRankTile) {
    __syncthreads();
    for (int k = threadIdx.x; k < kRankTile; k += 256)
      tile[k] = (t0 + k < n) ? d[t0 + k] : __builtin_nan("");
    __syncthreads();
    const int tend = min(kRankTile, n - t0);
    for (int c0 = 0; c0 < tend; c0 += 64) {
      const int j0 = t0 + c0;
      const double dj = tile[c0 + lane];
      const int j = j0 + lane;
      if (j0 + 64 <= i0) {          // every j before every member of the wave
#pragma unroll
        for (int q = 0; q < 16; ++q) r[q] += __popcll(__ballot(dj >= di[q]));
      } else if (j0 >= i0 + 16) {   // every j after
#pragma unroll
        for (int q = 0; q < 16; ++q) r[q] += __popcll(__ballot(dj > di[q]));
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) r[q] += __popcll(__ballot((dj > di[q]) || (dj == di[q] && j < i0 + q)));
      }
    }
  }
  int32_t* __restrict__ rank = ra.rank[blockIdx.y];
  int32_t* __restrict__ order = ra.order[blockIdx.y];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (lane == q && i0 + q < n) {
      if (rank) rank[i0 + q] = r[q];
      if (order) order[r[q]] = i0 + q;
    }
  }
}

// Ranks by sorting, for more than 2048 members when the caller's workspace
// provides the scratch (rank_scratch_bytes per depth array).  The order of
// the definition, "j comes before i" iff d_j > d_i or (d_j == d_i and j < i),
// is the ascending order of the pairs (key(d_j), j) with key(d) decreasing in
// d (the IEEE bits mapped to an order-preserving unsigned integer and
// complemented; -0 is taken as +0).  Tiles of 2048 pairs are sorted in LDS by
// a bitonic network (rank_tile_sort); then for every member and tile a
// binary search counts the tile's pairs below the member's (rank_tile_count,
// integer atomics, so the total does not depend on their order); the count
// is the rank.
constexpr int kSortTile = 2048;

__device__ __forceinline__ unsigned long long depth_key(double d) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(d + 0.0);
  const unsigned long long asc = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
  return ~asc;
}

struct RankSort {
  unsigned long long* key[2];
  int32_t* idx[2];
  int32_t* cnt[2];
};

__global__ __launch_bounds__(1024) void rank_tile_sort(RankArgs ra, RankSort rs, int n) {
  __shared__ unsigned long long k[kSortTile];
  __shared__ int32_t x[kSortTile];
  const int a = blockIdx.y, t = threadIdx.x;
  const double* __restrict__ d = ra.d[a];
  const int base = blockIdx.x * kSortTile;
  for (int e = t; e < kSortTile; e += 1024) {
    const int i = base + e;
    k[e] = i < n ? depth_key(d[i]) : ~0ull;      // padding sorts last
    x[e] = i < n ? i : INT_MAX;
    if (i < n) rs.cnt[a][i] = 0;
  }
  __syncthreads();
  for (int size = 2; size <= kSortTile; size <<= 1) {
    for (int j = size >> 1; j > 0; j >>= 1) {
      const int lo = (t / j) * 2 * j + (t % j), hi = lo + j;
      const bool up = (lo & size) == 0;
      const unsigned long long kl = k[lo], kh = k[hi];
      const int xl = x[lo], xh = x[hi];
      const bool gt = kl > kh || (kl == kh && xl > xh);
      if (gt == up) {
        k[lo] = kh; k[hi] = kl;
        x[lo] = xh; x[hi] = xl;
      }
      __syncthreads();
    }
  }
  for (int e = t; e < kSortTile; e += 1024) {
    rs.key[a][base + e] = k[e];
    rs.idx[a][base + e] = x[e];
  }
}

// Thread (member i, tile blockIdx.y): the tile's pairs below (key_i, i).
__global__ __launch_bounds__(256) void rank_tile_count(RankArgs ra, RankSort rs, int n, int arrays) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int tile = blockIdx.y;
  for (int a = 0; a < arrays; ++a) {
    const unsigned long long ki = depth_key(ra.d[a][i]);
    const unsigned long long* __restrict__ K = rs.key[a] + (size_t)tile * kSortTile;
    const int32_t* __restrict__ X = rs.idx[a] + (size_t)tile * kSortTile;
    int lo = 0, len = kSortTile;   // first position whose pair is not below (ki, i)
    while (len > 0) {
      const int half = len >> 1, mid = lo + half;
      const unsigned long long km = K[mid];
      if (km < ki || (km == ki && X[mid] < i)) {
        lo = mid + 1;
        len -= half + 1;
      } else {
        len = half;
      }
    }
    if (lo) atomicAdd(&rs.cnt[a][i], lo);
  }
}

__global__ __launch_bounds__(256) void rank_from_count(RankArgs ra, RankSort rs, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n) return;
  const int r = rs.cnt[a][i];
  if (ra.rank[a]) ra.rank[a][i] = r;
  if (ra.order[a]) ra.order[a][r] = i;
}

static RankSort carve_rank_sort(void* scratch, int64_t n, int arrays) {
  RankSort rs{};
  const size_t per = rank_scratch_bytes(n);
  for (int a = 0; a < arrays; ++a) {
    Carve c(static_cast<char*>(scratch) + (size_t)a * per);
    const size_t tiles = (size_t)((n + kSortTile - 1) / kSortTile) * kSortTile;
    rs.key[a] = c.take<unsigned long long>(tiles);
    rs.idx[a] = c.take<int32_t>(tiles);
    rs.cnt[a] = c.take<int32_t>((size_t)n);
  }
  return rs;
}

static void launch_rank_kernel(const RankArgs& ra, int64_t n, int arrays, hipStream_t st, void* scratch) {
  if (n > 2048 && scratch) {
    const RankSort rs = carve_rank_sort(scratch, n, arrays);
    const unsigned nb = (unsigned)((n + kSortTile - 1) / kSortTile);
    hipLaunchKernelGGL(rank_tile_sort, dim3(nb, arrays), 1024, 0, st, ra, rs, (int)n);
    hipLaunchKernelGGL(rank_tile_count, dim3((unsigned)((n + 255) / 256), nb), 256, 0, st, ra, rs, (int)n, arrays);
    hipLaunchKernelGGL(rank_from_count, dim3((unsigned)((n + 255) / 256), arrays), 256, 0, st, ra, rs, (int)n);
    return;
  }
  if (n <= 2048)
    hipLaunchKernelGGL(rank_kernel, dim3((unsigned)((n + 3) / 4), arrays), 256, 0, st, ra, (int)n);
  else
    hipLaunchKernelGGL(rank_lds_kernel, dim3((unsigned)((n + 63) / 64), arrays), 256, 0, st, ra, (int)n);
}

hipError_t launch_rank(const double* depth, int64_t n, int32_t* rank, int32_t* order, hipStream_t st,
                       void* scratch) {
  KernelTimer tm("rank", st);
  RankArgs ra{{depth, nullptr}, {rank, nullptr}, {order, nullptr}};
  launch_rank_kernel(ra, n, 1, st, scratch);
  return hipGetLastError();
}

hipError_t launch_rank2(const double* d0, int32_t* rank0, int32_t* order0, const double* d1, int32_t* rank1,
                        int32_t* order1, int64_t n, hipStream_t st, void* scratch) {
  KernelTimer tm("rank", st);
  RankArgs ra{{d0, d1}, {rank0, rank1}, {order0, order1}};
  launch_rank_kernel(ra, n, 2, st, scratch);
  return hipGetLastError();
}

// Value checks: codes 1 = probability outside [0,1] or NaN, 2 = U8 value not
// 0/1, 3 = non-finite field value, 4 = negative or non-finite weight.
template <typename T>
__global__ __launch_bounds__(256) void validate_kernel(const T* __restrict__ U, int64_t ld, int64_t n,
                                                       int64_t m, int kind, const float* __restrict__ w,
                                                       unsigned int* __restrict__ flag) {
  const int64_t tot = n * m;
  unsigned int code = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / m, x = e - i * m;
    const double v = to_double(U[i * ld + x]);
    if constexpr (sizeof(T) == 1) {
      if (kind == PID_ISO_NONE && !(v == 0.0 || v == 1.0)) code = 2;
    } else {
      if (kind == PID_ISO_NONE) {
        if (!(v >= 0.0 && v <= 1.0)) code = 1;
      } else if (!isfinite(v)) {
        code = 3;
      }
    }
    if (w && i == 0) {
      const float wx = w[x];
      if (!(wx >= 0.0f) || !isfinite(wx)) code = 4;
    }
  }
  if (code) atomicMax(flag, code);
}

__global__ void zero_flag_kernel(unsigned int* flag) { *flag = 0u; }

hipError_t launch_validate(const pid_ensemble& e, int iso_kind, unsigned int* flag, hipStream_t st) {
  hipLaunchKernelGGL(zero_flag_kernel, 1, 1, 0, st, flag);
  const int64_t tot = e.n * e.m;
  const int grid = (int)std::min<int64_t>((tot + 255) / 256, 16384);
  switch (e.dtype) {
    case PID_F64: hipLaunchKernelGGL(validate_kernel<double>, grid, 256, 0, st, (const double*)e.data, e.ld, e.n, e.m, iso_kind, e.weights, flag); break;
    case PID_F32: hipLaunchKernelGGL(validate_kernel<float>, grid, 256, 0, st, (const float*)e.data, e.ld, e.n, e.m, iso_kind, e.weights, flag); break;
    case PID_F16: hipLaunchKernelGGL(validate_kernel<f16>, grid, 256, 0, st, (const f16*)e.data, e.ld, e.n, e.m, iso_kind, e.weights, flag); break;
    case PID_BF16: hipLaunchKernelGGL(validate_kernel<bf16_t>, grid, 256, 0, st, (const bf16_t*)e.data, e.ld, e.n, e.m, iso_kind, e.weights, flag); break;
    default: hipLaunchKernelGGL(validate_kernel<uint8_t>, grid, 256, 0, st, (const uint8_t*)e.data, e.ld, e.n, e.m, iso_kind, e.weights, flag); break;
  }
  return hipGetLastError();
}

}  // namespace pidk

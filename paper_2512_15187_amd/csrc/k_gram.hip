// All-pairs PID numerators: G_ij = sum_x w_x u_i(x) u_j(x)  (Sec. 3.2 / 3.4).
//
// The inclusion numerators of every ordered pair are one symmetric Gram
// product of the N x M membership matrix (each column scaled by sqrt(w_x)),
// so only the upper triangle of 32x32 sub-tiles is computed.  The reduction
// dimension M (grid points) is split across workgroups (split-K); every
// workgroup streams its range of points in slabs: the slab is loaded from HBM
// with 16-byte loads into registers one slab ahead, run through the isovalue
// model, scaled, converted to the MFMA input type and stored to LDS, where the
// waves read 32-row fragments for their sub-tiles.  Masses m_i are summed in
// the same loader (FP32 per chunk, FP64 across slabs) by the workgroups of the
// diagonal super-tiles.  Partial sums (FP32, or INT32 for binary input) are
// written per split and reduced in a fixed order in FP64 by gram_reduce.
//
// Rows are grouped in super-blocks: one block of up to 8 row blocks when
// N <= 256, otherwise blocks of 4 row blocks (128 rows); a workgroup owns one
// super-tile (I <= J, at most 256 rows) and one split.  Sub-tiles of a super-tile are
// dealt out to 8 waves in contiguous runs (column-major on the diagonal,
// row-major off it) so that consecutive sub-tiles of a wave share a fragment.
// Workgroups are dispatched round-robin over the 8 XCDs; block b is mapped so
// that the super-tiles of one split land on the same XCD and share its L2.
#include "gram_kernel.h"
#include "pid_timing.h"

#include <algorithm>
#include <cstdlib>
#include <type_traits>

namespace pidk {

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of the split partials into the full symmetric
// G (N x N, row-major) and the masses.  A block owns RED_ELEMS consecutive
// partial elements, four per thread of a group (16-byte loads, so a group
// reads 256 contiguous bytes of each split); its 16 thread groups sum the
// splits k = g, g+16, g+32, ... (each in ascending k, up to eight loads in
// flight), and the group sums are
// added in order g = 0..15.  The order depends on nsplit only, so results are
// deterministic.  The masses follow the packed sub-tiles as elements tot,
// tot + 1, ..., four per thread as well.
constexpr int RED_ELEMS = 64;
constexpr int RED_GROUPS = 16;
constexpr int RED_EPT = 4;   // elements per thread

template <typename PT>
__global__ __launch_bounds__(256) void gram_reduce(const PT* __restrict__ part,
                                                   const double* __restrict__ part_mass,
                                                   int nsplit, int np, int n, double* __restrict__ G,
                                                   double* __restrict__ mass) {
  __shared__ double red[RED_GROUPS][RED_ELEMS];
  const int64_t tot = (int64_t)np * 1024;   // a multiple of RED_ELEMS
  const int g = threadIdx.x / (RED_ELEMS / RED_EPT);
  const int el0 = (threadIdx.x % (RED_ELEMS / RED_EPT)) * RED_EPT;
  const int64_t e0 = (int64_t)blockIdx.x * RED_ELEMS + el0;
  const int64_t nx = n;
  double s[RED_EPT] = {0.0, 0.0, 0.0, 0.0};
  if (e0 < tot) {
    const size_t stride = (size_t)np * 1024;
    struct V4 { PT v[RED_EPT]; };
    auto ld = [&](int k) -> V4 {
      const PT* p = part + (size_t)k * stride + (size_t)e0;
      if constexpr (sizeof(PT) == 4) {
        return __builtin_bit_cast(V4, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
      } else {
        V4 r;
#pragma unroll
        for (int q = 0; q < RED_EPT; ++q) r.v[q] = p[q];
        return r;
      }
    };
    auto add = [&](const V4& v) {
#pragma unroll
      for (int r = 0; r < RED_EPT; ++r) s[r] += (double)v.v[r];
    };
    int k = g;
    for (; k + 7 * RED_GROUPS < nsplit; k += 8 * RED_GROUPS) {   // eight splits in flight, added in order
      V4 a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = ld(k + q * RED_GROUPS);
#pragma unroll
      for (int q = 0; q < 8; ++q) add(a[q]);
    }
    for (; k + 3 * RED_GROUPS < nsplit; k += 4 * RED_GROUPS) {   // four splits in flight, added in order
      const V4 a0 = ld(k), a1 = ld(k + RED_GROUPS), a2 = ld(k + 2 * RED_GROUPS), a3 = ld(k + 3 * RED_GROUPS);
      add(a0); add(a1); add(a2); add(a3);
    }
    for (; k < nsplit; k += RED_GROUPS) add(ld(k));
  } else if (e0 < tot + nx) {
    // masses: four consecutive members per thread, four splits in flight
    const int64_t b0 = e0 - tot;
    const int nv = (int)min((int64_t)RED_EPT, nx - b0);
    auto ldm = [&](int k, double (&v)[RED_EPT]) {
#pragma unroll
      for (int r = 0; r < RED_EPT; ++r) v[r] = (r < nv) ? part_mass[(size_t)k * n + (size_t)(b0 + r)] : 0.0;
    };
    int k = g;
    for (; k + 3 * RED_GROUPS < nsplit; k += 4 * RED_GROUPS) {
      double v0[RED_EPT], v1[RED_EPT], v2[RED_EPT], v3[RED_EPT];
      ldm(k, v0); ldm(k + RED_GROUPS, v1); ldm(k + 2 * RED_GROUPS, v2); ldm(k + 3 * RED_GROUPS, v3);
#pragma unroll
      for (int r = 0; r < RED_EPT; ++r) { s[r] += v0[r]; s[r] += v1[r]; s[r] += v2[r]; s[r] += v3[r]; }
    }
    for (; k < nsplit; k += RED_GROUPS) {
      double v[RED_EPT];
      ldm(k, v);
#pragma unroll
      for (int r = 0; r < RED_EPT; ++r) s[r] += v[r];
    }
  }
#pragma unroll
  for (int r = 0; r < RED_EPT; ++r) red[g][el0 + r] = s[r];
  __syncthreads();
  if (threadIdx.x >= RED_ELEMS) return;
  const int el = threadIdx.x;
  const int64_t e = (int64_t)blockIdx.x * RED_ELEMS + el;
  if (e >= tot + nx) return;
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < RED_GROUPS; ++q) t += red[q][el];
  if (e >= tot) {
    mass[e - tot] = t;
    return;
  }
  const int p = (int)(e >> 10);
  const int ij = (int)(e & 1023);
  int C = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (C * (C + 1) / 2 > p) --C;
  while ((C + 1) * (C + 2) / 2 <= p) ++C;
  const int R = p - C * (C + 1) / 2;
  const int i = R * 32 + (ij >> 5), j = C * 32 + (ij & 31);
  if (i >= n || j >= n) return;
  if (R == C && i > j) return;   // diagonal sub-tile: take the upper copy
  G[(size_t)i * n + j] = t;
  G[(size_t)j * n + i] = t;
}

// Depths of member i:
//   IN_in(i)  = S_i / (N m_i),  S_i = sum_j G_ij
//   IN_out(i) = (sum_j G_ji / m_j) / N   (terms with m_j = 0 are 0)
// With an exact integer Gram (INT8 scheme) the lanes form the IN_out terms
// (one correctly rounded division each) for a chunk of j into LDS and one
// lane adds them in ascending j: the fixed order that makes binary results
// bitwise reproducible.  Otherwise every lane sums its strided j and the
// partials meet in a fixed butterfly and wave order (deterministic, not
// sequential).  S_i and sum_k m_k always take the parallel order: for an
// integer Gram they are exact in any order.
constexpr int DEP_CHUNK = 1024;

// All per-member outputs after the reduction, one block of 256 threads per
// member i: the inclusion row P_ij = G_ij / m_i (0 when m_i = 0; when asked
// for), the depths above, and, with `mean` set, the PID-mean ratios of the
// same ensemble.  Their numerators are the Gram row sums:
//   A_i = sum_x w u_i(x) s(x),  s = sum_j u_j   =>   A_i = sum_j G_ij = S_i,
// so IN_in = A_i / (N m_i) is the all-pairs IN_in (the recall identity of
// Sec. 4.1) and IN_out = A_i / sum_k m_k, with sum_k m_k formed by every
// block in the same order.
struct FinishArgs {
  const double* G;
  const double* mass;
  int mean;                 // also write the PID-mean outputs
  int n;
  double* P;
  double *m_out, *in_in, *in_out, *depth;
  double *mm_out, *mm_in, *mm_outo, *mm_depth;   // PID-mean outputs
};

// sum over the 64 lanes, the same butterfly on every lane
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma clang fp contract(off)
  for (int o = 32; o >= 1; o >>= 1) v = v + __shfl_xor(v, o, 64);
  return v;
}

template <bool SERIAL_OUT>
__global__ __launch_bounds__(256) void pairs_finish(FinishArgs f) {
#pragma clang fp contract(off)
  __shared__ double tg[SERIAL_OUT ? DEP_CHUNK : 1];
  __shared__ double red[3][4];
  const int i = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int n = f.n;
  const double* row = f.G + (size_t)i * n;   // G_ij = G_ji (symmetric)
  const double mi = f.mass[i];
  double S = 0.0, O = 0.0, md = 0.0;
  for (int j = t; j < n; j += 256) {
    const double g = row[j];
    const double mj = f.mass[j];
    if (f.P) f.P[(size_t)i * n + j] = (mi > 0.0) ? g / mi : 0.0;
    S = S + g;
    md = md + mj;
    if constexpr (!SERIAL_OUT) O = O + ((mj > 0.0) ? g / mj : 0.0);
  }
  S = wave_sum_d(S);
  md = wave_sum_d(md);
  if constexpr (!SERIAL_OUT) O = wave_sum_d(O);
  if (lane == 0) { red[0][wv] = S; red[1][wv] = O; red[2][wv] = md; }
  if constexpr (SERIAL_OUT) {
    // (every thread passes the same number of barriers)
    double acc = 0.0;
    for (int j0 = 0; j0 < n; j0 += DEP_CHUNK) {
      const int cnt = min(DEP_CHUNK, n - j0);
      for (int q = t; q < cnt; q += 256) {
        const double mj = f.mass[j0 + q];
        tg[q] = (mj > 0.0) ? row[j0 + q] / mj : 0.0;
      }
      __syncthreads();
      if (t == 0)
        for (int q = 0; q < cnt; ++q) acc = acc + tg[q];
      __syncthreads();
    }
    O = acc;
  } else {
    __syncthreads();
  }
  if (t != 0) return;
  S = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  if constexpr (!SERIAL_OUT) O = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  const double tot = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  const double ii = (mi > 0.0) ? S / ((double)n * mi) : 0.0;
  const double oo = O / (double)n;
  if (f.m_out) f.m_out[i] = mi;
  if (f.in_in) f.in_in[i] = ii;
  if (f.in_out) f.in_out[i] = oo;
  if (f.depth) f.depth[i] = ii < oo ? ii : oo;
  if (f.mean) {
    const double moo = (tot > 0.0) ? S / tot : 0.0;
    if (f.mm_out) f.mm_out[i] = mi;
    if (f.mm_in) f.mm_in[i] = ii;
    if (f.mm_outo) f.mm_outo[i] = moo;
    if (f.mm_depth) f.mm_depth[i] = ii < moo ? ii : moo;
  }
}

// ---------------------------------------------------------------------------
// Host side.

hipError_t launch_pid_pairs(const PairsPlan& p, const pid_ensemble& e, int iso_kind,
                            const ExtractHost& exh, const pid_out& out, void* ws, hipStream_t st,
                            const pid_out* mean_out) {
  Carve c(ws);
  GramArgs ga{};
  ga.U = e.data;
  ga.ld = e.ld;
  ga.n = (int)e.n;
  ga.m = e.m;
  ga.w = e.weights;
  ga.ex = __builtin_bit_cast(Extract, exh);
  ga.nbt = p.nbt;
  ga.sb = p.sb;
  ga.nsuper = p.nsuper;
  ga.ntiles_super = p.ntiles_super;
  ga.np = p.np;
  ga.nsplit = p.nsplit;
  ga.slabs = p.slabs;
  ga.part = c.take<char>((size_t)p.nsplit * p.np * 1024 * p.part_elem);
  ga.part_mass = c.take<double>((size_t)p.nsplit * e.n);
  double* G = c.take<double>((size_t)e.n * e.n);
  double* mass = c.take<double>((size_t)e.n);
  const int eb = elem_bytes_of(e.dtype);
  ga.vec = (((reinterpret_cast<uintptr_t>(e.data) & 15) == 0) && ((e.ld * eb) % 16 == 0) &&
            (e.weights == nullptr || (reinterpret_cast<uintptr_t>(e.weights) & 15) == 0)) ? 1 : 0;
  const int mt = mtype_of(p.scheme);
  const int mode = iso_mode(iso_kind);
  const int grid = p.nsplit * p.ntiles_super;
  const int rows = (p.nsuper > 1) ? 64 * p.sb : 32 * p.sb;   // most rows a workgroup loads
  bool ok = false;
  if (mode == MODE_MODEL) ok = gram_dispatch_model(e.dtype, mt, ga, p.maxt, rows, grid, p.lds_bytes, st);
  else switch (e.dtype) {
    case PID_F64: ok = gram_dispatch_f64(mt, mode, ga, p.maxt, rows, grid, p.lds_bytes, st); break;
    case PID_F32: ok = gram_dispatch_f32(mt, mode, ga, p.maxt, rows, grid, p.lds_bytes, st); break;
    case PID_F16: ok = gram_dispatch_f16(mt, mode, ga, p.maxt, rows, grid, p.lds_bytes, st); break;
    case PID_BF16: ok = gram_dispatch_bf16(mt, mode, ga, p.maxt, rows, grid, p.lds_bytes, st); break;
    default: ok = gram_dispatch_u8(mt, mode, ga, p.maxt, rows, grid, p.lds_bytes, st); break;
  }
  if (!ok) return hipErrorNotSupported;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t work = (int64_t)p.np * 1024 + e.n;
  const int rgrid = (int)((work + RED_ELEMS - 1) / RED_ELEMS);
  {
  KernelTimer tm("gram_reduce", st);
  if (p.part_elem == 8)
    hipLaunchKernelGGL(gram_reduce<double>, rgrid, 256, 0, st, (const double*)ga.part, ga.part_mass, p.nsplit, p.np,
                       (int)e.n, G, mass);
  else if (mtype_of(p.scheme) == MT_I8)
    hipLaunchKernelGGL(gram_reduce<int>, rgrid, 256, 0, st, (const int*)ga.part, ga.part_mass, p.nsplit, p.np,
                       (int)e.n, G, mass);
  else
    hipLaunchKernelGGL(gram_reduce<float>, rgrid, 256, 0, st, (const float*)ga.part, ga.part_mass, p.nsplit, p.np,
                       (int)e.n, G, mass);
  }
  {
    KernelTimer tm("pairs_finish", st);
    FinishArgs f{};
    f.G = G;
    f.mass = mass;
    f.n = (int)e.n;
    f.P = out.inclusion;
    f.m_out = out.mass; f.in_in = out.in_in; f.in_out = out.in_out; f.depth = out.depth;
    if (mean_out) {
      f.mean = 1;
      f.mm_out = mean_out->mass; f.mm_in = mean_out->in_in; f.mm_outo = mean_out->in_out;
      f.mm_depth = mean_out->depth;
    }
    if (mt == MT_I8) hipLaunchKernelGGL(pairs_finish<true>, (int)e.n, 256, 0, st, f);
    else hipLaunchKernelGGL(pairs_finish<false>, (int)e.n, 256, 0, st, f);
  }
  return hipGetLastError();
}

}  // namespace pidk

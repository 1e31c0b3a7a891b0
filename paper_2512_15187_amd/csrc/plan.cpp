// Launch plans and workspace sizes of the depth calls.  Host code only (no
// kernels): the geometry of every launch depends on the shape, dtype, isovalue
// model and scheme of a call and on the device's CU count, never on the
// environment, so that a call's accumulation order -- and hence its bitwise
// result -- is fixed by its arguments.
#include <algorithm>
#include <cstdint>
#include <climits>

#include "pid_internal.h"

namespace pidk {

int elem_bytes_of(int dtype) {
  switch (dtype) {
    case PID_F64: return 8;
    case PID_F32: return 4;
    case PID_F16: case PID_BF16: return 2;
    default: return 1;
  }
}

// ---------------------------------------------------------------- all-pairs
// Largest ensemble of the all-pairs calls (the Gram sub-tile and launch
// arithmetic is 32-bit below it).
constexpr int64_t kMaxPairsN = 32768;
// Largest grid.y of a launch.
constexpr int64_t kMaxGridY = 65535;

int mtype_of(int scheme) {
  switch (scheme) {
    case SCH_F16: return MT_F16;
    case SCH_BF16: return MT_BF16;
    case SCH_BF16_SPLIT: return MT_BF16X3;
    case SCH_I8: return MT_I8;
    case SCH_F32: return MT_F32;
    default: return MT_F64;
  }
}

static int mt_bytes(int mt) {
  switch (mt) {
    case MT_F16: case MT_BF16: case MT_BF16X3: return 2;
    case MT_I8: return 1;
    case MT_F32: return 4;
    default: return 8;
  }
}

// chunks (16 B of input) per row per slab of the register-fed Gram kernel
static int cpr_of(int eb_in, int mt) {
  // slab rows of at most 256 bytes in LDS per plane, and of 256 bytes of input
  int cpr = 16;
  const int epc = 16 / eb_in;
  while (cpr > 1 && cpr * epc * mt_bytes(mt) > 256) cpr >>= 1;
  return cpr;
}

int iso_mode(int iso_kind) {
  switch (iso_kind) {
    case PID_ISO_GAUSSIAN: return MODE_GAUSS;
    case PID_ISO_STEP: return MODE_STEP;
    case PID_ISO_RAMP: case PID_ISO_TENT: case PID_ISO_DENSITY: return MODE_MODEL;
    default: return MODE_NONE;
  }
}

// (input dtype, MFMA type, extraction mode) combinations that are built.
bool gram_supported(int dtype, int mt, int mode) {
  if (mode == MODE_MODEL) {   // fields: FP16 MFMA, the accurate BF16 split, the VALU comparators
    if (dtype == PID_F32) return mt == MT_F16 || mt == MT_BF16X3 || mt == MT_F32;
    if (dtype == PID_F16) return mt == MT_F16 || mt == MT_F32;
    if (dtype == PID_F64) return mt == MT_F64;
    return false;
  }
  switch (dtype) {
    case PID_F32:
      if (mt == MT_I8) return mode == MODE_STEP;
      if (mt == MT_F16 || mt == MT_F32) return true;
      return mode != MODE_STEP;                       // BF16, BF16x3, F64
    case PID_F16:
      if (mt == MT_I8) return mode == MODE_STEP;
      if (mt == MT_F16) return true;
      if (mt == MT_F32) return mode != MODE_STEP;
      if (mt == MT_F64) return mode == MODE_NONE;
      return false;
    case PID_BF16:
      return (mt == MT_BF16 || mt == MT_F32) && mode == MODE_NONE;
    case PID_F64:
      if (mt == MT_F64) return true;
      return (mt == MT_F32 || mt == MT_F16) && mode == MODE_NONE;
    case PID_U8:
      if (mt == MT_I8) return mode == MODE_NONE || mode == MODE_STEP;
      return (mt == MT_F16 || mt == MT_F32) && mode == MODE_NONE;
    default:
      return false;
  }
}

bool pairs_supported(int dtype, int iso_kind, int scheme) {
  return gram_supported(dtype, mtype_of(scheme), iso_mode(iso_kind));
}

PairsPlan pairs_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted, int scheme) {
  PairsPlan p{};
  p.scheme = scheme;
  if (n > kMaxPairsN) {   // (the N x N matrix alone would be 8.6 GB at the limit)
    p.unsupported = 1;
    return p;
  }
  const int mt = mtype_of(scheme);
  const int eb = elem_bytes_of(dtype);
  p.nbt = (int)((n + 31) / 32);
  // one diagonal super-tile of up to 8 row blocks when N <= 256, else
  // super-blocks of 4 row blocks (128 rows) and all their pairs I <= J
  p.sb = (p.nbt <= 8) ? p.nbt : 4;
  p.nsuper = (p.nbt + p.sb - 1) / p.sb;
  p.ntiles_super = p.nsuper * (p.nsuper + 1) / 2;
  p.np = p.nbt * (p.nbt + 1) / 2;
  const int tmax = (p.nsuper > 1) ? p.sb * p.sb : p.sb * (p.sb + 1) / 2;
  p.maxt = ((tmax + 7) / 8 <= 2) ? 2 : 5;
  const int cpr = cpr_of(eb, mt);
  p.ks = cpr * (16 / eb);
  p.slabs = (m + p.ks - 1) / p.ks;
  // splits: about one workgroup per CU, at least 2 slabs per split and at
  // most 16384 points of FP32 accumulation per split.  FP32 values through
  // the Gaussian model into a 16-bit MFMA type, one super-tile of at most 128
  // rows: two (smaller) workgroups per CU, so that one evaluates the model
  // while the other waits at a barrier.
  const int cus = device_cu_count();
  const bool two_per_cu = eb == 4 && iso_mode(iso_kind) == MODE_GAUSS &&
                          (mt == MT_F16 || mt == MT_BF16) && p.nsuper == 1 && p.sb <= 4;
  int64_t want = std::max<int64_t>(1, (int64_t)cus * (two_per_cu ? 2 : 1) / p.ntiles_super);
  want = std::min<int64_t>(want, std::max<int64_t>(1, p.slabs / 2));
  const int64_t min_splits = (m + 16383) / 16384;
  if (mt != MT_I8 && mt != MT_F64) want = std::max(want, min_splits);
  p.nsplit = (int)(((want + 7) / 8) * 8);
  p.slabs_per_split = (p.slabs + p.nsplit - 1) / p.nsplit;
  if ((int64_t)p.nsplit * p.ntiles_super > INT32_MAX) p.unsupported = 1;   // one workgroup per (split, super-tile)
  const int rows = (p.nsuper > 1) ? 64 * p.sb : 32 * p.sb;
  const int rowb = p.ks * mt_bytes(mt) + 16;
  const int planes = (mt == MT_BF16X3) ? 2 : 1;
  p.lds_bytes = (size_t)2 * planes * rows * rowb + (size_t)rows * 8;   // two slab buffers + row masses
  p.part_elem = (mt == MT_F64) ? 8 : 4;
  (void)iso_kind; (void)weighted;
  return p;
}

size_t pairs_workspace(const PairsPlan& p, int64_t n) {
  Carve c(nullptr);
  c.take<char>((size_t)p.nsplit * p.np * 1024 * p.part_elem);
  c.take<double>((size_t)p.nsplit * n);   // partial masses
  c.take<double>((size_t)n * n);          // G
  c.take<double>((size_t)n);              // masses
  return c.off + 256;
}

// ---------------------------------------------------------------- PID-mean
static bool is_binary(int dtype, int iso_kind, bool weighted) {
  if (weighted) return false;
  return iso_kind == PID_ISO_STEP || (dtype == PID_U8 && iso_kind == PID_ISO_NONE);
}

// Member groups of a column-sum pass: enough blocks of 4 waves to fill the
// GPU (8 per CU), at least 16 members per group, at most 64 groups.
int colsum_groups(int64_t n, int64_t m, int eb) {
  const int64_t bx = (m + 64 * (16 / eb) - 1) / (64 * (16 / eb));
  int64_t g = ((int64_t)device_cu_count() * 8 + bx - 1) / bx;
  g = std::min<int64_t>(g, std::max<int64_t>(1, (n + 15) / 16));
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 64));
}

// At most this many point tiles per workgroup of the unpipelined kernels:
// per-lane FP32 sums stay short.
constexpr int64_t kTilesPerWorkgroup = 16;

MeanPlan mean_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted) {
  MeanPlan p{};
  p.binary = is_binary(dtype, iso_kind, weighted) ? 1 : 0;
  if (p.binary) {   // U8 masks or thresholded values: packed on the fly, then the popcount passes
    p.bits = 1;
    p.unsupported = b1_plan(n, m).unsupported;
    return p;
  }
  const int eb = elem_bytes_of(dtype);
  const int ppl = 16 / eb;
  const int tp = 64 * ppl;
  const int64_t cus = device_cu_count();
  const int64_t tpw = kTilesPerWorkgroup;
  p.ntiles = (m + tp - 1) / tp;

  // LDS-staged single pass (soft masks, 128 < N <= 256, no straddling
  // 16-byte chunk at the end of a row): waves of 32 rows, a ring of four
  // tile slots.  (For N <= 128 the tiles of eight-row waves are too small
  // per barrier; the register pipeline below is faster there.)
  if (iso_kind == PID_ISO_NONE && dtype != PID_U8 && n > 128 && n <= 256 && (m * eb) % 16 == 0) {
    const int rpw = 32;
    const int nw = (int)((n + rpw - 1) / rpw);
    const int tpp = 128 / eb;
    const int cb = (dtype == PID_F64) ? 8 : 4;
    const size_t lds = (size_t)4 * nw * rpw * 128 + (weighted ? (size_t)4 * nw * 256 : 0) +
                       (size_t)2 * nw * tpp * cb + (size_t)nw * rpw * 16;
    const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(163840 / (int64_t)lds, 32 / nw));
    const int64_t tiles = (m + tpp - 1) / tpp;
    p.dma_rpw = rpw;
    p.dma_nwaves = nw;
    p.dma_lds = lds;
    p.dma_grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, cus * per_cu));
  }

  // Pipelined single pass (soft input, N <= 256; FP64 N <= 128).  Each tile
  // buffer holds MPW members x LB bytes per lane: 4 members x 16 B and
  // 8 members x 8 B (up to 16 waves, 128 registers per lane), 32 members x
  // 4 B (8 waves, 256 registers per lane), so that two buffers, the sums
  // and the addressing fit without spills.  It needs one full tile; rows
  // that are not aligned take the kernel below.
  const bool soft = dtype != PID_U8 &&
                    (iso_kind == PID_ISO_NONE || (iso_kind != PID_ISO_STEP && eb != 2));
  if (soft) {
    int mpw = 0;
    if (n <= 32) mpw = 4;
    else if (n <= 128) mpw = 8;
    else if (n <= 256 && eb <= 4) mpw = 32;
    const int lb = (mpw == 4) ? 16 : (mpw == 8 ? 8 : 4);
    const int ptp = (mpw && lb >= eb) ? 64 * (lb / eb) : 0;
    if (ptp == 0) mpw = 0;
    if (mpw && m >= ptp) {
      p.mpw = mpw;
      p.nwaves = (int)((n + mpw - 1) / mpw);
      p.two_pass = 0;
      p.groups = 1;
      p.pipe_lb = lb;
      const int64_t pt = (m + ptp - 1) / ptp;
      // the workgroups that fit at once (16 waves per CU, 8 with 32 members
      // per wave), each streaming its share of the tiles
      const int64_t resident = cus * std::max(1, (mpw == 32 ? 8 : 16) / p.nwaves);
      p.pipe_grid = (int)std::max<int64_t>(1, std::min<int64_t>(pt, resident));
      const int cb = (dtype == PID_F64) ? 8 : 4;
      p.lds_bytes = (size_t)2 * p.nwaves * ptp * cb + (size_t)2 * p.nwaves * mpw * 8 +
                    (weighted ? (size_t)2 * ptp * 4 : 0);   // column sums, FP64 sums, tile weights
      // the unpipelined kernel for rows that are not aligned: at most 16
      // members per wave, at most tpw tiles per workgroup
      p.fb_mpw = (n <= 32) ? 4 : (n <= 64 ? 8 : 16);
      p.fb_nwaves = (int)((n + p.fb_mpw - 1) / p.fb_mpw);
      p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, std::max<int64_t>((p.ntiles + tpw - 1) / tpw, cus * 2)));
      return p;
    }
  }

  // members per wave: the smallest slice that covers N with at most 8 waves;
  // FP32 soft input may use 16 waves of 16 members (N <= 256) within the
  // 128 registers a 1024-thread workgroup allows; beyond: two passes.
  int mpw = 4;
  if (n > 32) mpw = 8;
  if (n > 64) mpw = 16;
  int nw = (int)((n + mpw - 1) / mpw);
  const int max_waves = (eb == 4) ? 16 : 8;
  p.two_pass = 0;
  p.groups = 1;
  if (nw > max_waves) {
    p.two_pass = 1;
    nw = 8;
    // 16-bit input: 8 members per wave (about 125 registers, two workgroups
    // per CU) rather than 16 (about 210, one workgroup per CU)
    if (eb == 2) mpw = 8;
    p.groups = (int)((n + (int64_t)nw * mpw - 1) / ((int64_t)nw * mpw));
    p.colsum_groups = colsum_groups(n, m, eb);
  }
  p.mpw = mpw;
  p.nwaves = nw;
  // at most tpw tiles per workgroup (short FP32 / INT32 lane sums), and at
  // least two workgroups per CU when there are enough tiles
  int64_t g = std::max<int64_t>((p.ntiles + tpw - 1) / tpw, cus * 2);
  if (p.two_pass) g = std::max<int64_t>((p.ntiles + tpw - 1) / tpw, std::max<int64_t>(1, cus * 2 / p.groups));
  if (p.groups > kMaxGridY) p.unsupported = 1;   // member groups are grid.y
  p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, g));
  const int cb = (dtype == PID_F64) ? 8 : 4;
  p.lds_bytes = p.two_pass ? 0 : (size_t)2 * nw * tp * cb;
  return p;
}

size_t mean_workspace(const MeanPlan& p, int64_t n, int64_t m) {
  if (p.bits) return b1_workspace(b1_plan(n, m), n, true);
  Carve c(nullptr);
  c.take<double>((size_t)std::max(std::max(p.grid, p.pipe_grid), p.dma_grid) * 2 * n);   // partials
  c.take<double>((size_t)2 * n);            // reduced A and m
  if (p.two_pass) {
    c.take<double>((size_t)m);              // column sums
    c.take<double>((size_t)m * (size_t)p.colsum_groups);   // their member-group partials
  }
  return c.off + 256;
}

// The two-pass configuration of mean_plan with soft arithmetic: the row pass
// of the all-pairs depths without the matrix.
MeanPlan rows_plan(int64_t n, int64_t m, int dtype) {
  MeanPlan p{};
  const int eb = elem_bytes_of(dtype);
  const int64_t cus = device_cu_count();
  p.ntiles = (m + 64 * (16 / eb) - 1) / (64 * (16 / eb));
  p.mpw = (n <= 32) ? 4 : ((n <= 64 || eb == 2) ? 8 : 16);   // (16-bit input: as in mean_plan)
  p.nwaves = (int)std::min<int64_t>(8, (n + p.mpw - 1) / p.mpw);
  p.two_pass = 1;
  p.groups = (int)((n + (int64_t)p.nwaves * p.mpw - 1) / ((int64_t)p.nwaves * p.mpw));
  if (p.groups > kMaxGridY) p.unsupported = 1;
  const int64_t g = std::max<int64_t>((p.ntiles + kTilesPerWorkgroup - 1) / kTilesPerWorkgroup,
                                      std::max<int64_t>(1, cus * 2 / p.groups));
  p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(p.ntiles, g));
  return p;
}

size_t pairs_linear_workspace(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted) {
  const MeanPlan p1 = mean_plan(n, m, dtype, iso_kind, weighted);
  const MeanPlan p3 = rows_plan(n, m, dtype);
  // the same pieces, in the same order, as launch_pairs_linear carves
  Carve c(nullptr);
  c.take<char>(mean_workspace(p1, n, m));
  c.take<double>((size_t)n);                     // masses
  c.take<double>((size_t)n);                     // IN_in
  c.take<double>((size_t)n);                     // coefficients 1 / m_j
  c.take<double>((size_t)m);                     // t(x)
  c.take<double>((size_t)m * (size_t)colsum_groups(n, m, elem_bytes_of(dtype)));   // member-group partials of t
  c.take<double>((size_t)p3.grid * 2 * n);       // row partials
  c.take<double>((size_t)2 * n);                 // reduced m, B
  return c.off + 256;
}

// Bit-packed binary PID-mean (k_bits.hip): groups of 255 members for the
// column counts, KT planes for counts up to n, row tiles of 64 lanes x WPL
// words (WPL = 4 up to 16 planes, 2 beyond), 64 members per block.
B1Plan b1_plan(int64_t n, int64_t m) {
  B1Plan p{};
  p.W = (m + 31) / 32;
  p.Wp = (p.W + 3) / 4 * 4;
  // member groups of the first pass: at most 255 members each (8 count
  // planes), and enough of them that chunks x groups fills the GPU (about
  // 2048 waves), down to 8 members per group
  const int64_t chunks = (m + 2047) / 2048;
  const int64_t want = std::min<int64_t>((n + 7) / 8, (2048 + chunks - 1) / chunks);
  p.groups = (int)std::min<int64_t>(INT32_MAX, std::max<int64_t>((n + 254) / 255, want));
  p.chunk = (int)((n + p.groups - 1) / p.groups);
  int bits = 1;   // bits of the largest column count, n
  while (bits < 31 && (INT64_C(1) << bits) <= n) ++bits;
  p.kt = bits <= 8 ? 8 : (bits <= 16 ? 16 : 32);
  p.ntiles = (int)std::min<int64_t>(INT32_MAX, (p.W + 63) / 64);   // row tiles of one word per lane (the most)
  p.mgroups = (int)std::min<int64_t>(INT32_MAX, (n + 63) / 64);
  if (p.groups > kMaxGridY || p.mgroups > kMaxGridY || (p.W + 63) / 64 > INT32_MAX || (m + 2047) / 2048 > INT32_MAX)
    p.unsupported = 1;
  return p;
}

size_t b1_workspace(const B1Plan& p, int64_t n, bool packed_copy) {
  Carve c(nullptr);
  c.take<uint32_t>((size_t)p.groups * 8 * p.Wp);                // group count planes
  c.take<uint32_t>((size_t)p.kt * p.Wp);                        // count planes
  c.take<long long>((size_t)2 * n * p.ntiles);                  // row partials
  c.take<long long>((size_t)2 * n + 1);                         // reduced m, S and the total
  if (packed_copy) c.take<uint32_t>((size_t)n * p.Wp);          // packed copy of U8 masks
  return c.off + 256;
}

// Reliability-weighted PID-mean: the same pieces, in the same order, as
// launch_pid_mean_weighted carves.
size_t mean_weighted_workspace(int64_t n, int64_t m, int dtype) {
  const MeanPlan p = rows_plan(n, m, dtype);
  Carve c(nullptr);
  c.take<double>((size_t)n);                                          // coefficients
  c.take<double>((size_t)m);                                          // s_r(x)
  c.take<double>((size_t)m * (size_t)colsum_groups(n, m, elem_bytes_of(dtype)));   // its member-group partials
  c.take<double>((size_t)p.grid * 2 * n);                             // row partials
  c.take<double>((size_t)2 * n);                                      // reduced m, A
  return c.off + 256;
}

// Sorting ranks: tiles of 2048 (key, index) pairs and a count per member.
size_t rank_scratch_bytes(int64_t n) {
  if (n <= 2048) return 0;
  Carve c(nullptr);
  const size_t tiles = (size_t)((n + 2047) / 2048) * 2048;
  c.take<unsigned long long>(tiles);
  c.take<int32_t>(tiles);
  c.take<int32_t>((size_t)n);
  return (c.off + 255) / 256 * 256;
}

}  // namespace pidk

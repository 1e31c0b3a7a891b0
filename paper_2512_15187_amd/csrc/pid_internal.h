// Host-side interface between the C ABI (api.cpp) and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pid.h"

namespace pidk {

struct Extract;  // device_common.h

// How a stored value becomes a membership probability (compile-time mode of
// every loader; Sec. 3.5).
enum Mode { MODE_NONE = 0, MODE_GAUSS = 1, MODE_STEP = 2,
            MODE_MODEL = 3 };   // MODEL: the piecewise-linear models (ramp, tent, density)
int iso_mode(int iso_kind);
int elem_bytes_of(int dtype);

// Host copy of the isovalue model, converted once per call.
struct ExtractHost {
  int side;
  float cf, af;
  float c_dn, c_up;
  double cd, ad;
  int model;   // PID_ISO_RAMP / TENT / DENSITY under MODE_MODEL
};

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------------- PID-mean
struct MeanPlan {
  int mpw;          // members per wave
  int nwaves;       // waves per workgroup
  int two_pass;     // 1: column sums s(x) go through memory (N too large for one pass)
  int groups;       // member groups (grid.y) in the two-pass case
  int64_t ntiles;   // point tiles of 64 * (16 / elem_bytes) points
  int grid;         // workgroups along the points
  int binary;       // exact integer arithmetic
  size_t lds_bytes;
  int pipe_lb;      // >0: pipelined single pass with LB-byte loads (aligned rows)
  int pipe_grid;    // its grid
  int fb_mpw, fb_nwaves;   // the unpipelined kernel's slices when rows are not aligned
  int colsum_groups;   // two-pass: member groups of the column-sum pass
  int dma_rpw;      // >0: LDS-staged single pass, rows per wave (soft masks)
  int dma_nwaves, dma_grid;
  size_t dma_lds;
  int unsupported;  // 1: no launch geometry keeps the exact integer sums in range
  int bits;         // 1: binary input (U8 masks, thresholded values), packed in the first pass
};
MeanPlan mean_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted);
size_t mean_workspace(const MeanPlan& p, int64_t n, int64_t m);
hipError_t launch_pid_mean(const MeanPlan& p, const pid_ensemble& e, int iso_kind,
                           const ExtractHost& ex, const pid_out& out, void* ws, hipStream_t st);
// Bit-packed binary masks (PID_B1): exact integer PID-mean from popcounts.
struct B1Plan {
  int64_t W;        // 32-point words per row
  int64_t Wp;       // W rounded up to 4: row stride of the count planes and of a packed copy
  int groups;       // member groups of the column counts (<= 255 members each)
  int chunk;        // members per group
  int kt;           // bit planes of the total count: 8, 16 or 32 (counts up to n)
  int ntiles;       // row tiles of the row pass
  int mgroups;      // member groups (64) of the row pass
  int unsupported;
};
B1Plan b1_plan(int64_t n, int64_t m);
size_t b1_workspace(const B1Plan& p, int64_t n, bool packed_copy);
hipError_t launch_b1_mean(const pid_ensemble& e, const pid_out& out, void* ws, hipStream_t st);
// U8 0/1 masks (iso_kind PID_ISO_NONE) or thresholded values (PID_ISO_STEP):
// packed in the first pass, then the popcount passes.
hipError_t launch_mask_bits_mean(const pid_ensemble& e, int iso_kind, const ExtractHost& ex, const pid_out& out,
                                 void* ws, hipStream_t st);
// U8 0/1 masks -> PID_B1 rows of out_ldw 32-bit words.
hipError_t launch_pack_bits(const pid_ensemble& e, uint32_t* out, int64_t out_ldw, hipStream_t st);

// PID-mean against a mean contour weighted by member_w (N device doubles).
size_t mean_weighted_workspace(int64_t n, int64_t m, int dtype);
hipError_t launch_pid_mean_weighted(const pid_ensemble& e, int iso_kind, const ExtractHost& ex,
                                    const double* member_w, const pid_out& out, void* ws, hipStream_t st);
// Member groups of a column-sum pass; the two-pass row plan of the all-pairs
// depths without the matrix.
int colsum_groups(int64_t n, int64_t m, int eb);
MeanPlan rows_plan(int64_t n, int64_t m, int dtype);

// All-pairs depths (no inclusion matrix) in three streaming passes.
size_t pairs_linear_workspace(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted);
hipError_t launch_pairs_linear(const pid_ensemble& e, int iso_kind, const ExtractHost& ex, const pid_out& out,
                               void* ws, hipStream_t st);

// ---------------------------------------------------------------- all-pairs
enum Scheme { SCH_F64 = 1, SCH_F32 = 2, SCH_F16 = 3, SCH_BF16 = 4, SCH_BF16_SPLIT = 5, SCH_I8 = 6 };
// Element type the Gram product multiplies in.
enum MType { MT_F16 = 0, MT_BF16 = 1, MT_BF16X3 = 2, MT_I8 = 3, MT_F32 = 4, MT_F64 = 5 };
int mtype_of(int scheme);

struct PairsPlan {
  int scheme;
  int nbt;          // 32-row blocks covering N
  int sb;           // row blocks per super-block
  int nsuper;       // super-blocks
  int ntiles_super; // super-tiles (I <= J)
  int np;           // upper 32x32 sub-tiles (packed)
  int maxt;         // sub-tiles per wave (register tiles)
  int nsplit;       // K splits (multiple of 8)
  int64_t slabs;    // slabs of points along M
  int64_t slabs_per_split;
  int ks;           // points per slab
  size_t lds_bytes;
  int part_elem;    // bytes per partial element (4 or 8)
  int unsupported;  // 1: N or the launch grid beyond what the kernels address
};
PairsPlan pairs_plan(int64_t n, int64_t m, int dtype, int iso_kind, bool weighted, int scheme);
size_t pairs_workspace(const PairsPlan& p, int64_t n);
// True when the Gram kernel is built for this input dtype, scheme and iso kind.
bool pairs_supported(int dtype, int iso_kind, int scheme);
bool gram_supported(int dtype, int mt, int mode);
// mean_out non-null: also write the PID-mean outputs, from the Gram row sums
// (A_i = sum_j G_ij) and the masses of the same pass.
hipError_t launch_pid_pairs(const PairsPlan& p, const pid_ensemble& e, int iso_kind,
                            const ExtractHost& ex, const pid_out& out, void* ws, hipStream_t st,
                            const pid_out* mean_out = nullptr);

// ---------------------------------------------------------------- misc
hipError_t launch_extract(const pid_ensemble& e, int iso_kind, const ExtractHost& ex, void* u_out,
                          int out_dtype, hipStream_t st);
// Scratch bytes per depth array of the sorting ranks (0: n <= 2048, ranked
// directly).
size_t rank_scratch_bytes(int64_t n);
// Ranks (and order) of depth; with scratch (rank_scratch_bytes(n) bytes per
// array) more than 2048 members are ranked by sorting, otherwise by direct
// comparison.
hipError_t launch_rank(const double* depth, int64_t n, int32_t* rank, int32_t* order, hipStream_t st,
                       void* scratch = nullptr);
// Both rankings of pid_both in one launch.
hipError_t launch_rank2(const double* d0, int32_t* rank0, int32_t* order0, const double* d1, int32_t* rank1,
                        int32_t* order1, int64_t n, hipStream_t st,
                        void* scratch = nullptr);
// Contour-boxplot bands: one byte per point (pid_bands).
hipError_t launch_bands(const pid_ensemble& e, int iso_kind, const ExtractHost& ex, const int32_t* order,
                        int64_t k_inner, int64_t k_outer, double threshold, uint8_t* out, hipStream_t st);
// Largest stored value (NaN skipped) into *out (device).
hipError_t launch_field_max(const pid_ensemble& e, double* out, hipStream_t st);
// Writes 0 to *flag_dev when all values pass, else a nonzero code.
hipError_t launch_validate(const pid_ensemble& e, int iso_kind, unsigned int* flag_dev, hipStream_t st);

int device_cu_count();

}  // namespace pidk

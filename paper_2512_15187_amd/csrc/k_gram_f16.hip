// Instantiations of the Gram kernel for f16 input.
#include "gram_kernel.h"

namespace pidk {

bool gram_dispatch_f16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st) {
  if (!gram_supported(PID_F16, mt, mode)) return false;
  if (mt == MT_F16 && mode == MODE_NONE) { launch_gram_t<f16, MT_F16, MODE_NONE>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F16 && mode == MODE_GAUSS) { launch_gram_t<f16, MT_F16, MODE_GAUSS>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F16 && mode == MODE_STEP) { launch_gram_t<f16, MT_F16, MODE_STEP>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F32 && mode == MODE_NONE) { launch_gram_t<f16, MT_F32, MODE_NONE>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F32 && mode == MODE_GAUSS) { launch_gram_t<f16, MT_F32, MODE_GAUSS>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F64 && mode == MODE_NONE) { launch_gram_t<f16, MT_F64, MODE_NONE>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_I8 && mode == MODE_STEP) { launch_gram_t<f16, MT_I8, MODE_STEP>(ga, maxt, rows, grid, lds, st); return true; }
  return false;
}

bool gram_dispatch_bf16(int mt, int mode, const GramArgs& ga, int maxt, int rows, int grid, size_t lds, hipStream_t st) {
  if (!gram_supported(PID_BF16, mt, mode)) return false;
  if (mt == MT_BF16 && mode == MODE_NONE) { launch_gram_t<bf16_t, MT_BF16, MODE_NONE>(ga, maxt, rows, grid, lds, st); return true; }
  if (mt == MT_F32 && mode == MODE_NONE) { launch_gram_t<bf16_t, MT_F32, MODE_NONE>(ga, maxt, rows, grid, lds, st); return true; }
  return false;
}

}  // namespace pidk

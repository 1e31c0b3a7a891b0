// Instantiations of the Gram kernel for the piecewise-linear probability
// models (ramp, tent, density) on FP32, FP16 and FP64 fields.
#include "gram_kernel.h"

namespace pidk {

bool gram_dispatch_model(int dtype, int mt, const GramArgs& ga, int maxt, int rows, int grid, size_t lds,
                         hipStream_t st) {
  if (!gram_supported(dtype, mt, MODE_MODEL)) return false;
  constexpr int M = MODE_MODEL;
  if (dtype == PID_F32) {
    if (mt == MT_F16) { launch_gram_t<float, MT_F16, M>(ga, maxt, rows, grid, lds, st); return true; }
    if (mt == MT_BF16X3) { launch_gram_t<float, MT_BF16X3, M>(ga, maxt, rows, grid, lds, st); return true; }
    if (mt == MT_F32) { launch_gram_t<float, MT_F32, M>(ga, maxt, rows, grid, lds, st); return true; }
  } else if (dtype == PID_F16) {
    if (mt == MT_F16) { launch_gram_t<f16, MT_F16, M>(ga, maxt, rows, grid, lds, st); return true; }
    if (mt == MT_F32) { launch_gram_t<f16, MT_F32, M>(ga, maxt, rows, grid, lds, st); return true; }
  } else if (dtype == PID_F64) {
    if (mt == MT_F64) { launch_gram_t<double, MT_F64, M>(ga, maxt, rows, grid, lds, st); return true; }
  }
  return false;
}

}  // namespace pidk

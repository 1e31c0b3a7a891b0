// Stand-ins for the kernel launchers, so that the host code of the library
// (argument checks, plans, workspace sizes, the serving calls) can be built
// with g++ and the sanitizers and run without a GPU.  Every launcher reports
// hipErrorNotSupported; the host-side tests only reach them when an argument
// check they expect to fail passes.
#include "../../paper_2512_15187_amd/csrc/pid_internal.h"

namespace pidk {
hipError_t launch_pid_mean(const MeanPlan&, const pid_ensemble&, int, const ExtractHost&, const pid_out&, void*,
                           hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_pairs_linear(const pid_ensemble&, int, const ExtractHost&, const pid_out&, void*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_pid_pairs(const PairsPlan&, const pid_ensemble&, int, const ExtractHost&, const pid_out&, void*,
                            hipStream_t, const pid_out*) { return hipErrorNotSupported; }
hipError_t launch_extract(const pid_ensemble&, int, const ExtractHost&, void*, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_rank(const double*, int64_t, int32_t*, int32_t*, hipStream_t, void*) { return hipErrorNotSupported; }
hipError_t launch_rank2(const double*, int32_t*, int32_t*, const double*, int32_t*, int32_t*, int64_t, hipStream_t, void*) {
  return hipErrorNotSupported;
}
hipError_t launch_bands(const pid_ensemble&, int, const ExtractHost&, const int32_t*, int64_t, int64_t, double,
                        uint8_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_validate(const pid_ensemble&, int, unsigned int*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_pid_mean_weighted(const pid_ensemble&, int, const ExtractHost&, const double*, const pid_out&,
                                    void*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_field_max(const pid_ensemble&, double*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_b1_mean(const pid_ensemble&, const pid_out&, void*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mask_bits_mean(const pid_ensemble&, int, const ExtractHost&, const pid_out&, void*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_pack_bits(const pid_ensemble&, uint32_t*, int64_t, hipStream_t) { return hipErrorNotSupported; }
}  // namespace pidk

// Small-n TSQR kernels, n = 1..32: FP32 input and arithmetic, row-major with any leading dimension.
#include "tsqr_small_inst.hpp"

namespace tsnmf {
hipError_t launch_small_f32_row(int n, const StreamArgs& a, hipStream_t stream) {
    using T_ = float;
    using TI_ = float;
    constexpr int LOAD_ = LOAD_ROW;
    TSNMF_SMALL_SWITCH
}
}  // namespace tsnmf

namespace tsnmf {
int rows_per_lane_f32(int n, bool staged) {
    using T_ = float;
    TSNMF_SMALL_RPL_SWITCH
}
int rows_per_lane_f64(int n, bool staged) {
    using T_ = double;
    TSNMF_SMALL_RPL_SWITCH
}
}  // namespace tsnmf

// Small-n TSQR kernels, n = 1..32: FP32 input widened exactly to FP64, FP64 arithmetic, column-major.
#include "tsqr_small_inst.hpp"

namespace tsnmf {
hipError_t launch_small_f32w_col(int n, const StreamArgs& a, hipStream_t stream) {
    using T_ = double;
    using TI_ = float;
    constexpr int LOAD_ = LOAD_COL;
    TSNMF_SMALL_SWITCH
}
}  // namespace tsnmf

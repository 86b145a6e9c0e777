// Small-n TSQR kernels, n = 1..32: FP64 input and arithmetic, contiguous row-major blocks.
#include "tsqr_small_inst.hpp"

namespace tsnmf {
hipError_t launch_small_f64_staged(int n, const StreamArgs& a, hipStream_t stream) {
    using T_ = double;
    using TI_ = double;
    constexpr int LOAD_ = LOAD_ROW_STAGED;
    TSNMF_SMALL_SWITCH
}
}  // namespace tsnmf

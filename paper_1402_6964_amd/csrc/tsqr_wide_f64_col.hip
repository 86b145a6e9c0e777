// Wide TSQR kernels (33..128 columns): FP64 input and arithmetic, column-major.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
hipError_t launch_wide_f64_col(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<double, double, 4, LOAD_COL, 16, 4>(a, stream);
    return launch_wide_w<double, double, 8, LOAD_COL, 16, 4>(a, stream);
}
}  // namespace tsnmf

// Wide TSQR kernels (33..128 columns): FP64 input and arithmetic, row-major.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
hipError_t launch_wide_f64_row(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<double, double, 4, LOAD_ROW, 16, 4>(a, stream);
    return launch_wide_w<double, double, 8, LOAD_ROW, 16, 4>(a, stream);
}
// Rows through a buffer resource per 64-row chunk (64 ld sizeof(TI) < 2^31).
hipError_t launch_wide_f64_rowbuf(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<double, double, 4, LOAD_ROW_BUF>(a, stream);
    return launch_wide_w<double, double, 8, LOAD_ROW_BUF>(a, stream);
}
}  // namespace tsnmf

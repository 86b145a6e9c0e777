// Wide TSQR kernels (33..128 columns): FP32 input and arithmetic, column-major.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
// Column-major blocks read whole column segments per wave, so more waves with
// fewer columns each cost no extra L2 traffic: 8 waves x 8 columns for up to
// 64 columns, 22 rows per lane (5e7 x 64: 13.9 ms with 4 waves x 16 columns,
// 11.8 ms here).  Row-major blocks are read row by row by every wave, which
// favours fewer waves.
hipError_t launch_wide_f32_col(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<float, float, 8, LOAD_COL, 8, 22>(a, stream);
    return launch_wide_w<float, float, 8, LOAD_COL>(a, stream);
}
}  // namespace tsnmf

// Wide TSQR kernels (33..128 columns): FP32 input and arithmetic, row-major.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
// Up to 64 columns (4 waves, several workgroups per CU, so one workgroup's
// loads overlap another's steps): per-element loads, 12 rows per lane.
hipError_t launch_wide_f32_row(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<float, float, 4, LOAD_ROW, 16, 12>(a, stream);
    return launch_wide_w<float, float, 8, LOAD_ROW>(a, stream);
}
// Rows through a buffer resource per 64-row chunk (64 ld sizeof(TI) < 2^31).
hipError_t launch_wide_f32_rowbuf(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_f32_row(a, stream);
    return launch_wide_w<float, float, 8, LOAD_ROW_BUF>(a, stream);
}
}  // namespace tsnmf

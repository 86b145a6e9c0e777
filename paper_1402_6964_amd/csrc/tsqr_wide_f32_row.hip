// Wide TSQR kernels (33..128 columns): FP32 input and arithmetic, row-major.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
// Per-element loads, for row strides beyond the buffer path's 32-bit offsets.
hipError_t launch_wide_f32_row(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<float, float, 4, LOAD_ROW, 16, 12>(a, stream);
    return launch_wide_w<float, float, 8, LOAD_ROW>(a, stream);
}
// Rows through a buffer resource per 64-row chunk (64 ld sizeof(TI) < 2^31).
hipError_t launch_wide_f32_rowbuf(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<float, float, 4, LOAD_ROW_BUF, 16, 12>(a, stream);
    return launch_wide_w<float, float, 8, LOAD_ROW_BUF, 16, 12>(a, stream);
}
// Rows read coalesced and regrouped through LDS (16 columns per wave).
hipError_t launch_wide_f32_rowstg(const WideArgs& a, hipStream_t stream) {
    if (a.n <= 64) return launch_wide_w<float, float, 4, LOAD_ROW_STAGED, 16, 12>(a, stream);
    return launch_wide_w<float, float, 8, LOAD_ROW_STAGED, 16, 12>(a, stream);
}
}  // namespace tsnmf

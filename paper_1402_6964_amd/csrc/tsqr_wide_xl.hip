// Wide TSQR kernels for 129..256 columns (every input type and layout): 8
// waves x 32 columns per slab, the running R of each workgroup in global
// memory.
#include "tsqr_wide_inst.hpp"

namespace tsnmf {
hipError_t launch_xl_f32_row(const WideArgs& a, hipStream_t s) { return launch_wide_xl<float, float, LOAD_ROW_STAGED>(a, s); }
hipError_t launch_xl_f32_col(const WideArgs& a, hipStream_t s) { return launch_wide_xl<float, float, LOAD_COL>(a, s); }
hipError_t launch_xl_f64_row(const WideArgs& a, hipStream_t s) { return launch_wide_xl<double, double, LOAD_ROW>(a, s); }
hipError_t launch_xl_f64_col(const WideArgs& a, hipStream_t s) { return launch_wide_xl<double, double, LOAD_COL>(a, s); }
hipError_t launch_xl_f32w_row(const WideArgs& a, hipStream_t s) { return launch_wide_xl<double, float, LOAD_ROW>(a, s); }
hipError_t launch_xl_f32w_col(const WideArgs& a, hipStream_t s) { return launch_wide_xl<double, float, LOAD_COL>(a, s); }
size_t xl_rslot_bytes() { return xl_slot_bytes(); }
}  // namespace tsnmf

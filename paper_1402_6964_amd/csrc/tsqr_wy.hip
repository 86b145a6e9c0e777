// Launchers of the compact-WY leaf (33..64 columns, FP32 row blocks): the
// leaf kernel over the row slabs, then the FP64 G-ary tree of the wide path
// over the slab factors.
#include "tsqr_wide_inst.hpp"
#include "tsqr_wy.hpp"

namespace tsnmf {

namespace {
constexpr int kWyWaves = 8;
constexpr int kWyTiles = 4;      // 16-row tiles per wave: 64 rows, 512-row blocks

template <int NT, int LOAD>
hipError_t launch_wy_nt(const WideArgs& a, hipStream_t stream) {
    using S = WY<NT, kWyWaves, kWyTiles>;
    auto kern = tsqr_wy_kernel<NT, kWyWaves, kWyTiles, LOAD>;
    const size_t lds = S::lds_bytes();
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.nstreams), dim3(kWyWaves * 64), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    return launch_wide_tree<16, 4, 4>(a, stream);
}
}  // namespace

int wy_block_rows() { return WY<4, kWyWaves, kWyTiles>::BR; }

hipError_t launch_wy_f32_col(const WideArgs& a, hipStream_t s) {
    return a.n <= 48 ? launch_wy_nt<3, LOAD_COL>(a, s) : launch_wy_nt<4, LOAD_COL>(a, s);
}
hipError_t launch_wy_f32_row(const WideArgs& a, hipStream_t s) {
    return a.n <= 48 ? launch_wy_nt<3, LOAD_ROW>(a, s) : launch_wy_nt<4, LOAD_ROW>(a, s);
}

}  // namespace tsnmf

// Launch helper for the small-n TSQR kernel; each translation unit that
// includes this file instantiates the kernels of one (compute, input) type pair
// for n = 1..32, so the instantiations compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "tsqr_small.hpp"

namespace tsnmf {

// Rows per lane of one block: as many as the register file allows while the
// block (RPL * n values per lane) and the step-0 partial sums stay resident.
// For FP32 widths 17, 20, 26 and 28 the budget rule lands a few registers
// above 256 (one wave per SIMD); they take the next smaller block.
template <typename T, int N> constexpr int small_rpl() {
    constexpr int words = (int)(sizeof(T) / 4);
    constexpr int budget = words == 1 ? 168 : 64;  // block registers, in elements of T
    constexpr int r = budget / N;
    constexpr int rpl = r >= 8 ? 8 : (r >= 6 ? 6 : (r >= 4 ? 4 : (r >= 2 ? 2 : 1)));
    constexpr bool tight = words == 1 && (N == 17 || N == 20 || N == 26 || N == 28);
    return !tight ? rpl : (rpl == 8 ? 6 : 4);
}

// One workgroup per group of leaves; later levels by ticket (tsqr_coop_tree.hip).
hipError_t launch_coop_tree(int n, const TreeArgs& t, hipStream_t stream);

template <typename T, typename TI, int N, int LOAD>
hipError_t launch_small_n(const StreamArgs& a, hipStream_t stream) {
    constexpr int RPL = small_rpl<T, N>();
    using S = Small<T, TI, N, RPL>;
    const size_t lds = S::lds_bytes(LOAD == LOAD_ROW_STAGED);
    auto kern = tsqr_small_kernel<T, TI, N, RPL, LOAD>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const unsigned grid = (unsigned)((a.nstreams + 3) / 4);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    // reduction tree (FP64 whatever the leaf type; its kernels live in one
    // translation unit)
    return launch_coop_tree(N, a.tree, stream);
}

#define TSNMF_SMALL_CASE(N) \
    case N: return launch_small_n<T_, TI_, N, LOAD_>(a, stream);

#define TSNMF_SMALL_SWITCH                                                             \
    switch (n) {                                                                       \
        TSNMF_SMALL_CASE(1) TSNMF_SMALL_CASE(2) TSNMF_SMALL_CASE(3) TSNMF_SMALL_CASE(4)     \
        TSNMF_SMALL_CASE(5) TSNMF_SMALL_CASE(6) TSNMF_SMALL_CASE(7) TSNMF_SMALL_CASE(8)     \
        TSNMF_SMALL_CASE(9) TSNMF_SMALL_CASE(10) TSNMF_SMALL_CASE(11) TSNMF_SMALL_CASE(12)  \
        TSNMF_SMALL_CASE(13) TSNMF_SMALL_CASE(14) TSNMF_SMALL_CASE(15) TSNMF_SMALL_CASE(16) \
        TSNMF_SMALL_CASE(17) TSNMF_SMALL_CASE(18) TSNMF_SMALL_CASE(19) TSNMF_SMALL_CASE(20) \
        TSNMF_SMALL_CASE(21) TSNMF_SMALL_CASE(22) TSNMF_SMALL_CASE(23) TSNMF_SMALL_CASE(24) \
        TSNMF_SMALL_CASE(25) TSNMF_SMALL_CASE(26) TSNMF_SMALL_CASE(27) TSNMF_SMALL_CASE(28) \
        TSNMF_SMALL_CASE(29) TSNMF_SMALL_CASE(30) TSNMF_SMALL_CASE(31) TSNMF_SMALL_CASE(32) \
        default: return hipErrorInvalidValue;                                          \
    }

#define TSNMF_SMALL_RPL_CASE(N) \
    case N: return small_rpl<T_, N>();

#define TSNMF_SMALL_RPL_SWITCH                                                                   \
    switch (n) {                                                                                 \
        TSNMF_SMALL_RPL_CASE(1) TSNMF_SMALL_RPL_CASE(2) TSNMF_SMALL_RPL_CASE(3) TSNMF_SMALL_RPL_CASE(4)     \
        TSNMF_SMALL_RPL_CASE(5) TSNMF_SMALL_RPL_CASE(6) TSNMF_SMALL_RPL_CASE(7) TSNMF_SMALL_RPL_CASE(8)     \
        TSNMF_SMALL_RPL_CASE(9) TSNMF_SMALL_RPL_CASE(10) TSNMF_SMALL_RPL_CASE(11) TSNMF_SMALL_RPL_CASE(12)  \
        TSNMF_SMALL_RPL_CASE(13) TSNMF_SMALL_RPL_CASE(14) TSNMF_SMALL_RPL_CASE(15) TSNMF_SMALL_RPL_CASE(16) \
        TSNMF_SMALL_RPL_CASE(17) TSNMF_SMALL_RPL_CASE(18) TSNMF_SMALL_RPL_CASE(19) TSNMF_SMALL_RPL_CASE(20) \
        TSNMF_SMALL_RPL_CASE(21) TSNMF_SMALL_RPL_CASE(22) TSNMF_SMALL_RPL_CASE(23) TSNMF_SMALL_RPL_CASE(24) \
        TSNMF_SMALL_RPL_CASE(25) TSNMF_SMALL_RPL_CASE(26) TSNMF_SMALL_RPL_CASE(27) TSNMF_SMALL_RPL_CASE(28) \
        TSNMF_SMALL_RPL_CASE(29) TSNMF_SMALL_RPL_CASE(30) TSNMF_SMALL_RPL_CASE(31) TSNMF_SMALL_RPL_CASE(32) \
        default: return 1;                                                                       \
    }

}  // namespace tsnmf

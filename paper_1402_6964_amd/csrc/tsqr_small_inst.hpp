// Launch helper for the small-n TSQR kernel; each translation unit that
// includes this file instantiates the kernels of one (compute, input) type pair
// for n = 1..32, so the instantiations compile in parallel.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "tsqr_small.hpp"

namespace tsnmf {

// Rows per lane of one block: as many as fit beside the block's partial sums
// in 256 registers (two waves per SIMD).  FP32 widths 9..32 take the largest
// value that the compiler fits without accumulation registers or spills
// (measured per width; the allocation does not grow monotonically with the
// block); other widths follow a register budget.
constexpr int kRplF32[33] = {8, 8, 8, 8, 8, 8, 8, 8, 8,            // 0..8
                             11, 11, 11, 10, 9, 11, 11, 10,       // 9..16
                             9, 8, 8, 7, 7, 7, 7, 6,              // 17..24
                             6, 5, 6, 5, 5, 5, 5, 5};             // 25..32
// Direct (unstaged) loads keep more addresses live: smaller blocks from 23
// columns on.
constexpr int kRplF32Direct[33] = {8, 8, 8, 8, 8, 8, 8, 8, 8,      // 0..8
                                   11, 11, 11, 10, 9, 11, 11, 10, // 9..16
                                   9, 8, 8, 7, 7, 7, 6, 6,        // 17..24
                                   5, 5, 5, 4, 4, 4, 4, 4};       // 25..32
template <typename T, int N, int LOAD = LOAD_ROW_STAGED> constexpr int small_rpl() {
    if constexpr (sizeof(T) == 4) {
        return LOAD == LOAD_ROW_STAGED ? kRplF32[N] : kRplF32Direct[N];
    } else {
        constexpr int r = 64 / N;                      // FP64: 64 block registers' worth of elements
        return r >= 8 ? 8 : (r >= 6 ? 6 : (r >= 4 ? 4 : (r >= 2 ? 2 : 1)));
    }
}

// One workgroup per group of leaves; later levels by ticket (tsqr_coop_tree.hip).
hipError_t launch_coop_tree(int n, const TreeArgs& t, hipStream_t stream);

template <typename T, typename TI, int N, int LOAD>
hipError_t launch_small_n(const StreamArgs& a, hipStream_t stream) {
    constexpr int RPL = small_rpl<T, N, LOAD>();
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
    case N: return staged ? small_rpl<T_, N, LOAD_ROW_STAGED>() : small_rpl<T_, N, LOAD_ROW>();

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

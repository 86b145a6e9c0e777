// Launch helper for the wide TSQR path (33..128 columns): the leaf kernel
// over row slabs followed by the FP64 tree over the slab factors.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "tsqr_wide.hpp"

namespace tsnmf {

// 16 columns per wave, W = 4 waves (up to 64 columns) or 8 (up to 128), and
// as many rows per lane as 128 block registers hold: fewer columns per wave
// mean a shorter butterfly per step and more rows to spread each step's fixed
// cost (reflector scalars, pivot exchange, barrier) over.
template <typename T> constexpr int wide_rpl() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T, typename TI, int W, int LOAD>
hipError_t launch_wide_w(const WideArgs& a, hipStream_t stream) {
    constexpr int NW = 16;
    constexpr int RPL = wide_rpl<T>();
    using S = Wide<T, TI, NW, W, RPL>;
    const size_t lds = S::lds_bytes();
    auto kern = tsqr_wide_kernel<T, TI, NW, W, RPL, LOAD>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.nstreams), dim3(W * 64), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    constexpr int NMAX = NW * W;
    constexpr int TW = NMAX <= 64 ? NMAX / 16 : NMAX / 8;    // 4 or 8 lanes per column
    const int64_t pairs = (a.tree.leaves + 1) / 2;
    auto tk = tsqr_wide_tree_kernel<NMAX, TW>;
    hipLaunchKernelGGL(tk, dim3((unsigned)pairs), dim3(TW * 64), 0, stream, a.tree, a.n);
    return hipGetLastError();
}

}  // namespace tsnmf

// Launch helper for the wide TSQR path (33..256 columns): the leaf kernel
// over row slabs followed by the G-ary FP64 tree over the slab factors.
#pragma once
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "tsqr_wide.hpp"

namespace tsnmf {

// 16 columns per wave, W = 4 waves (up to 64 columns) or 8 (up to 128), and
// as many rows per lane as 128 block registers hold: fewer columns per wave
// mean a shorter butterfly per step and more rows to spread each step's fixed
// cost (reflector scalars, pivot exchange, barrier) over.
template <typename T> constexpr int wide_rpl() { return sizeof(T) == 4 ? 11 : 5; }

// FP64 tree over the slab factors of `a`: groups of 4 stacked factors, each
// factored by the wide kernel in FP64 (NW x W columns).
template <int NW, int W, int RPLD, bool RG = false>
hipError_t launch_wide_tree(const WideArgs& a, hipStream_t stream) {
    constexpr int G = 4;
    using M = Wide<double, double, NW, W, RPLD, RG>;
    const size_t mlds = M::lds_bytes();
    auto mk = tsqr_wide_merge_kernel<NW, W, RPLD, G, RG>;
    if (mlds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)mk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds);
        if (e != hipSuccess) return e;
    }
    const int64_t groups = (a.tree.leaves + G - 1) / G;
    hipLaunchKernelGGL(mk, dim3((unsigned)groups), dim3(W * 64), mlds, stream, a.tree, a.n);
    return hipGetLastError();
}

template <typename T, typename TI, int W, int LOAD, int NW = 16, int RPL = wide_rpl<T>(), bool RG = false,
          int RPLD = 4>
hipError_t launch_wide_w(const WideArgs& a, hipStream_t stream) {
    using S = Wide<T, TI, NW, W, RPL, RG>;
    const size_t lds = S::lds_bytes(LOAD == LOAD_ROW_STAGED);
    auto kern = tsqr_wide_kernel<T, TI, NW, W, RPL, LOAD, RG>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)a.nstreams), dim3(W * 64), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    return launch_wide_tree<NW, W, RPLD, RG>(a, stream);
}

// 129..256 columns: 8 waves x 32 columns, R of each workgroup in a global
// slot (a.tree.rglob, one per leaf workgroup; the tree's workgroups reuse the
// first ones after the leaves are done).  Every R slot holds
// xl_slot_bytes() bytes.
constexpr int kXlRplF32 = 4;
constexpr int kXlRplF64 = 2;
constexpr size_t xl_slot_bytes() {
    return Wide<float, float, 32, 8, kXlRplF32, true>::slot_bytes() > Wide<double, double, 32, 8, kXlRplF64, true>::slot_bytes()
               ? Wide<float, float, 32, 8, kXlRplF32, true>::slot_bytes()
               : Wide<double, double, 32, 8, kXlRplF64, true>::slot_bytes();
}
template <typename T, typename TI, int LOAD>
hipError_t launch_wide_xl(const WideArgs& a, hipStream_t stream) {
    return launch_wide_w<T, TI, 8, LOAD, 32, sizeof(T) == 4 ? kXlRplF32 : kXlRplF64, true, kXlRplF64>(a, stream);
}

}  // namespace tsnmf

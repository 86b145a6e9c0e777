// FP64 reduction tree over the slab factors of the n <= 32 path: launch of
// the cooperative tree kernel (tsqr_small.hpp), one workgroup per group of
// leaves, later levels by ticket.  Instantiated in tsqr_coop_tree_*.hip,
// eight widths per file so that they compile in parallel.
#pragma once
#include "tsqr_coop.hpp"
#include "tsqr_small_inst.hpp"

namespace tsnmf {

template <int N> hipError_t launch_coop_tree_n(const TreeArgs& t, hipStream_t stream) {
    const int G = coop_group<N>(t.group);
    const int64_t groups = (t.leaves + G - 1) / G;
    hipLaunchKernelGGL(tsqr_coop_tree_kernel<N>, dim3((unsigned)groups), dim3(CoopTree<N>::W * 64), 0, stream, t);
    return hipGetLastError();
}

hipError_t launch_coop_tree_1_8(int n, const TreeArgs& t, hipStream_t stream);
hipError_t launch_coop_tree_9_16(int n, const TreeArgs& t, hipStream_t stream);
hipError_t launch_coop_tree_17_24(int n, const TreeArgs& t, hipStream_t stream);
hipError_t launch_coop_tree_25_32(int n, const TreeArgs& t, hipStream_t stream);

}  // namespace tsnmf

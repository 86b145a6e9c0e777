// TSQR of X = A (x) A without X in memory (FP32 row blocks formed from the
// factor A, FP64 tree): q = 1..5 columns of A, n = q^2.
#include "tsqr_small_inst.hpp"

namespace tsnmf {

namespace {
template <int N> hipError_t launch_kron_n(const StreamArgs& a, hipStream_t stream) {
    // the block height of the FP32 staged kernel of the same width, so a plan
    // made for the explicit X runs unchanged
    constexpr int RPL = small_rpl<float, N, LOAD_ROW_STAGED>();
    using S = Small<float, float, N, RPL>;
    const size_t lds = S::lds_bytes(false);
    auto kern = tsqr_small_kernel<float, float, N, RPL, LOAD_KRON>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)((a.nstreams + 3) / 4)), dim3(256), lds, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    return launch_coop_tree(N, a.tree, stream);
}
}  // namespace

hipError_t launch_small_kron(int q, const StreamArgs& a, hipStream_t stream) {
    switch (q) {
        case 1: return launch_kron_n<1>(a, stream);
        case 2: return launch_kron_n<4>(a, stream);
        case 3: return launch_kron_n<9>(a, stream);
        case 4: return launch_kron_n<16>(a, stream);
        case 5: return launch_kron_n<25>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tsnmf

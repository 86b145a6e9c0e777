// Leaf kernel for short FP64 slabs of the n <= 32 path (Sec. 3.1: the map
// stage factors blocks of rows).  A slab of at most 8 x 128 rows is one block
// held by the eight waves of a workgroup, factored by the cooperative
// Householder steps of the tree passes (the waves' partial sums added through
// LDS in wave order): n dependent steps per slab instead of n per 128 rows,
// which pays when there are too few slabs to fill the GPU (a 1,000-row leaf,
// one workgroup per slab).  The leaf node and its column sums go where the
// one-wave leaf stores them, and the tree runs unchanged.
#pragma once
#include "tsqr_coop_tree.hpp"

namespace tsnmf {

constexpr int64_t kCoopLeafRows = 8 * 64 * 2;   // CoopTree<N>::CAP for every N

template <int N>
__global__ void __launch_bounds__(512) tsqr_coop_leaf_kernel(StreamArgs a) {
    using CT = CoopTree<N>;
    using S = Small<double, double, N, CT::RPL>;
    static_assert(CT::CAP == kCoopLeafRows, "one block per slab");
    __shared__ CoopTreeLds<N> lds;
    const int wv = (int)(threadIdx.x >> 6);
    const int L = lane_id();
    const int64_t sid = blockIdx.x;
    double* Rl = lds.sR[wv];
    for (int i = L; i < S::RS; i += 64) Rl[i] = 0.0;
    wave_lds_sync();
    const int64_t r0 = sid * a.slab;
    const int64_t r1 = min(a.m, r0 + a.slab);
    double x[CT::RPL][N];
    S::template load<LOAD_ROW>(x, a, r0 + (int64_t)wv * S::BR, r1, nullptr);   // rows past r1 read as 0
    double acc = 0.0;
    S::colsum_block(x, acc);
    S::template step<0, CT::W, false>(x, Rl, lds.xchg, lds.wb[wv]);
    // column sums: each wave's, added in wave order
    int src = 0;                                        // lane holding column L's sum
    for (int s2 = 0; s2 < S::PN; ++s2) src |= ((L >> s2) & 1) << (5 - s2);
    const double v = lane_gather(acc, src);
    if (L < N) lds.csn[wv * N + L] = v;
    __syncthreads();
    if (wv != 0) return;
    double* out = a.tree.nodes + sid * (int64_t)N * N;
    int off = 0;
    for (int j = 0; j < N; ++j) {
        if (L < N) out[j * N + L] = L >= j ? Rl[off + (L - j)] : 0.0;
        off += pow2ceil(N - j);
    }
    if (L < N) {
        double cs = 0.0;
        for (int w = 0; w < CT::W; ++w) cs += lds.csn[w * N + L];
        a.tree.node_cs[sid * N + L] = cs;
    }
}

template <int N> hipError_t launch_coop_leaf_n(const StreamArgs& a, hipStream_t stream) {
    if (a.slab > kCoopLeafRows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tsqr_coop_leaf_kernel<N>, dim3((unsigned)a.nstreams), dim3(CoopTree<N>::W * 64), 0, stream,
                       a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    profile_split(stream);
    return launch_coop_tree(N, a.tree, stream);
}

hipError_t launch_coop_leaf_1_16(int n, const StreamArgs& a, hipStream_t stream);
hipError_t launch_coop_leaf_17_32(int n, const StreamArgs& a, hipStream_t stream);

}  // namespace tsnmf

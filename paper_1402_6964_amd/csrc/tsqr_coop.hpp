// Cooperative FP64 reduction tree over the slab factors of the n <= 32 path
// (and of the small classes of the batched kernel).
#pragma once
#include "tsqr_small.hpp"

namespace tsnmf {

// One pass of a workgroup (8 waves) reduces a group of G consecutive nodes of
// the current tree level to one node: the G stacked n x n triangles are rows of
// a single block of 8 x 128 rows, factored by the same structured Householder
// steps in FP64 with the waves' partial sums added through LDS in wave order
// (Sec. 3.5: the reduce stage factors the stacked R factors).  The node goes to
// the next level; by ticket, the last workgroup of each group of G continues
// with that group, so all levels run in one launch.  The pass that finds a
// single node at the next level writes the final R (column-major, rows
// flipped to a nonnegative diagonal) and the column sums.  Groups and orders
// are fixed, so the result is deterministic.
template <int N, int W_ = 8> struct CoopTree {
    static constexpr int W = W_;                      // waves per workgroup
    static constexpr int RPL = 2;                     // FP64 rows per lane
    static constexpr int CAP = W * 64 * RPL;          // rows per pass
    static constexpr int G = CAP / N < 64 ? CAP / N : 64;   // nodes per pass
};

template <int N, int W = 8> struct CoopTreeLds {
    using S = Small<double, double, N, CoopTree<N, W>::RPL>;
    double sR[W][S::RS];
    double xchg[2 * W * 64];
    alignas(16) double wb[W][S::BCE];
    double csn[CoopTree<N, W>::CAP];                   // the group's column sums
    int go;
};

// The whole workgroup (W waves) reduces group `group0` of level 0 and climbs.
// Nodes per group: t.group when set (2 .. CT::G), else a default by width.
// A pass costs about the same per stacked row whatever the group size, but
// it runs on one workgroup, so smaller groups spread the first level over
// more workgroups; measured on 2048 slab factors, 16 nodes per pass (20 for
// 10..19 columns) beat the full 1024-row pass (n = 25: 88 against 132 us).
template <int N, int W = 8> __host__ __device__ constexpr int coop_group(int group) {
    constexpr int cap = CoopTree<N, W>::G;
    constexpr int dflt = N >= 20 ? 16 : (N >= 10 ? 20 : cap);
    const int g = group == 0 ? dflt : group;
    return g >= 2 && g < cap ? g : cap;
}

// Factor `rows` stacked FP64 rows at `src` (n wide) with WA of the W waves
// (WA = the fewest that hold them, a power of two): idle waves only match the
// per-step barriers, so a small group runs at the speed of a small workgroup.
template <int N, int W, int WA>
__device__ __forceinline__ void coop_factor(const double* src, int rows, double* Rl, double* xchg, double* wb, int wv,
                                            int L) {
    using CT = CoopTree<N, W>;
    using S = Small<double, double, N, CT::RPL>;
    if (wv < WA) {
        double x[CT::RPL][N];
#pragma unroll
        for (int r = 0; r < CT::RPL; ++r) {
            const int b = wv * (64 * CT::RPL) + r * 64 + L;
            const bool ok = b < rows;
            const double* rowp = src + (int64_t)min(b, rows - 1) * N;
#pragma unroll
            for (int c = 0; c < N; ++c) x[r][c] = ok ? rowp[c] : 0.0;
        }
        S::template step<0, WA, false>(x, Rl, xchg, wb);
    } else if constexpr (WA > 1) {
        for (int j = 0; j < N; ++j) __syncthreads();   // one barrier per step of the active waves
    }
}

template <int N, int W = 8>
__device__ __forceinline__ void coop_tree_run(const TreeArgs& t, int64_t group0, CoopTreeLds<N, W>& lds) {
    using CT = CoopTree<N, W>;
    using S = Small<double, double, N, CT::RPL>;
    const int G = coop_group<N, W>(t.group);
    constexpr int64_t NN = (int64_t)N * N;
    double* xchg = lds.xchg;
    int& go = lds.go;
    const int wv = (int)(threadIdx.x >> 6);
    const int L = lane_id();
    double* Rl = lds.sR[wv];

    int64_t group = group0;       // group index within the current level
    int64_t count = t.leaves;     // nodes at the current level
    int64_t base = 0;             // node offset of the current level
    int64_t tbase = 0;            // ticket offset of the next level
    while (true) {
        const int64_t first = group * G;
        const int rows = (int)min((int64_t)G, count - first) * N;
        for (int i = L; i < S::RS; i += 64) Rl[i] = 0.0;
        wave_lds_sync();
        const double* src = t.nodes + (base + first) * NN;    // stacked rows, n wide
        // The group's column sums (rows / n nodes of n values, contiguous):
        // loaded by every thread now, so that they arrive during the factor,
        // and summed in node order after it.
        const double* csrc = t.node_cs + (base + first) * N;
        double pre[CT::RPL];
#pragma unroll
        for (int u = 0; u < CT::RPL; ++u) {
            const int e = (int)threadIdx.x + u * W * 64;
            pre[u] = e < rows ? csrc[e] : 0.0;
        }
        const int need = (rows + 64 * CT::RPL - 1) / (64 * CT::RPL);
        double* wb = lds.wb[wv];
        if (need <= 1) coop_factor<N, W, 1>(src, rows, Rl, xchg, wb, wv, L);
        else if (W >= 2 && need <= 2) coop_factor<N, W, (W >= 2 ? 2 : 1)>(src, rows, Rl, xchg, wb, wv, L);
        else if (W >= 4 && need <= 4) coop_factor<N, W, (W >= 4 ? 4 : 1)>(src, rows, Rl, xchg, wb, wv, L);
        else coop_factor<N, W, W>(src, rows, Rl, xchg, wb, wv, L);
        wave_lds_sync();
#pragma unroll
        for (int u = 0; u < CT::RPL; ++u) {
            const int e = (int)threadIdx.x + u * W * 64;
            if (e < rows) lds.csn[e] = pre[u];
        }
        __syncthreads();
        double cs = 0.0;
        if (wv == 0 && L < N) {
            const int cnt = rows / N;
            for (int q = 0; q < cnt; ++q) cs += lds.csn[q * N + L];
        }
        const int64_t ncount = (count + G - 1) / G;
        if (ncount == 1) {                                   // root
            if (wv == 0) {
                int off = 0;
                for (int j = 0; j < N; ++j) {
                    const double djj = Rl[off];
                    if (L < N) t.R[(int64_t)L * N + j] = L >= j ? (djj < 0.0 ? -Rl[off + L - j] : Rl[off + L - j]) : 0.0;
                    off += pow2ceil(N - j);
                }
                if (t.colsum != nullptr && L < N) t.colsum[L] = cs;
            }
            return;
        }
        const int64_t nbase = base + count;
        if (wv == 0) {
            double* out = t.nodes + (nbase + group) * NN;
            int off = 0;
            for (int j = 0; j < N; ++j) {
                if (L < N) out[j * N + L] = L >= j ? Rl[off + (L - j)] : 0.0;
                off += pow2ceil(N - j);
            }
            if (L < N) t.node_cs[(nbase + group) * N + L] = cs;
        }
        // Only wave 0 stored, and its thread 0 takes the ticket: one release
        // fence (an L2 write-back) per pass, not one per wave; with a hundred
        // workgroups finishing a level together the write-backs queue up.
        if (wv == 0) grid_release();
        __syncthreads();
        const int64_t ngroup = group / G;
        const int gsize = (int)min((int64_t)G, ncount - ngroup * G);
        if (threadIdx.x == 0) {
            const int old = __hip_atomic_fetch_add(t.tickets + tbase + ngroup, 1, __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            const int last = old == gsize - 1;
            if (last) __hip_atomic_store(t.tickets + tbase + ngroup, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            go = last;
        }
        __syncthreads();
        if (!go) return;
        grid_acquire();
        tbase += (ncount + G - 1) / G;
        base = nbase;
        count = ncount;
        group = ngroup;
    }
}

template <int N>
__global__ void __launch_bounds__(512) tsqr_coop_tree_kernel(TreeArgs t) {
    __shared__ CoopTreeLds<N> lds;
    coop_tree_run<N>(t, blockIdx.x, lds);
}

}  // namespace tsnmf

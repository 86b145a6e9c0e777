// Blocked Householder leaf with a compact-WY trailing update on the matrix
// cores, for 33..64 columns (FP32 row blocks, FP64 running R).
//
// Same algebra as the unblocked leaf (tsqr_small.hpp): the row block B and
// the running R of the slab form [R; B], reflector j is [e_j; y_j] with
// y_j = B(:, j) / (alpha - beta), and only R is kept.  Columns are taken in
// panels of 16 (Sec. 3.1 allows any order of the Householder steps as long as
// each reflector sees the columns already transformed by the previous ones):
//   - the 16 steps of a panel touch only the panel's columns (vector ALUs);
//   - then the panel's reflectors are applied to the trailing columns at once.
//     With V = [E_P; Y] (E_P the unit vectors of the panel's rows of R) the
//     product H_p0 ... H_p15 is I - V T V^T; instead of forming T, the rows of
//     W = T^T V^T [R; B](:, trail) follow from the forward recurrence
//         w_j = tau_j (m_j - sum_{k < j} (y_k^T y_j) w_k),
//         m_j = R(j, trail) + y_j^T B(:, trail),
//     and then R(P, trail) -= W, B(:, trail) -= Y W.
//   Y^T [Y | B(:, trail)] and Y W are matrix products: v_mfma_f32_16x16x4_f32.
//
// Register layout: a wave holds 16 * TW rows of the block and all NT * 16
// columns as 16 x 16 tiles; in tile (t, u) lane (g, c) = (L / 16, L % 16)
// register i holds B(16 t + 4 g + i, 16 u + c).  This is the layout of both
// MFMA operands of Y^T B (the contraction runs over rows: four per
// instruction, one per lane group) and of the MFMA accumulator of Y W, so the
// trailing columns never leave their registers.  Only Y is re-laid out (rows
// across lanes) through LDS once per panel for the A operand of Y W.
// Inside a panel step the pivot column is broadcast within each 16-lane row
// by DPP row_newbcast, the partial dot products of the lane groups are added
// by two permlane swaps and those of the W waves through LDS (one barrier per
// step); every wave then forms the same FP64 reflector scalars.
#pragma once
#include "tsqr_wide.hpp"

namespace tsnmf {

typedef float wy_f4 __attribute__((ext_vector_type(4)));

// Value of lane N (0..15) of this lane's 16-lane row.
template <int N> __device__ __forceinline__ float row_bcast(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + N, 0xf, 0xf, true));
}

// The same value, opaque to the optimiser.  Lane coordinates are passed
// through it once per row block, so that the address and lane-mask
// computations of the unrolled steps stay inside the block loop instead of
// being hoisted out of it (hundreds of values held in registers across it).
__device__ __forceinline__ int opaque_v(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ int opaque_s(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

template <int NT, int W, int TW> struct WY {
    static_assert(NT >= 1 && NT <= 4, "WY leaf covers up to 64 columns");
    static constexpr int NP = 16 * NT;            // padded width
    static constexpr int BW = 16 * TW;            // rows of a block held by one wave
    static constexpr int BR = W * BW;             // rows per block
    static constexpr int YS = 17;                 // Y staging row stride (odd: no bank conflicts)
    // LDS, in bytes: R (NP x NP FP64, row-major) | dot partials [2][W][16] f32 |
    // Z partials [W][16][NP] f32 | -W [16][NP] f32 | Y staging [W][BW][YS] f32 |
    // tau, s [2][16] f64 | column-sum partials [W][NP] f64
    static constexpr size_t oR = 0;
    static constexpr size_t oD = oR + (size_t)NP * NP * 8;
    static constexpr size_t oZ = oD + (size_t)2 * W * 16 * 4;
    static constexpr size_t oW = oZ + (size_t)W * 16 * NP * 4;
    static constexpr size_t oY = oW + (size_t)16 * NP * 4;
    static constexpr size_t oS = (oY + (size_t)W * BW * YS * 4 + 7) & ~(size_t)7;
    static constexpr size_t oC = oS + (size_t)2 * 16 * 8;
    static constexpr size_t lds_bytes() { return oC + (size_t)W * NP * 8; }

    struct Ctx {
        double* R;
        float* dsum;
        float* zp;
        float* wneg;
        float* ys;
        double* tau;
        double* sv;
        int wv, L, g, c, n;
    };

    // ---- one Householder step inside panel P (global column j = 16 P + JJ) ----
    template <int P, int JJ>
    static __device__ __forceinline__ void step(float (&x)[TW][NT][4], const Ctx& k, float& s_own) {
        constexpr int j = 16 * P + JJ;
        if (j >= k.n) return;                          // uniform
        const int col = 16 * P + k.c;
        // row j of R for this lane's panel column, and R(j, j): written at
        // step j of the previous block, read here before this step's barrier
        const double rj = k.R[j * NP + col];
        const double alpha = k.R[j * NP + j];
        float bc[TW][4];
        float d = 0.0f;
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bc[t][i] = row_bcast<JJ>(x[t][P][i]);
                d = __builtin_fmaf(bc[t][i], x[t][P][i], d);
            }
        d = allreduce_stage<5>(d);                     // add the four lane groups
        d = allreduce_stage<4>(d);
        float D = d;
        if constexpr (W > 1) {
            float* db = k.dsum + (j & 1) * (W * 16);   // alternate buffers: one barrier per step
            if (k.L < 16) db[k.wv * 16 + k.L] = d;
            __syncthreads();
            D = db[k.c];
#pragma unroll
            for (int q = 1; q < W; ++q) D += db[q * 16 + k.c];
        }
        // reflector scalars in FP64, the same in every wave (same inputs, same order)
        const double sigma = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(D), JJ));
        const bool live = sigma != 0.0;
        const double nrm = sqrt_normal(__builtin_fma(alpha, alpha, sigma));
        const double beta = live ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
        const double amb = alpha - beta;
        const double q = rcp_fast<double>(beta * amb);  // unused unless live
        const double inv_beta = amb * q;
        const double s = live ? beta * q : 0.0;         // 1 / (alpha - beta)
        const double tau = live ? (beta - alpha) * inv_beta : 0.0;
        const double w = __builtin_fma(s, (double)D, rj);   // v^T [R; B](:, col)
        if (k.wv == 0 && k.g == 0 && k.c >= JJ) k.R[j * NP + col] = k.c == JJ ? beta : __builtin_fma(-tau, w, rj);
        if (k.wv == 0 && k.L == 0) {
            k.tau[JJ] = tau;
            k.sv[JJ] = s;
        }
        if (k.c == JJ) s_own = (float)s;
        // B(:, col) += B(:, j) w / beta on the panel columns right of j
        const float cw = (k.c > JJ && live) ? (float)(inv_beta * w) : 0.0f;
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) x[t][P][i] = __builtin_fmaf(bc[t][i], cw, x[t][P][i]);
    }

    template <int P, int JJ>
    static __device__ __forceinline__ void steps(float (&x)[TW][NT][4], const Ctx& k, float& s_own) {
        if constexpr (JJ < 16) {
            step<P, JJ>(x, k, s_own);
            steps<P, JJ + 1>(x, k, s_own);
        }
    }

    // ---- trailing update of panel P: W from Y^T [Y | B(:, trail)], then B -= Y W ----
    template <int P>
    static __device__ __forceinline__ void trail(float (&x)[TW][NT][4], const Ctx& k, float s_own) {
        constexpr int NU = NT - P;                     // tiles P (Y^T Y) .. NT-1
        // Y in place: column 16 P + c scaled by s = 1 / (alpha - beta) of its step
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) x[t][P][i] *= s_own;
        wy_f4 z[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            z[u] = wy_f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    z[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[t][P][i], x[t][P + u][i], z[u], 0, 0, 0);
        }
        // this wave's partial Z(4 g + e, 16 (P + u) + c); the barrier also
        // orders this panel's last R writes before wave 0 reads them below
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int e = 0; e < 4; ++e) k.zp[(k.wv * 16 + 4 * k.g + e) * NP + 16 * (P + u) + k.c] = z[u][e];
        __syncthreads();
        // Z summed over the waves in wave order, in place into wave 0's rows
        if constexpr (W > 1) {
            constexpr int ZC = NP - 16 * P;            // columns 16 P .. NP-1
            for (int e = (int)threadIdx.x; e < 16 * ZC; e += W * 64) {
                const int jj = e / ZC, col = 16 * P + e % ZC;
                float zsum = k.zp[jj * NP + col];
#pragma unroll
                for (int q = 1; q < W; ++q) zsum += k.zp[(q * 16 + jj) * NP + col];
                k.zp[jj * NP + col] = zsum;
            }
            __syncthreads();
        }
        // wave 0: W by the forward recurrence, one trailing column per lane;
        // R(P, trail) -= W; -W to LDS in FP32
        if (k.wv == 0) {
            const int col = 16 * (P + 1) + k.L;
            if (col < NP) {
                double acc[16];                        // m_jj, less the terms of earlier rows
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) acc[jj] = k.R[(16 * P + jj) * NP + col] + (double)k.zp[jj * NP + col];
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const double wj = k.tau[jj] * acc[jj];
                    k.R[(16 * P + jj) * NP + col] -= wj;
                    k.wneg[jj * NP + col] = (float)(-wj);
#pragma unroll
                    for (int kk = jj + 1; kk < 16; ++kk)      // y_jj^T y_kk
                        acc[kk] = __builtin_fma(-(double)k.zp[jj * NP + 16 * P + kk], wj, acc[kk]);
                    // one row of y^T y at a time: keeps the loads of later rows
                    // from being hoisted (and held in registers) here
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        // Y with rows across lanes (A operand of Y W) through this wave's staging area
        float* ys = k.ys + (size_t)k.wv * BW * YS;
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) ys[(16 * t + 4 * k.g + i) * YS + k.c] = x[t][P][i];
        __syncthreads();                               // -W is ready (also orders the staging writes)
        float yt[TW][4];
#pragma unroll
        for (int t = 0; t < TW; ++t)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) yt[t][s4] = ys[(16 * t + (k.L & 15)) * YS + 4 * s4 + k.g];
#pragma unroll
        for (int u = 1; u < NU; ++u) {
            float wb[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) wb[s4] = k.wneg[(4 * s4 + k.g) * NP + 16 * (P + u) + k.c];
#pragma unroll
            for (int t = 0; t < TW; ++t) {
                wy_f4 a = wy_f4{x[t][P + u][0], x[t][P + u][1], x[t][P + u][2], x[t][P + u][3]};
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) a = __builtin_amdgcn_mfma_f32_16x16x4f32(yt[t][s4], wb[s4], a, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) x[t][P + u][i] = a[i];
            }
        }
    }

    template <int P>
    static __device__ __forceinline__ void panels(float (&x)[TW][NT][4], const Ctx& k) {
        if constexpr (P < NT) {
            if (16 * P >= k.n) return;
            float s_own = 0.0f;
            steps<P, 0>(x, k, s_own);
            if constexpr (P + 1 < NT) {
                if (16 * (P + 1) < k.n) trail<P>(x, k, s_own);
            }
            panels<P + 1>(x, k);
        }
    }
};

// One workgroup (W waves) factors slab `sid` of `a` and stores leaf node `sid`.
template <int NT, int W, int TW, int LOAD>
__device__ __forceinline__ void wy_slab(const WideArgs& a, int64_t sid, unsigned char* smem) {
    using S = WY<NT, W, TW>;
    constexpr int NP = S::NP;
    typename S::Ctx k;
    k.R = (double*)(smem + S::oR);
    k.dsum = (float*)(smem + S::oD);
    k.zp = (float*)(smem + S::oZ);
    k.wneg = (float*)(smem + S::oW);
    k.ys = (float*)(smem + S::oY);
    k.tau = (double*)(smem + S::oS);
    k.sv = k.tau + 16;
    k.wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    k.L = lane_id();
    k.g = k.L >> 4;
    k.c = k.L & 15;
    k.n = a.n;
    double* csw = (double*)(smem + S::oC);
    const int n = a.n;
    const int tid = (int)threadIdx.x;
    for (int i = tid; i < NP * NP; i += W * 64) k.R[i] = 0.0;

    const int64_t r0 = sid * a.slab;
    const int64_t r1 = min(a.m, r0 + a.slab);
    const float* X = (const float*)a.X;
    double cs[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) cs[u] = 0.0;
    __syncthreads();
    for (int64_t b0 = r0; b0 < r1; b0 += S::BR) {
        float x[TW][NT][4];
        const int64_t wr = b0 + (int64_t)k.wv * S::BW;      // this wave's first row
        if (LOAD == LOAD_COL && b0 + S::BR <= r1) {
            // whole block in range: one base pointer per column tile, the
            // rows at constant offsets from it
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int colu = 16 * u + k.c;
                const float* pu = X + (int64_t)min(colu, n - 1) * a.ld + wr + 4 * k.g;
#pragma unroll
                for (int t = 0; t < TW; ++t)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float v = __builtin_nontemporal_load(pu + 16 * t + i);
                        x[t][u][i] = colu < n ? v : 0.0f;
                    }
            }
        } else {
#pragma unroll
            for (int t = 0; t < TW; ++t)
#pragma unroll
                for (int u = 0; u < NT; ++u) {
                    const int colu = 16 * u + k.c;
                    const bool okc = colu < n;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t row = wr + 16 * t + 4 * k.g + i;
                        const bool ok = okc && row < r1;
                        const float* p = LOAD == LOAD_COL ? X + min(row, a.m - 1) + (int64_t)min(colu, n - 1) * a.ld
                                                          : X + min(row, a.m - 1) * a.ld + min(colu, n - 1);
                        const float v = LOAD == LOAD_COL ? __builtin_nontemporal_load(p) : *p;
                        x[t][u][i] = ok ? v : 0.0f;
                    }
                }
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {                 // l1 column sums: FP32 over four rows, then FP64
#pragma unroll
            for (int t = 0; t < TW; ++t)
                cs[u] += (double)(__builtin_fabsf(x[t][u][0]) + __builtin_fabsf(x[t][u][1]) +
                                  __builtin_fabsf(x[t][u][2]) + __builtin_fabsf(x[t][u][3]));
        }
        // the first step of this block reuses LDS slots the previous block's
        // last steps and panel update may still be reading
        if (b0 != r0) __syncthreads();
        typename S::Ctx kb = k;
        kb.L = opaque_v(k.L);
        kb.g = kb.L >> 4;
        kb.c = kb.L & 15;
        kb.wv = opaque_s(k.wv);
        kb.n = opaque_s(k.n);
        S::template panels<0>(x, kb);
    }
    __syncthreads();
    // leaf node: row-major n x n FP64, zeros below the diagonal
    double* out = a.tree.nodes + sid * (int64_t)n * n;
    for (int i = tid; i < n * n; i += W * 64) {
        const int r = i / n, cc = i % n;
        out[i] = cc >= r ? k.R[r * NP + cc] : 0.0;
    }
    // column sums: lane groups, then waves in order
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        double v = allreduce_stage<5>(cs[u]);
        v = allreduce_stage<4>(v);
        if (k.L < 16) csw[k.wv * NP + 16 * u + k.L] = v;
    }
    __syncthreads();
    if (a.tree.node_cs != nullptr && tid < n) {
        double v = csw[tid];
        for (int q = 1; q < W; ++q) v += csw[q * NP + tid];
        a.tree.node_cs[sid * n + tid] = v;
    }
}

template <int NT, int W, int TW, int LOAD>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(2))) tsqr_wy_kernel(WideArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    wy_slab<NT, W, TW, LOAD>(a, blockIdx.x, smem);
}

}  // namespace tsnmf

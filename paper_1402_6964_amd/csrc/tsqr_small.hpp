// Streaming Householder TSQR kernel for n <= 32 columns (one wave per slab).
//
// Each wave owns a contiguous slab of rows and keeps the n x n R factor of
// all rows it has seen so far (Sec. 3.1: only R is formed).  It reads its slab
// in row blocks of 64 * RPL rows -- lane L holds rows L, L + 64, ... of the
// block, one register per (row, column) -- and folds each block into R with
// the structured Householder QR of [R; B]: reflector j is [e_j; y] with
// y = B(:, j) / (alpha - beta), so it touches row j of R and all block rows.
// With d_k = B(:, j)^T B(:, k) (k >= j), sigma = d_j and alpha = R(j, j):
//     beta = -sign(alpha) sqrt(alpha^2 + sigma),  tau = (beta - alpha) / beta,
//     w_k  = R(j, k) + d_k / (alpha - beta)        (= v^T [R; B](:, k)),
//     R(j, k) <- R(j, k) - tau w_k  (R(j, j) <- beta),
//     B(:, k) <- B(:, k) + (1 / beta) B(:, j) w_k  (since tau / (alpha - beta) = -1 / beta).
// All d_k of one step come from one reduce-scatter butterfly (wave.hpp), so
// value k - j of step j lives in a fixed lane pattern; row j of R is stored in
// LDS indexed by that value number, so the R update is one lane-parallel op,
// and the w_k reach every lane through a small LDS slot per wave.
// The block's l1 column sums (Sec. 3.3) are reduced by one more butterfly and
// accumulated in FP64.
//
// The slab factors are then combined by the FP64 tree of tsqr_coop.hpp.
#pragma once
#include "tsqr_tree.hpp"
#include "wave.hpp"

namespace tsnmf {

// LOAD_KRON: no X in memory; row i p + i' of X = A (x) A is formed from rows
// i and i' of the small factor A (p x q, row-major, ld) as the products
// A(i, a) A(i', b) in column a q + b (the construction of the flow-cytometry
// matrix in Sec. 5.2).
enum LoadKind : int { LOAD_ROW = 0, LOAD_ROW_STAGED = 1, LOAD_COL = 2, LOAD_KRON = 4 };
// Largest slab (bytes) of the FP32 staged path, which addresses a slab
// through one buffer resource with a 32-bit byte range.
constexpr int64_t kMaxBufSlabBytes = ((int64_t)1 << 31) - 4096;

struct StreamArgs {
    const void* X;         // input of element type TI, rows [0, m)
    int64_t m;             // rows
    int64_t ld;            // leading dimension (elements)
    int64_t slab;          // rows per stream
    int64_t nstreams;      // streams (one wave each) = tree leaves
    TreeArgs tree;         // reduction tree and final outputs
    int64_t kp;            // LOAD_KRON: rows p of the factor A (X has p^2 rows)
};

// 1 / x: the hardware estimate in FP32; in FP64 the estimate refined by two
// Newton steps (each squares the relative error).
template <typename T> __device__ __forceinline__ T rcp_fast(T x);
template <> __device__ __forceinline__ float rcp_fast<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp_fast<double>(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float abs_t(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double abs_t(double a) { return __builtin_fabs(a); }
template <typename T> __device__ __forceinline__ T sqrt_t(T x);
template <> __device__ __forceinline__ float sqrt_t<float>(float x) { return __builtin_sqrtf(x); }
template <> __device__ __forceinline__ double sqrt_t<double>(double x) { return __builtin_sqrt(x); }

// sqrt(x) for x in the normal FP64 range (not zero, not infinite): the
// hardware reciprocal-square-root estimate refined by one coupled Newton step
// for g = sqrt(x) and h = 1 / (2 sqrt(x)) (Goldschmidt's iteration), then one
// residual correction of g, so the result is within an ulp or two.
__device__ __forceinline__ double sqrt_normal(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}

// sqrt(x) and 1 / sqrt(x) for x in the normal FP64 range, from the same
// refinement as sqrt_normal: after the coupled Newton step h = 1 / (2
// sqrt(x)) has about twice the estimate's correct bits (enough for the
// reflector scalars that use it), and g gets the residual correction.
struct SqrtRsq {
    double g, y;
};
__device__ __forceinline__ SqrtRsq sqrt_rsq_normal(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    return {__builtin_fma(d, h, g), 2.0 * h};
}

// T: arithmetic of the block (its dot products and updates); TI: input
// element type; R, alpha, sigma and the reflector scalars are kept in FP64
// (TR), so that the running factor of a long slab does not accumulate FP32
// rounding from block to block.
template <typename T, typename TI, int N, int RPL> struct Small {
    static_assert(N >= 1 && N <= 32, "small kernel covers 1..32 columns");
    using TR = double;
    static constexpr int BR = 64 * RPL;                   // rows per block
    static constexpr int PN = ilog2(pow2ceil(N));         // butterfly order of n values
    static constexpr int roff(int j) {
        int o = 0;
        for (int t = 0; t < j; ++t) o += pow2ceil(N - t);
        return o;
    }
    static constexpr int RS = roff(N);                    // R slots per wave (elements of T)
    static constexpr int SS = (N % 2) ? N : N + 1;        // staging row stride, odd -> no bank conflicts
    static constexpr int STG = 64 * SS;                   // staging elements (TI) per wave
    // w slot per wave (T): one value per butterfly index, 16-byte multiple
    static constexpr int BCE = (int)(((pow2ceil(N) * sizeof(T) + 15) & ~(size_t)15) / sizeof(T));
    // LDS of a workgroup of `wpg` waves: every wave's R, then every wave's
    // staging area (staged loads only), then every wave's w slot
    static constexpr size_t r_bytes(int wpg = 4) { return (size_t)wpg * RS * sizeof(TR); }
    static constexpr size_t stage_off(int wpg = 4) { return (r_bytes(wpg) + 15) & ~(size_t)15; }
    static constexpr size_t bc_off(bool staged, int wpg = 4) {
        return stage_off(wpg) + (staged ? ((size_t)wpg * STG * sizeof(TI) + 15) & ~(size_t)15 : 0);
    }
    static constexpr size_t lds_bytes(bool staged, int wpg = 4) {
        return bc_off(staged, wpg) + (size_t)wpg * BCE * sizeof(T);
    }

    // ---- one Householder step (column J) -------------------------------------
    // With `xchg` non-null, W waves of a workgroup hold different rows of the
    // same block: after its butterfly each wave publishes its 64 lane values,
    // and every wave adds all W of them in wave order (the same sums in every
    // wave, so the W copies of R stay identical).
    // LB: `wb` is the wave's w slot (BCE elements, 16-byte aligned); the
    // lanes store w_{J+v} at index v (padding indices v >= n - J get w = 0,
    // never read) and every lane reads all of them back with 16-byte
    // broadcast reads, which keeps the per-column broadcasts off the vector
    // ALU (the leaf, bound by vector issue).  Without LB each w_k is read
    // from its lane into a scalar register, which is shorter in latency (the
    // tree, bound by the latency of its steps).
    template <int J, int W = 1, bool LB = true>
    static __device__ __forceinline__ void step(T (&x)[RPL][N], TR* Rl, T* xchg, T* wb) {
        if constexpr (J < N) {
            constexpr int CNT = N - J;
            constexpr int V = pow2ceil(CNT);
            constexpr int P = ilog2(V);
            const int L = lane_id();
            T p[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (v < CNT) {
                    T s = x[0][J] * x[0][J + v];
#pragma unroll
                    for (int r = 1; r < RPL; ++r) s = fma_t(x[r][J], x[r][J + v], s);
                    p[v] = s;
                } else {
                    p[v] = T(0);
                }
            }
            T D = butterfly<P, CNT>(p);              // lane L: d_{J + vidx(L)}
            if constexpr (W > 1) {
                const int wv = (int)(threadIdx.x >> 6);
                T* xb = xchg + (J & 1) * (W * 64);   // alternate buffers: one barrier per step
                xb[wv * 64 + L] = D;
                __syncthreads();
                D = xb[L];
#pragma unroll
                for (int q = 1; q < W; ++q) D += xb[q * 64 + L];
            }
            const int vi = bfly_vidx<P>(L);
            TR* row = Rl + roff(J);
            const TR rj = row[vi];                   // R(J, J + vi), zero in padding slots
            const TR DR = (TR)D;
            const TR sigma = lane_bcast(DR, 0);
            const TR alpha = lane_bcast(rj, 0);
            // sigma is wave-uniform (a lane broadcast): a column already zero
            // below the diagonal of this block (sigma = 0) leaves R and the
            // block unchanged, so the whole step is skipped by a scalar branch
            // and the common path carries no selects.  Otherwise alpha^2 +
            // sigma > 0 and beta is nonzero.
            const bool live = sigma != TR(0);
            if (live) {
                TR beta, inv_beta, tau, w;
                if constexpr (sizeof(T) == 4) {
                    // FP32 block: sigma is a nonzero FP32 value, so alpha^2 +
                    // sigma and |alpha| + nrm lie far inside the normal FP64
                    // range.  With beta = -sign(alpha) nrm: 1 / beta =
                    // -sign(alpha) / nrm, tau = 1 + |alpha| / nrm, and
                    // 1 / (alpha - beta) = sign(alpha) / (|alpha| + nrm), whose
                    // sign goes into D, so one reciprocal (no cancellation)
                    // follows the square root on the step's critical path.
                    const SqrtRsq sr = sqrt_rsq_normal(fma_t(alpha, alpha, sigma));
                    const TR aa = abs_t(alpha);
                    beta = __builtin_copysign(sr.g, -alpha);
                    inv_beta = __builtin_copysign(sr.y, -alpha);
                    tau = fma_t(aa, sr.y, TR(1));
                    const TR t = rcp_fast<TR>(aa + sr.g);
                    w = fma_t(t, __builtin_copysign(TR(1), alpha) * DR, rj);
                } else {
                    const TR nrm = sqrt_t<TR>(fma_t(alpha, alpha, sigma));
                    beta = alpha >= TR(0) ? -nrm : nrm;
                    inv_beta = rcp_fast<TR>(beta);
                    const TR s = rcp_fast<TR>(alpha - beta);
                    tau = (beta - alpha) * inv_beta;
                    w = fma_t(s, DR, rj);
                }
                TR rn = fma_t(-tau, w, rj);
                if (vi == 0) rn = beta;
                row[vi] = rn;
                // the block update B(:, k) += (1 / beta) B(:, j) w_k takes
                // w_k / beta, formed once per value instead of scaling B(:, j)
                const T wt = (T)(w * inv_beta);
                if constexpr (LB) {
                    wb[vi] = wt;                     // lanes sharing vi store the same value
                    wave_lds_sync();
                }
                if constexpr (!LB) {
#pragma unroll
                    for (int v = 1; v < CNT; ++v) {
                        const T wk = lane_bcast(wt, bfly_lane(v, P));
#pragma unroll
                        for (int r = 0; r < RPL; ++r) x[r][J + v] = fma_t(x[r][J], wk, x[r][J + v]);
                    }
                } else {
                    const T* wr = (const T*)__builtin_assume_aligned(wb, 16);
                    constexpr int E = 16 / (int)sizeof(T);   // values per 16-byte read
#pragma unroll
                    for (int q = 0; q < (CNT + E - 1) / E; ++q) {
                        T wq[E];
                        if constexpr (E == 4) {
                            const float4 f = ((const float4*)wr)[q];
                            wq[0] = f.x; wq[1] = f.y; wq[2] = f.z; wq[3] = f.w;
                        } else {
                            const double2 f = ((const double2*)wr)[q];
                            wq[0] = f.x; wq[1] = f.y;
                        }
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const int v = q * E + e;
                            if (v >= 1 && v < CNT) {
#pragma unroll
                                for (int r = 0; r < RPL; ++r) x[r][J + v] = fma_t(x[r][J], wq[e], x[r][J + v]);
                            }
                        }
                    }
                }
            }
            step<J + 1, W, LB>(x, Rl, xchg, wb);
        }
    }

    // ---- staged load through a buffer resource -----------------------------------
    // The resource covers the slab's rows only, and reads past its end return
    // zero, so the block needs no per-element bounds masks.  `boff` is the
    // block's byte offset within the slab.
    static __device__ __forceinline__ void load_staged_buf(T (&x)[RPL][N], __amdgpu_buffer_rsrc_t rs, int boff,
                                                           TI* St) {
        static_assert(sizeof(T) == sizeof(TI) && sizeof(TI) == 4, "buffer staging is for FP32 input");
        const int L = lane_id();
        const int vo = boff + L * 4;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const int e = (r * N + c) * 64;
                x[r][c] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, e * 4, 2));
            }
        }
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
#pragma unroll
            for (int c = 0; c < N; ++c) {
                const int el = c * 64 + L;
                St[(el / N) * SS + (el % N)] = (TI)x[r][c];
            }
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < N; ++c) x[r][c] = (T)St[L * SS + c];
            wave_lds_sync();
        }
    }

    // ---- load one block of rows [b0, min(b0 + BR, r1)) ---------------------------
    template <int LOAD>
    static __device__ __forceinline__ void load(T (&x)[RPL][N], const StreamArgs& a, int64_t b0,
                                                int64_t r1, TI* St) {
        const int L = lane_id();
        const TI* X = (const TI*)a.X;
        if constexpr (LOAD == LOAD_ROW_STAGED) {
            // The block is contiguous (ld == N).  Read it with coalesced loads in
            // memory order (register (r, c) <- element (r N + c) 64 + L), then
            // turn each 64-row chunk into one row per lane through LDS.
            static_assert(sizeof(T) == sizeof(TI), "staged load keeps the input type");
            const TI* Xb = X + b0 * (int64_t)N + L;
            const int valid = (int)((min(r1, b0 + (int64_t)BR) - b0) * N) - L;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    const int e = (r * N + c) * 64;
                    x[r][c] = e < valid ? (T)__builtin_nontemporal_load(Xb + e) : T(0);
                }
            }
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    const int el = c * 64 + L;            // element within this 64-row chunk
                    St[(el / N) * SS + (el % N)] = (TI)x[r][c];
                }
                wave_lds_sync();
#pragma unroll
                for (int c = 0; c < N; ++c) x[r][c] = (T)St[L * SS + c];
                wave_lds_sync();
            }
        } else if constexpr (LOAD == LOAD_KRON) {
            // X = A (x) A with A p x Q row-major (ld): one FP32 product per
            // element, as an explicit X would hold it
            constexpr int Q = N == 1 ? 1 : N == 4 ? 2 : N == 9 ? 3 : N == 16 ? 4 : 5;
            static_assert(Q * Q == N, "LOAD_KRON widths are squares up to 25");
            const float* A = (const float*)a.X;
            const uint64_t p = (uint64_t)a.kp;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = b0 + r * 64 + L;
                const bool ok = i < r1;
                const uint64_t ii = (uint64_t)min(i, a.m - 1);
                const uint64_t ia = ii / p, ib = ii - ia * p;
                float fa[Q], fb[Q];
#pragma unroll
                for (int c = 0; c < Q; ++c) {
                    fa[c] = A[ia * a.ld + c];
                    fb[c] = A[ib * a.ld + c];
                }
#pragma unroll
                for (int ca = 0; ca < Q; ++ca)
#pragma unroll
                    for (int cb = 0; cb < Q; ++cb) x[r][ca * Q + cb] = ok ? (T)(fa[ca] * fb[cb]) : T(0);
            }
        } else if constexpr (LOAD == LOAD_COL) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = b0 + r * 64 + L;
                const bool ok = i < r1;
                const TI* Xi = X + i;
#pragma unroll
                for (int c = 0; c < N; ++c)
                    x[r][c] = ok ? (T)__builtin_nontemporal_load(Xi + (int64_t)c * a.ld) : T(0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = b0 + r * 64 + L;
                const bool ok = i < r1;
                const TI* Xi = X + i * a.ld;
#pragma unroll
                for (int c = 0; c < N; ++c) x[r][c] = ok ? (T)Xi[c] : T(0);
            }
        }
    }

    static __device__ __forceinline__ void colsum_block(const T (&x)[RPL][N], double& acc) {
        constexpr int V = 1 << PN;
        T p[V];
#pragma unroll
        for (int c = 0; c < V; ++c) {
            if (c < N) {
                T s = abs_t(x[0][c]);
#pragma unroll
                for (int r = 1; r < RPL; ++r) s += abs_t(x[r][c]);
                p[c] = s;
            } else {
                p[c] = T(0);
            }
        }
        acc += (double)butterfly<PN, N>(p);
    }
};

// One wave factors slab `sid` of `a` and stores leaf node `sid`.  `smem` is the
// workgroup's LDS laid out as in Small::lds_bytes for WPG waves, `wv` the
// wave's slot in it.
template <typename T, typename TI, int N, int RPL, int LOAD, int WPG = 4>
__device__ __forceinline__ void small_slab(const StreamArgs& a, int64_t sid, unsigned char* smem, int wv) {
    using S = Small<T, TI, N, RPL>;
    const int L = lane_id();
    double* Rl = (double*)smem + wv * S::RS;
    TI* St = (TI*)(smem + S::stage_off(WPG)) + wv * S::STG;
    T* wb = (T*)(smem + S::bc_off(LOAD == LOAD_ROW_STAGED, WPG)) + wv * S::BCE;

    for (int i = L; i < S::RS; i += 64) Rl[i] = 0.0;
    wave_lds_sync();

    const int64_t r0 = sid * a.slab;
    const int64_t r1 = min(a.m, r0 + a.slab);
    double acc = 0.0;
    constexpr bool kBuf = LOAD == LOAD_ROW_STAGED && sizeof(TI) == 4 && sizeof(T) == 4;
    if constexpr (kBuf) {
        // Buffer resource over this slab: base at row r0, range = the slab's
        // bytes.  Callers keep slabs of this path below 2 GiB (kMaxBufSlabBytes).
        // The slab index is wave-uniform; reading it through readfirstlane
        // lets the compiler keep the resource in scalar registers (otherwise
        // every load is wrapped in a loop over distinct lane values).
        const int64_t r0u = ((int64_t)__builtin_amdgcn_readfirstlane((int)(r0 >> 32)) << 32) |
                            (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)r0);
        const int slab_bytes = __builtin_amdgcn_readfirstlane((int)((r1 - r0) * N * (int64_t)sizeof(TI)));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)((const TI*)a.X + r0u * N), 0, slab_bytes, 0x00020000);
        for (int64_t b0 = r0; b0 < r1; b0 += S::BR) {
            T x[RPL][N];
            S::load_staged_buf(x, rs, (int)((b0 - r0) * N * (int64_t)sizeof(TI)), St);
            S::colsum_block(x, acc);
            S::template step<0>(x, Rl, nullptr, wb);
        }
    } else {
        for (int64_t b0 = r0; b0 < r1; b0 += S::BR) {
            T x[RPL][N];
            S::template load<LOAD>(x, a, b0, r1, St);
            S::colsum_block(x, acc);
            S::template step<0>(x, Rl, nullptr, wb);
        }
    }
    wave_lds_sync();

    // Leaf node of the tree: R in FP64, row-major with zeros below the diagonal.
    double* out = a.tree.nodes + sid * (int64_t)N * N;
    int off = 0;
    for (int j = 0; j < N; ++j) {
        if (L < N) out[j * N + L] = L >= j ? Rl[off + (L - j)] : 0.0;
        off += pow2ceil(N - j);
    }
    int src = 0;                                        // lane holding column L's sum
    for (int s2 = 0; s2 < S::PN; ++s2) src |= ((L >> s2) & 1) << (5 - s2);
    const double v = lane_gather(acc, src);
    if (L < N) a.tree.node_cs[sid * N + L] = v;
}

template <typename T, typename TI, int N, int RPL, int LOAD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) tsqr_small_kernel(StreamArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wv = (int)(threadIdx.x >> 6);
    const int64_t sid = (int64_t)blockIdx.x * 4 + wv;
    if (sid >= a.nstreams) return;                      // whole wave; no block barriers used
    small_slab<T, TI, N, RPL, LOAD>(a, sid, smem, wv);
}

}  // namespace tsnmf

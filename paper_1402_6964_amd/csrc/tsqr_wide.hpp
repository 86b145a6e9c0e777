// Streaming Householder TSQR for 33..256 columns: W waves per slab, each wave
// owning every W-th column (wave w holds columns w, w + W, ...; NW <= 32 per
// wave) of the same 64 * RPL rows of a block.
//
// The algebra is that of the small kernel (structured Householder on
// [R; B], tsqr_small.hpp), spread over waves by columns: at step j the wave
// that owns column j forms sigma = ||B(:, j)||^2 (one all-reduce) and the
// reflector scalars from alpha = R(j, j) in FP64, and publishes them with the
// pivot column B(:, j) through LDS (double-buffered, one block barrier per
// step); every wave then forms the dot products with its own columns with one
// reduce-scatter butterfly, applies the reflector to its own columns and keeps
// its own part of R(j, :) in LDS.  Steps come in rounds of W with the same
// local pivot column (Wide::level): the round index is a compile-time
// constant, so the pivot is read straight from its registers and the finished
// columns left of it drop out of the dot products and updates.
#pragma once
#include "tsqr_small.hpp"

namespace tsnmf {

// Row-major loads through a buffer resource per 64-row chunk (wide kernels
// only; needs 64 ld sizeof(TI) < 2^31).
constexpr int LOAD_ROW_BUF = 3;

struct WideArgs {
    const void* X;
    int64_t m;
    int64_t ld;
    int64_t slab;
    int64_t nstreams;
    int32_t n;
    int32_t pad_;
    TreeArgs tree;
};

// R is kept in FP64 (like the small kernel), compactly: wave w stores, for
// each row j, only its columns k >= j, i.e. local columns c0(j)..NW-1 with
// c0(j) = ceil((j - w) / W) (0 for j <= w), row after row.  Up to 128 columns
// it lives in LDS; above (RG) it does not fit (n = 256 needs 257 KB in FP64)
// and lives in a global slot of the workgroup, each wave touching only its
// own part (so its own program order orders the accesses).
template <typename T, typename TI, int NW, int W, int RPL, bool RG = false> struct Wide {
    static constexpr int P = ilog2(NW);
    static_assert((1 << P) == NW && NW <= 32, "NW must be a power of two <= 32");
    static constexpr int BR = 64 * RPL;
    static constexpr int NMAX = NW * W;
    static constexpr int RW = NMAX * NW - W * NW * (NW - 1) / 2 + NMAX;   // FP64 slots per wave (bound)
    static constexpr size_t pv_elems() { return (size_t)2 * (RPL * 64 + 1); } // two pivot slots (T)
    static constexpr int NS = 8;                      // published reflector scalars per slot (FP64)
    static constexpr size_t lds_core() { return ((size_t)(RG ? 0 : W * RW) + 2 * NS) * 8 + pv_elems() * sizeof(T); }
    // staged row-major loads: two 64-row tiles of NMAX columns at an odd row
    // stride (NMAX + 1 elements of 4 bytes), after the rest
    static constexpr int SP = NMAX + 1;
    static constexpr size_t stage_off() { return (lds_core() + 15) & ~(size_t)15; }
    static constexpr size_t lds_bytes(bool staged = false) { return staged ? stage_off() + 2 * 64 * SP * 4 : lds_core(); }
    static constexpr size_t slot_bytes() { return (size_t)W * RW * 8; }   // global R of one workgroup (RG)

    // The W steps j = Q W + o (o = 0 .. W-1) whose pivot is local column Q of
    // wave o.  Q is a compile-time index, so the pivot is read straight from
    // its registers and only local columns Q .. NW-1 take part: columns left of
    // Q are finished in every wave.  Column Q itself is finished in waves
    // wv < o (it was their pivot earlier in this round); it is still
    // transformed there, harmlessly, and its R entries are not stored.
    template <int Q>
    static __device__ __forceinline__ void level(T (&x)[RPL][NW], int n, int wv, int L, double* Rw, double* apub,
                                                 T* pv, int& off) {
        if constexpr (Q < NW) {
            constexpr int CNT = NW - Q;              // local columns Q .. NW-1
            constexpr int V = pow2ceil(CNT);
            constexpr int PV = ilog2(V);
            if (Q * W >= n) return;
            const int vi = bfly_vidx<PV>(L);         // this lane's value: local column Q + vi
            for (int o = 0; o < W; ++o) {
                const int j = Q * W + o;
                if (j >= n) break;
                const int c0 = Q + (wv < o ? 1 : 0); // first live local column of this wave
                T* slot = pv + (j & 1) * (RPL * 64 + 1);
                double* sc = apub + (j & 1) * NS;    // this step's reflector scalars
                const int c = Q + vi;
                const bool mine = vi < CNT && c >= c0;
                // R(j, :) of this wave, written at step j of the previous block:
                // from global memory (RG) it is read before the step's other
                // work, so its latency overlaps it
                double rj_pre = 0.0;
                if constexpr (RG) rj_pre = mine ? Rw[off + c - c0] : 0.0;
                if (wv == o) {
                    // The owner holds the whole pivot column: it alone forms
                    // sigma and the reflector scalars (FP64) and publishes
                    // them with the column, so the other waves skip both.
#pragma unroll
                    for (int r = 0; r < RPL; ++r) slot[r * 64 + L] = x[r][Q];
                    T sg = x[0][Q] * x[0][Q];
#pragma unroll
                    for (int r = 1; r < RPL; ++r) sg = fma_t(x[r][Q], x[r][Q], sg);
                    const double sigma = (double)wave_sum(sg);
                    // R(j, j): first entry of the owner's row j (lane 0 holds local column Q)
                    const double alpha = RG ? lane_bcast(rj_pre, 0) : Rw[off];
                    const bool lv = sigma != 0.0;
                    double beta, inv_beta, s_, tau_;
                    if constexpr (sizeof(T) == 4) {
                        // FP32 block: a live sigma is a nonzero FP32 value, so
                        // alpha^2 + sigma and |alpha| + nrm are normal FP64
                        // numbers.  With beta = -sign(alpha) nrm: 1 / beta and
                        // tau = 1 + |alpha| / nrm come from the refined
                        // reciprocal square root, and 1 / (alpha - beta) =
                        // sign(alpha) / (|alpha| + nrm) takes one reciprocal
                        // (the results are unused unless live).
                        const SqrtRsq sr = sqrt_rsq_normal(__builtin_fma(alpha, alpha, sigma));
                        const double aa = __builtin_fabs(alpha);
                        beta = lv ? __builtin_copysign(sr.g, -alpha) : alpha;
                        inv_beta = __builtin_copysign(sr.y, -alpha);
                        s_ = __builtin_copysign(rcp_fast<double>(aa + sr.g), alpha);
                        tau_ = __builtin_fma(aa, sr.y, 1.0);
                    } else {
                        const double nrm = __builtin_sqrt(__builtin_fma(alpha, alpha, sigma));
                        beta = lv ? (alpha >= 0.0 ? -nrm : nrm) : alpha;
                        inv_beta = rcp_fast<double>(beta);
                        s_ = rcp_fast<double>(alpha - beta);
                        tau_ = (beta - alpha) * inv_beta;
                    }
                    if (L == 0) {
                        sc[0] = beta;
                        sc[1] = lv ? s_ : 0.0;                               // s = 1 / (alpha - beta)
                        sc[2] = lv ? tau_ : 0.0;                             // tau
                        sc[3] = lv ? inv_beta : 0.0;                         // 1 / beta for the block update
                    }
                }
                __syncthreads();
                T xp[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) xp[r] = slot[r * 64 + L];
                const double beta = sc[0];
                const double s = sc[1];
                const double tau = sc[2];
                const T cb = (T)sc[3];
                T p[V];
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    if (v < CNT) {
                        T d = xp[0] * x[0][Q + v];
#pragma unroll
                        for (int r = 1; r < RPL; ++r) d = fma_t(xp[r], x[r][Q + v], d);
                        p[v] = d;
                    } else {
                        p[v] = T(0);
                    }
                }
                const T D = butterfly<PV, CNT>(p);
                const bool piv = wv == o && vi == 0;
                const double rj = RG ? rj_pre : (mine ? Rw[off + c - c0] : 0.0);
                double w = __builtin_fma(s, (double)D, rj);
                if (piv) w = -beta;
                double rn = __builtin_fma(-tau, w, rj);
                if (piv) rn = beta;
                if (mine) Rw[off + c - c0] = rn;
                const T wt = (T)w;
                T t[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) t[r] = cb * xp[r];
#pragma unroll
                for (int v = 0; v < CNT; ++v) {
                    const T wk = lane_bcast(wt, bfly_lane(v, PV));
#pragma unroll
                    for (int r = 0; r < RPL; ++r) x[r][Q + v] = fma_t(t[r], wk, x[r][Q + v]);
                }
                off += NW - c0;
            }
            level<Q + 1>(x, n, wv, L, Rw, apub, pv, off);
        }
    }
};

// The W waves of the workgroup factor slab `sid` of `a` and store leaf node
// `sid`; with RG their R lives in global slot `rslot` of a.tree.rglob.
template <typename T, typename TI, int NW, int W, int RPL, int LOAD, bool RG = false>
__device__ __forceinline__ void wide_slab(const WideArgs& a, int64_t sid, unsigned char* smem, int64_t rslot = 0) {
    using S = Wide<T, TI, NW, W, RPL, RG>;
    constexpr int P = S::P;
    // The wave index is uniform across the wave; reading it through
    // readfirstlane keeps it, the R base and the owner tests in scalar
    // registers.
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int L = lane_id();
    const int n = a.n;
    double* Rw;                                        // this wave's part of R (compact rows)
    double* apub;                                      // reflector scalars of steps j (two slots by parity)
    if constexpr (RG) {
        Rw = a.tree.rglob + ((size_t)rslot * W + wv) * S::RW;
        apub = (double*)smem;
    } else {
        Rw = (double*)smem + (size_t)wv * S::RW;
        apub = (double*)smem + (size_t)W * S::RW;
    }
    T* pv = (T*)(apub + 2 * S::NS);

    for (int i = L; i < S::RW; i += 64) Rw[i] = 0.0;

    const int64_t r0 = sid * a.slab;
    const int64_t r1 = min(a.m, r0 + a.slab);
    const TI* X = (const TI*)a.X;
    double acc = 0.0;
    __syncthreads();
    for (int64_t b0 = r0; b0 < r1; b0 += S::BR) {
        T x[RPL][NW];
        if constexpr (LOAD == LOAD_ROW_BUF) {
            // Row-major rows through one buffer resource per 64-row chunk
            // (the caller keeps 64 ld sizeof(TI) below 2^31): the column
            // offset of each load is a scalar (this wave's column k), the row
            // offset is the same register for every chunk, and rows past r1
            // read as zero.  No address arithmetic per element, so the loads
            // of a block issue back to back.
            const int vo = L * (int)a.ld * (int)sizeof(TI);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t c0 = b0 + r * 64;
                const int nr = (int)max((int64_t)0, min((int64_t)64, r1 - c0));
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    (void*)(X + c0 * a.ld), 0, nr * (int)a.ld * (int)sizeof(TI), 0x00020000);
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    const int k = wv + W * c;
                    const int so = min(k, n - 1) * (int)sizeof(TI);
                    TI v;
                    if constexpr (sizeof(TI) == 4)
                        v = __builtin_bit_cast(TI, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
                    else
                        v = __builtin_bit_cast(TI, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
                    x[r][c] = k < n ? (T)v : T(0);
                }
            }
        } else if constexpr (LOAD == LOAD_ROW_STAGED) {
            // Row-major rows read coalesced: thread t takes column t % NMAX of
            // rows t / NMAX + (64 / NW) q, q < NW, of every 64-row chunk, so
            // consecutive threads read consecutive addresses, and the loads of
            // the whole block are issued at once (as many registers as the
            // block itself).  Then chunk by chunk through an LDS tile (two
            // buffers, one barrier per chunk) into the cyclic column layout:
            // a lane reads row L of its wave's columns.  With the odd row
            // stride both the tile writes and the column reads hit 64
            // different banks.
            static_assert(sizeof(TI) == 4 && sizeof(T) == 4, "staged wide loads are for FP32 input");
            constexpr int NM = S::NMAX, SP = S::SP, RSTEP = 64 / NW;
            const int tid = (int)threadIdx.x;
            const int col = tid % NM, row0 = tid / NM;
            const bool colok = col < n;
            TI y[RPL][NW];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t c0 = b0 + r * 64 + row0;
                const TI* p = X + min(c0, a.m - 1) * a.ld + col;
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int64_t i = c0 + RSTEP * q;
                    y[r][q] = colok && i < r1 ? __builtin_nontemporal_load(p + (int64_t)(RSTEP * q) * a.ld) : TI(0);
                }
            }
            TI* st = (TI*)(smem + S::stage_off());
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                TI* sb = st + (r & 1) * 64 * SP;
#pragma unroll
                for (int q = 0; q < NW; ++q) sb[(row0 + RSTEP * q) * SP + col] = y[r][q];
                __syncthreads();
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    const int k = wv + W * c;
                    x[r][c] = k < n ? (T)sb[L * SP + k] : T(0);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = b0 + r * 64 + L;
                const bool ok = i < r1;
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    // column-major loads take the wave index in its vector
                    // form: with a scalar column offset the compiler
                    // serialises them (one address pair reused, a full wait
                    // per load)
                    const int k = (LOAD == LOAD_COL ? (int)(threadIdx.x >> 6) : wv) + W * c;
                    const bool okc = ok && k < n;
                    const TI* p = LOAD == LOAD_COL ? X + min(i, a.m - 1) + (int64_t)min(k, n - 1) * a.ld
                                                   : X + min(i, a.m - 1) * a.ld + min(k, n - 1);
                    const TI v = LOAD == LOAD_COL ? __builtin_nontemporal_load(p) : *p;
                    x[r][c] = okc ? (T)v : T(0);
                }
            }
        }
        {   // l1 column sums of the block, own columns
            T p[NW];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                T s = abs_t(x[0][c]);
#pragma unroll
                for (int r = 1; r < RPL; ++r) s += abs_t(x[r][c]);
                p[c] = s;
            }
            acc += (double)butterfly<P>(p);
        }
        // Step 0 of this block reuses the pivot and scalar slots of parity 0,
        // which the previous block's step n - 1 (n odd) may still be reading.
        if (b0 != r0) __syncthreads();
        int off = 0;                                 // start of row j in this wave's storage
        S::template level<0>(x, n, wv, L, Rw, apub, pv, off);
    }
    __syncthreads();
    // leaf node: row-major n x n FP64, zeros below the diagonal
    double* out = a.tree.nodes + sid * (int64_t)n * n;
    int off = 0;
    for (int j = 0; j < n; ++j) {
        const int c0 = j > wv ? (j - wv + W - 1) / W : 0;
        if (L < NW) {
            const int k = wv + W * L;
            if (k < n) out[(int64_t)j * n + k] = L >= c0 ? Rw[off + L - c0] : 0.0;
        }
        off += NW - c0;
    }
    int src = 0;                                     // lane holding local column L's sum
    for (int s2 = 0; s2 < P; ++s2) src |= ((L >> s2) & 1) << (5 - s2);
    const double v = lane_gather(acc, src);
    if (a.tree.node_cs != nullptr && L < NW && wv + W * L < n) a.tree.node_cs[sid * n + wv + W * L] = v;
}

template <typename T, typename TI, int NW, int W, int RPL, int LOAD, bool RG = false>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(2))) tsqr_wide_kernel(WideArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    wide_slab<T, TI, NW, W, RPL, LOAD, RG>(a, blockIdx.x, smem, blockIdx.x);
}

// ---- FP64 G-ary tree for wide factors -------------------------------------------
//
// A group of up to G stacked n x n nodes (row-major, so the group is a (G n) x n
// row-major matrix) is factored by the wide streaming kernel in FP64 into one
// node of the next level (Sec. 3.5: the reduce stage factors the stacked R
// factors).  The workgroup that finishes the last group of the next level's
// group (by ticket) climbs; the one that produces the single top node writes R
// (rows flipped to a nonnegative diagonal) and the column sums.  `go` is a
// workgroup-shared flag.
template <int NW, int W, int RPLD, int G, bool RG = false>
__device__ __forceinline__ void wide_merge_run(const TreeArgs& t, int n, int64_t group0, unsigned char* smem, int* go,
                                               int64_t rslot = 0) {
    const int tid = (int)threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    int64_t group = group0, count = t.leaves, base = 0, tbase = 0;
    while (true) {
        const int64_t first = group * G;
        const int cnt = (int)min((int64_t)G, count - first);
        const int64_t nbase = base + count;
        const int64_t ncount = (count + G - 1) / G;
        WideArgs a{};
        a.X = t.nodes + (base + first) * nn;
        a.m = (int64_t)cnt * n;
        a.ld = n;
        a.slab = a.m;
        a.nstreams = 1;
        a.n = n;
        a.tree = t;
        a.tree.nodes = t.nodes + (nbase + group) * nn;
        a.tree.node_cs = nullptr;
        wide_slab<double, double, NW, W, RPLD, LOAD_ROW_BUF, RG>(a, 0, smem, rslot);
        double* cs_out = t.node_cs + (nbase + group) * n;
        for (int c = tid; c < n; c += W * 64) {
            double s = 0.0;
            for (int q = 0; q < cnt; ++q) s += t.node_cs[(base + first + q) * n + c];
            cs_out[c] = s;
        }
        __syncthreads();
        if (ncount == 1) {
            // top: R column-major with rows flipped to a nonnegative diagonal
            const double* top = t.nodes + (nbase + group) * nn;
            for (int i = tid; i < n * n; i += W * 64) {
                const int r = i % n, c = i / n;
                const double d = top[(int64_t)r * n + r];
                const double v = top[(int64_t)r * n + c];
                t.R[i] = c >= r ? (d < 0.0 ? -v : v) : 0.0;
            }
            if (t.colsum != nullptr)
                for (int c = tid; c < n; c += W * 64) t.colsum[c] = cs_out[c];
            return;
        }
        grid_release();
        __syncthreads();
        const int64_t ngroup = group / G;
        const int gsize = (int)min((int64_t)G, ncount - ngroup * G);
        if (tid == 0) {
            const int old = __hip_atomic_fetch_add(t.tickets + tbase + ngroup, 1, __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            const int last = old == gsize - 1;
            if (last) __hip_atomic_store(t.tickets + tbase + ngroup, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *go = last;
        }
        __syncthreads();
        if (!*go) return;
        grid_acquire();
        tbase += (ncount + G - 1) / G;
        base = nbase;
        count = ncount;
        group = ngroup;
    }
}


template <int NW, int W, int RPLD, int G, bool RG = false>
__global__ void __launch_bounds__(W * 64) tsqr_wide_merge_kernel(TreeArgs t, int n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int go;
    wide_merge_run<NW, W, RPLD, G, RG>(t, n, blockIdx.x, smem, &go, blockIdx.x);
}

}  // namespace tsnmf



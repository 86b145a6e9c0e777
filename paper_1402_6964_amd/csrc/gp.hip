// Gaussian projection Y = G^T X (Sec. 2.3; Sec. 3.2 / Algorithm 1) with G
// generated on the fly and never stored.
//
// G(i, l) is a fixed function of (seed, global row i, column l): Philox4x32
// with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11) on counter
// (i mod 2^32, i >> 32, l / 4, 0) and key (seed mod 2^32, seed >> 32) gives
// four 32-bit words, turned into uniforms u = ((x >> 8) + 1) 2^-24 in (0, 1]
// and into the normals of columns 4q .. 4q + 3 by Box-Muller.  The hardware
// log2 / sqrt / sin / cos (sin and cos take revolutions, so 2 pi u needs no
// multiply) are used; their error is below 1e-6 relative, far under the
// BF16 rounding of the matrix-core path.
//
// Like Algorithm 1's combiner, each workgroup sums the outer products g_i x_i^T
// of its rows (FP32 accumulation); a second kernel adds the workgroup partials
// in FP64 in a fixed order (the reduce step) and writes Y (k x n, column-major).
#include "common.hpp"
#include "wave.hpp"

namespace tsnmf {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t (&o)[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        // three-input XOR in one v_bitop3_b32 (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    o[0] = c0;
    o[1] = c1;
    o[2] = c2;
    o[3] = c3;
}

// Four normals G(i, 4q + s), s = 0..3.
__device__ __forceinline__ void gauss4(int64_t i, uint32_t q, uint32_t k0, uint32_t k1, float (&g)[4]) {
    uint32_t x[4];
    philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), q, 0u, k0, k1, x);
    float u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = __builtin_fmaf((float)(x[t] >> 8), 0x1p-24f, 0x1p-24f);   // exact
    const float ln2 = 0.693147180559945309f;
#pragma unroll
    for (int t = 0; t < 4; t += 2) {
        const float rad = __builtin_amdgcn_sqrtf(-2.0f * ln2 * __builtin_amdgcn_logf(u[t]));
        g[t] = rad * __builtin_amdgcn_cosf(u[t + 1]);
        g[t + 1] = rad * __builtin_amdgcn_sinf(u[t + 1]);
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two floats rounded to BF16 (nearest even) and packed: a in the low half.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{a, b}, bf16x2));
}

struct GpArgs {
    const void* X;
    int64_t m;
    int64_t ld;
    int32_t n;
    int32_t k;
    uint32_t key0, key1;
    int64_t row_offset;
    int64_t rows_per_wg;
    float* part;        // [grid.x][k][n] partial Y (only this workgroup's l-range is written)
    double* part_cs;    // [grid.x][n] partial column sums, or nullptr
};

__device__ __forceinline__ float load_f32(const void* X, int64_t idx, bool bf16) {
    if (bf16) {
        const uint16_t v = ((const uint16_t*)X)[idx];
        return __uint_as_float((uint32_t)v << 16);
    }
    return __builtin_nontemporal_load((const float*)X + idx);
}

// ---- matrix-core path ------------------------------------------------------------
//
// Workgroup = 8 waves; grid.y selects a 512-wide l-range and wave w its
// 64-wide slice (16 groups q of 4 columns).  A K step is 32 rows (the K of one
// 16x16x32 BF16 MFMA).  Lane L generates the Philox block of
// (row i0 + 8 (L / 16) + t, group q = qbase + (L % 16)) for t = 0..7: its four
// normals go to four different M-tiles (tile s holds columns 4q + s), so every
// normal is used once.  Rows of X come in chunks of 64 (two K steps), staged
// in LDS as BF16 column by column, so that the B operand of lane L (8
// consecutive rows of one column) is one 16-byte read; a column takes 72 BF16
// slots (144 bytes), so the 16 lanes of a read phase cover the 64 banks once.
// The next chunk is loaded into registers while the current one is generated
// and multiplied, and the staging is double-buffered, so one barrier per chunk
// orders writes and reads and the loads' latency is hidden behind the
// generator.
constexpr int kMfmaRows = 32;                       // K of one 16x16x32 BF16 MFMA
constexpr int kMfmaChunk = 64;                      // rows per barrier: two K steps
constexpr int kXsStride = 72;                       // BF16 slots per staged column

// COOP = S in {1, 2} (k <= 64 S: S slices of 64 columns l): 8 / S waves
// share each slice.  Wave w works on slice w % S, and its slot u = w / S
// generates rows t = u S .. u S + S - 1 of every lane's 8-row K segment (S
// Philox blocks per lane and K step instead of eight); the normals are
// exchanged through LDS (ash[slice][s][lane][t], double-buffered, one barrier
// per K step) so that every wave holds its slice's whole A operand, and slot u
// multiplies it with column tiles u, u + 8 / S, ... of X.  Without it only the
// first S waves of a small k would generate.  COOP = 0: one slice per wave.
template <bool BF16_IN, int COOP>
__global__ void __launch_bounds__(512) gp_mfma_kernel(GpArgs a) {
    __shared__ __align__(16) __bf16 xs[2][128 * kXsStride];   // [buffer][column][row]
    __shared__ double cs_sh[8][128];
    constexpr int kAsh = COOP * 4 * 64 * 8;           // one buffer: S slices x 4 tiles x 64 lanes x 8 rows
    __shared__ __align__(16) __bf16 ash[COOP ? 2 * kAsh : 8];
    const int tid = threadIdx.x;
    const int wv = tid >> 6, L = tid & 63;
    // grid.z: block of 128 columns (columns cb .. cb + n - 1 of X and Y)
    const int cb = (int)blockIdx.z * 128;
    const int n = min(128, a.n - cb), k = a.k;
    const int64_t ldp = a.n;                         // row length of the partial Y
    const int NT = (n + 15) / 16;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.m, r0 + a.rows_per_wg);
    constexpr int kWps = COOP ? 8 / COOP : 1;         // waves per slice
    const int slice = COOP ? wv % COOP : wv, slot = COOP ? wv / COOP : 0;
    const int lbase = blockIdx.y * 512 + slice * 64;  // first column l of this wave
    const uint32_t q = (uint32_t)((lbase >> 2) + (L & 15));
    const bool want_cs = a.part_cs != nullptr && blockIdx.y == 0;
    constexpr int kTiles = COOP ? COOP : 8;           // column tiles of X per wave
    floatx4 acc[4][kTiles];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < kTiles; ++t) acc[s][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    // Staging.  FP32 input: thread (column tid % 128, row group tid / 128)
    // loads 16 rows of one column.  BF16 input: thread (column pair tid % 64,
    // row group tid / 64) loads 8 rows of two adjacent columns, one dword a
    // row, and regroups them into two columns of row pairs (the staged form).
    constexpr int kGroups = BF16_IN ? 8 : 4;         // row groups of the 64-row chunk
    constexpr int kRows = kMfmaChunk / kGroups;      // rows per thread
    const int rgrp = BF16_IN ? tid >> 6 : tid >> 7;
    const int col_ld = BF16_IN ? 2 * (tid & 63) : tid & 127;   // (first) column of this thread
    const bool stager = col_ld < n;
    // both columns of the pair present, and every pair dword-aligned
    const bool pair_ok = col_ld + 1 < n && (a.ld & 1) == 0 && ((uintptr_t)a.X & 3) == 0;
    double csum = 0.0, csum1 = 0.0;                  // sums of the thread's column(s) over its rows
    float v[BF16_IN ? 1 : kRows];
    uint32_t d[BF16_IN ? kRows : 1];                 // row t: column col_ld low, col_ld + 1 high
    auto load_chunk = [&](int64_t i0) {
        const int64_t ib = i0 + rgrp * kRows;
        int64_t idx = ib * a.ld + cb + col_ld;       // one 64-bit multiply per chunk, one add per row
        if constexpr (BF16_IN) {
            const uint16_t* Xh = (const uint16_t*)a.X;
            if (pair_ok && ib + kRows <= r1) {       // whole row group: no masks
#pragma unroll
                for (int t = 0; t < kRows; ++t) {
                    d[t] = *(const uint32_t*)(Xh + idx);
                    idx += a.ld;
                }
            } else {
#pragma unroll
                for (int t = 0; t < kRows; ++t) {
                    const bool in = ib + t < r1;
                    const uint32_t lo = in && stager ? Xh[idx] : 0u;
                    const uint32_t hi = in && col_ld + 1 < n ? Xh[idx + 1] : 0u;
                    d[t] = lo | (hi << 16);
                    idx += a.ld;
                }
            }
        } else {
            if (stager && ib + kRows <= r1) {
#pragma unroll
                for (int t = 0; t < kRows; ++t) {
                    v[t] = __builtin_nontemporal_load((const float*)a.X + idx);
                    idx += a.ld;
                }
            } else {
#pragma unroll
                for (int t = 0; t < kRows; ++t) {
                    v[t] = stager && ib + t < r1 ? __builtin_nontemporal_load((const float*)a.X + idx) : 0.0f;
                    idx += a.ld;
                }
            }
        }
    };
    // A chunk is two K steps of 32 rows.  Step h multiplies the A operands of
    // its rows (au0 for h = 0, au1 for h = 1) with the staged X, and meanwhile
    // generates the A operands of the next step (au1, then au0 for the next
    // chunk), so the generator's vector instructions and the matrix-core
    // instructions are issued by the same wave side by side.  The step is cut
    // into four regions, one generated row pair and two column tiles each; the
    // B operands of a region are read from LDS one region ahead.
    const bool active = lbase < k;                   // waves past k only stage X
    const int64_t lrow = a.row_offset + 8 * (L >> 4);
    auto gen_pair = [&](int64_t row, u32x4 (&au)[4], int p) {
        float g0[4], g1[4];
        gauss4(row, q, a.key0, a.key1, g0);
        gauss4(row + 1, q, a.key0, a.key1, g1);
#pragma unroll
        for (int s = 0; s < 4; ++s) au[s][p] = pack_bf16(g0[s], g1[s]);
    };
    auto read_b = [&](const __bf16* xsb, int p, bf16x8 (&b)[2]) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *(const bf16x8*)(xsb + ((2 * p + j) * 16 + (L & 15)) * kXsStride + 8 * (L >> 4));
    };
    auto chunk = [&](const __bf16* xsb, int64_t i0, u32x4 (&au0)[4], u32x4 (&au1)[4]) {
        bf16x8 bq[2][2];
        read_b(xsb, 0, bq[0]);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int h = r >> 2, p = r & 3;
            if (r < 7) read_b(xsb + kMfmaRows * ((r + 1) >> 2), (r + 1) & 3, bq[(r + 1) & 1]);
            gen_pair(lrow + i0 + kMfmaRows * (h + 1) + 2 * p, h == 0 ? au1 : au0, p);
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[s][(2 * p + j) % kTiles] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, h == 0 ? au0[s] : au1[s]), bq[r & 1][j], acc[s][(2 * p + j) % kTiles],
                        0, 0, 0);
            // the region's 8 MFMAs spread over its generator instructions
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 16, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    int ab = 0;                                      // exchange buffer of the next K step (COOP)
    auto chunk_coop = [&](const __bf16* xsb, int64_t i0) {
        constexpr int S = COOP ? COOP : 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __bf16* aw = ash + ab * kAsh + slice * (4 * 64 * 8);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                float g[4];
                gauss4(lrow + i0 + kMfmaRows * h + slot * S + j, q, a.key0, a.key1, g);
#pragma unroll
                for (int s = 0; s < 4; ++s) aw[(s * 64 + L) * 8 + slot * S + j] = (__bf16)g[s];
            }
            __syncthreads();
            u32x4 au[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) au[s] = *(const u32x4*)(aw + (s * 64 + L) * 8);
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int nt = slot + kWps * j;
                if (nt < NT) {
                    const bf16x8 b =
                        *(const bf16x8*)(xsb + (nt * 16 + (L & 15)) * kXsStride + kMfmaRows * h + 8 * (L >> 4));
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[s][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, au[s]), b,
                                                                            acc[s][j], 0, 0, 0);
                }
            }
            ab ^= 1;
        }
    };
    u32x4 au0[4], au1[4];
    if (!COOP && active) {
#pragma unroll
        for (int p = 0; p < 4; ++p) gen_pair(lrow + r0 + 2 * p, au0, p);
    }
    load_chunk(r0);
    int buf = 0;
    for (int64_t i0 = r0; i0 < r1; i0 += kMfmaChunk, buf ^= 1) {
        // every thread stages its column(s) (zeros past n), so the column
        // tiles past n multiply zeros
        __bf16* const dst = xs[buf] + col_ld * kXsStride + rgrp * kRows;
        if constexpr (BF16_IN) {
            if (want_cs) {
#pragma unroll
                for (int t = 0; t < kRows; ++t) {
                    csum += (double)__builtin_fabsf(__uint_as_float(d[t] << 16));
                    csum1 += (double)__builtin_fabsf(__uint_as_float(d[t] & 0xffff0000u));
                }
            }
            u32x4 c0, c1;                            // columns col_ld, col_ld + 1: rows 2u, 2u + 1 in word u
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c0[u] = (d[2 * u] & 0xffffu) | (d[2 * u + 1] << 16);
                c1[u] = (d[2 * u] >> 16) | (d[2 * u + 1] & 0xffff0000u);
            }
            *(u32x4*)dst = c0;
            *(u32x4*)(dst + kXsStride) = c1;
        } else {
            if (want_cs) {
#pragma unroll
                for (int t = 0; t < kRows; ++t) csum += (double)__builtin_fabsf(v[t]);
            }
#pragma unroll
            for (int h = 0; h < kRows / 8; ++h) {
                u32x4 pk;
#pragma unroll
                for (int t = 0; t < 4; ++t) pk[t] = pack_bf16(v[8 * h + 2 * t], v[8 * h + 2 * t + 1]);
                *(u32x4*)(dst + 8 * h) = pk;
            }
        }
        if (i0 + kMfmaChunk < r1) load_chunk(i0 + kMfmaChunk);
        __syncthreads();
        if constexpr (COOP) chunk_coop(xs[buf], i0);
        else if (active) chunk(xs[buf], i0, au0, au1);
    }
    // partial Y: tile (s, nt), element (row rho = 4 (L / 16) + e, column L % 16)
    float* P = a.part + (int64_t)blockIdx.x * k * ldp + cb;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < kTiles; ++t) {
            const int nt = COOP ? slot + kWps * t : t;
            const int c = nt * 16 + (L & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = 4 * ((lbase >> 2) + 4 * (L >> 4) + e) + s;
                if (nt < NT && c < n && l < k) P[(int64_t)l * ldp + c] = acc[s][t][e];
            }
        }
    if (a.part_cs != nullptr && blockIdx.y == 0) {
        __syncthreads();
        cs_sh[rgrp][col_ld] = csum;
        if (BF16_IN) cs_sh[rgrp][col_ld + 1] = csum1;
        __syncthreads();
        if (tid < n) {
            double t = 0.0;
#pragma unroll
            for (int g = 0; g < kGroups; ++g) t += cs_sh[g][tid];
            a.part_cs[(int64_t)blockIdx.x * ldp + cb + tid] = t;
        }
    }
}

// ---- vector-ALU path (FP32) ---------------------------------------------------------
//
// Workgroup = 8 waves; grid.y selects a 512-wide l-range.  Wave w owns columns
// 16 w .. 16 w + 15 of Y, lane L the groups q = qbase + L and qbase + 64 + L
// (8 columns l), so a lane accumulates an 8 x 16 tile in FP32.  Rows go 4 at
// a time: the 512 threads generate the 4 x 512 block of G (one Philox call
// each) and stage the 4 x n rows of X in LDS; every lane then reads its 8 G
// values and the wave's 16 X values (one broadcast) per row.
constexpr int kSimdRows = 4;

template <bool UPPER, bool PART>
__global__ void __launch_bounds__(512) gp_simd_kernel(GpArgs a) {
    __shared__ __align__(16) float gs[2][kSimdRows][512];
    __shared__ __align__(16) float xsm[2][kSimdRows][128];
    __shared__ double cs_sh[4][128];
    const int tid = threadIdx.x;
    const int wv = tid >> 6, L = tid & 63;
    const int cb = (int)blockIdx.z * 128;            // block of 128 columns
    const int n = min(128, a.n - cb), k = a.k;
    const int64_t ldp = a.n;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.m, r0 + a.rows_per_wg);
    const int lbase = blockIdx.y * 512;
    float acc[8][16];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[e][c] = 0.0f;
    double csum = 0.0;
    const int gen_row = tid >> 7, gen_q = tid & 127;   // G generation: row and group of this thread
    int buf = 0;
    for (int64_t i0 = r0; i0 < r1; i0 += kSimdRows, buf ^= 1) {
        {
            float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};    // columns past k are not generated
            if (lbase + 4 * gen_q < k)
                gauss4(a.row_offset + i0 + gen_row, (uint32_t)((lbase >> 2) + gen_q), a.key0, a.key1, g);
            *(float4*)&gs[buf][gen_row][4 * gen_q] = make_float4(g[0], g[1], g[2], g[3]);
            if (tid < kSimdRows * 128) {
                const int rr = tid >> 7, c = tid & 127;
                const int64_t i = i0 + rr;
                float v = 0.0f;
                if (c < n && i < r1) v = load_f32(a.X, i * a.ld + cb + c, false);
                csum += (double)__builtin_fabsf(v);
                xsm[buf][rr][c] = v;
            }
        }
        __syncthreads();
        // waves whose columns of X lie past n skip their products (PART: n
        // not a multiple of 128), and so does the upper half of the columns l
        // when k <= 256 (UPPER false)
        if (!PART || 16 * wv < n) {
#pragma unroll
            for (int rr = 0; rr < kSimdRows; ++rr) {
                const float4 ga = *(const float4*)&gs[buf][rr][4 * L];
                float gv[8] = {ga.x, ga.y, ga.z, ga.w, 0.0f, 0.0f, 0.0f, 0.0f};
                if constexpr (UPPER) {
                    const float4 gb = *(const float4*)&gs[buf][rr][256 + 4 * L];
                    gv[4] = gb.x;
                    gv[5] = gb.y;
                    gv[6] = gb.z;
                    gv[7] = gb.w;
                }
                float xv[16];
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4) {
                    const float4 t4 = *(const float4*)&xsm[buf][rr][16 * wv + 4 * c4];
                    xv[4 * c4] = t4.x;
                    xv[4 * c4 + 1] = t4.y;
                    xv[4 * c4 + 2] = t4.z;
                    xv[4 * c4 + 3] = t4.w;
                }
#pragma unroll
                for (int e = 0; e < (UPPER ? 8 : 4); ++e)
#pragma unroll
                    for (int c = 0; c < 16; ++c) acc[e][c] = __builtin_fmaf(gv[e], xv[c], acc[e][c]);
            }
        }
    }
    float* P = a.part + (int64_t)blockIdx.x * k * ldp + cb;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int l = lbase + (e < 4 ? 4 * L + e : 256 + 4 * L + (e - 4));
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int cc = 16 * wv + c;
            if (cc < n && l < k) P[(int64_t)l * ldp + cc] = acc[e][c];
        }
    }
    if (a.part_cs != nullptr && blockIdx.y == 0) {
        if (tid < kSimdRows * 128) cs_sh[tid >> 7][tid & 127] = csum;
        __syncthreads();
        if (tid < n)
            a.part_cs[(int64_t)blockIdx.x * ldp + cb + tid] = cs_sh[0][tid] + cs_sh[1][tid] + cs_sh[2][tid] + cs_sh[3][tid];
    }
}

// Small k (k <= 4 LG, LG = 8, 16 or 32): lane L of wave w owns the column
// group q = L % LG (4 columns l) and columns 16 w .. 16 w + 15 of X, and
// sub-stream s = L / LG of the 64 / LG the wave runs: rows s + (64 / LG) r,
// r = 0..3, of each step of 4 (64 / LG) rows.  Every lane's 4 x 16 tile then
// holds useful sums (the kernel above gives each lane 8 columns l of a
// 512-wide range, most of them past a small k).  The step's G (one Philox
// block per row and group, the first 4 LG x 64 / LG threads) and X rows are
// staged in LDS with padded rows (the sub-streams of a read land in different
// banks); waves whose columns of X all lie past n skip the products.  At the
// end the sub-streams are added across lanes (permlane and DPP stages on the
// lane bits of s, in a fixed order) and the lanes of sub-stream 0 write the
// workgroup's partial.
template <int LG>
__global__ void __launch_bounds__(512) gp_simd_small_kernel(GpArgs a) {
    constexpr int SSW = 64 / LG;                     // sub-streams per wave
    constexpr int RS = kSimdRows * SSW;              // rows per step
    constexpr int GST = 4 * LG + 4;                  // G row stride (floats)
    constexpr int XST = 132;                         // X row stride (floats)
    __shared__ __align__(16) float gs[2][RS * GST];
    __shared__ __align__(16) float xsm[2][RS * XST];
    __shared__ double cs_sh[4][128];
    const int tid = threadIdx.x;
    const int wv = tid >> 6, L = tid & 63;
    const int cb = (int)blockIdx.z * 128;            // block of 128 columns
    const int n = min(128, a.n - cb), k = a.k;
    const int64_t ldp = a.n;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.m, r0 + a.rows_per_wg);
    const int qq = L % LG, sub = L / LG;
    const bool busy = 16 * wv < n;                   // this wave's columns of X exist
    float acc[4][16];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[e][c] = 0.0f;
    double csum = 0.0;
    const int gen_row = tid / LG, gen_q = tid % LG;  // generation: threads tid < RS LG
    const int xc = tid & 127, xr = tid >> 7;         // staging: column, first row
    int buf = 0;
    for (int64_t i0 = r0; i0 < r1; i0 += RS, buf ^= 1) {
        if (tid < RS * LG) {
            float g[4] = {0.0f, 0.0f, 0.0f, 0.0f};    // columns past k are not generated
            if (4 * gen_q < k) gauss4(a.row_offset + i0 + gen_row, (uint32_t)gen_q, a.key0, a.key1, g);
            *(float4*)&gs[buf][gen_row * GST + 4 * gen_q] = make_float4(g[0], g[1], g[2], g[3]);
        }
#pragma unroll
        for (int j = 0; j < RS / 4; ++j) {
            const int rr = xr + 4 * j;
            const int64_t i = i0 + rr;
            float v = 0.0f;
            if (xc < n && i < r1) v = load_f32(a.X, i * a.ld + cb + xc, false);
            csum += (double)__builtin_fabsf(v);
            xsm[buf][rr * XST + xc] = v;
        }
        __syncthreads();
        if (busy) {
#pragma unroll
            for (int r = 0; r < kSimdRows; ++r) {
                const int row = sub + SSW * r;
                const float4 g4 = *(const float4*)&gs[buf][row * GST + 4 * qq];
                const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
                float xv[16];
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4) {
                    const float4 t4 = *(const float4*)&xsm[buf][row * XST + 16 * wv + 4 * c4];
                    xv[4 * c4] = t4.x;
                    xv[4 * c4 + 1] = t4.y;
                    xv[4 * c4 + 2] = t4.z;
                    xv[4 * c4 + 3] = t4.w;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int c = 0; c < 16; ++c) acc[e][c] = __builtin_fmaf(gv[e], xv[c], acc[e][c]);
            }
        }
    }
    if (busy) {
        // add the sub-streams: lane bits log2(LG) .. 5, highest first
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                float v = acc[e][c];
                v = allreduce_stage<5>(v);
                if constexpr (LG <= 16) v = allreduce_stage<4>(v);
                if constexpr (LG <= 8) v = v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xf, 0xf, false));
                acc[e][c] = v;
            }
        if (sub == 0) {
            float* P = a.part + (int64_t)blockIdx.x * k * ldp + cb;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int l = 4 * qq + e;
#pragma unroll
                for (int c = 0; c < 16; ++c) {
                    const int cc = 16 * wv + c;
                    if (cc < n && l < k) P[(int64_t)l * ldp + cc] = acc[e][c];
                }
            }
        }
    }
    if (a.part_cs != nullptr && blockIdx.y == 0) {
        __syncthreads();
        cs_sh[xr][xc] = csum;
        __syncthreads();
        if (tid < n)
            a.part_cs[(int64_t)blockIdx.x * ldp + cb + tid] = cs_sh[0][tid] + cs_sh[1][tid] + cs_sh[2][tid] + cs_sh[3][tid];
    }
}

// ---- the generator alone: G^T 1 ------------------------------------------------------
//
// The projection of a column of ones, with nothing read from memory: the same
// launch shape and generation loop as gp_mfma_kernel (row ranges x 512-wide
// column ranges, 8 waves x 16 column groups, 32-row chunks in which lane L
// draws the Philox blocks of rows 8 (L / 16) .. 8 (L / 16) + 7 of group
// L % 16), so its time is the cost of drawing the normals of that kernel.
// Each lane sums its normals in FP32, the four lanes of a group are added,
// and the workgroup partials are summed in FP64 by gp_reduce_kernel (n = 1).
__global__ void __launch_bounds__(512) gp_colsum_kernel(GpArgs a) {
    const int tid = threadIdx.x;
    const int wv = tid >> 6, L = tid & 63;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_wg;
    const int64_t r1 = min(a.m, r0 + a.rows_per_wg);
    const int lbase = blockIdx.y * 512 + wv * 64;
    const uint32_t q = (uint32_t)((lbase >> 2) + (L & 15));
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t i0 = r0; i0 < r1 && lbase < a.k; i0 += kMfmaRows) {   // waves past k idle
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int64_t i = i0 + 8 * (L >> 4) + t;
            float g[4];
            gauss4(a.row_offset + i, q, a.key0, a.key1, g);
            const bool in = i < r1;
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[s] += in ? g[s] : 0.0f;
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = allreduce_stage<4>(allreduce_stage<5>(acc[s]));
    if (L < 16) {
        float* P = a.part + (int64_t)blockIdx.x * a.k;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int l = 4 * (int)q + s;
            if (l < a.k) P[l] = acc[s];
        }
    }
}

// Sum of the workgroup partials in FP64; Y column-major.  A workgroup of 16
// waves takes 64 consecutive outputs: wave w sums the partials of the w-th
// sixteenth of the workgroups (four interleaved FP64 accumulators, so that
// loads of different partials are in flight together), and the 16 wave sums
// are added in wave order, so the order of the additions is fixed.  Outputs
// past k n are the column sums (from part_cs) when colsum is set.
// With `yacc` set, the FP64 sums are added to yacc (k x n column-major,
// FP64) instead of being written to Y: a pass over row blocks accumulates
// G^T X block by block.
constexpr int kReduceWaves = 16;

__global__ void __launch_bounds__(kReduceWaves * 64) gp_reduce_kernel(const float* __restrict__ part, int64_t nparts,
                                                                     int k, int n, float* __restrict__ Y,
                                                                     const double* __restrict__ part_cs,
                                                                     double* __restrict__ colsum,
                                                                     double* __restrict__ yacc) {
    __shared__ double red[kReduceWaves][64];
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int64_t kn = (int64_t)k * n;
    const int64_t ncs = colsum != nullptr ? n : 0;
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const int64_t p0 = nparts * w / kReduceWaves, p1 = nparts * (w + 1) / kReduceWaves;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (t < kn) {
        int64_t p = p0;
        for (; p + 4 <= p1; p += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += (double)part[(p + u) * kn + t];
        }
        for (; p < p1; ++p) acc[0] += (double)part[p * kn + t];
    } else if (t < kn + ncs) {
        const int64_t c = t - kn;
        int64_t p = p0;
        for (; p + 4 <= p1; p += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += part_cs[(p + u) * n + c];
        }
        for (; p < p1; ++p) acc[0] += part_cs[p * n + c];
    }
    red[w][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (w != 0) return;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kReduceWaves; ++q) s += red[q][lane];
    if (t < kn) {
        const int l = (int)(t / n), c = (int)(t % n);
        if (yacc != nullptr) yacc[(int64_t)c * k + l] += s;
        else Y[(int64_t)c * k + l] = (float)s;
    } else if (t < kn + ncs) {
        colsum[t - kn] = s;
    }
}

unsigned reduce_blocks(int64_t outputs) { return (unsigned)((outputs + 63) / 64); }

constexpr int64_t kGpWorkgroups = 2048;

int64_t gp_rows_per_wg(int64_t m, int rows_multiple) {
    int64_t r = (m + kGpWorkgroups - 1) / kGpWorkgroups;
    return ((r + rows_multiple - 1) / rows_multiple) * rows_multiple;
}

}  // namespace

int gauss_colsum_impl(int64_t m, int k, uint64_t seed, int64_t row_offset, float* out, hipStream_t stream) {
    const int64_t rpw = gp_rows_per_wg(m, kMfmaChunk);
    const int64_t parts = (m + rpw - 1) / rpw;
    void* ws = nullptr;
    if (int st = workspace_get(kTicketBytes + (size_t)parts * k * 4 + 256, stream, &ws)) return st;
    GpArgs a{};
    a.m = m;
    a.n = 1;
    a.k = k;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.row_offset = row_offset;
    a.rows_per_wg = rpw;
    a.part = (float*)((char*)ws + kTicketBytes);
    const bool prof = profiling_on();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof)
        if (int st = profile_event(stream, &e0)) return st;
    hipLaunchKernelGGL(gp_colsum_kernel, dim3((unsigned)parts, (unsigned)((k + 511) / 512)), dim3(512), 0, stream, a);
    TSNMF_LAUNCH_CHECK();
    if (prof) {
        if (int st = profile_event(stream, &e1)) return st;
        profile_record(0, e0, e1);
    }
    hipLaunchKernelGGL(gp_reduce_kernel, dim3(reduce_blocks(k)), dim3(kReduceWaves * 64), 0, stream, a.part, parts, k,
                       1, out, nullptr, nullptr, nullptr);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

size_t gp_workspace_bytes(int64_t m, int n, int k) {
    const int64_t rpw = gp_rows_per_wg(m, kMfmaChunk);
    const int64_t parts = (m + rpw - 1) / rpw;
    return kTicketBytes + (size_t)parts * k * n * 4 + (size_t)parts * n * 8 + 1024;
}

int gauss_proj_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, int k, uint64_t seed,
                    int64_t row_offset, float* Y, double* colsum, hipStream_t stream, double* yacc) {
    const bool bf16 = (flags & TSNMF_DTYPE_MASK) == TSNMF_BF16;
    const bool mfma = bf16 || (flags & TSNMF_GP_MFMA_BF16) != 0;
    // rows per workgroup: a multiple of the matrix-core kernel's 64-row
    // chunk (and so of the vector kernel's 4 rows) for either path
    const int64_t rpw = gp_rows_per_wg(m, kMfmaChunk);
    const int64_t parts = (m + rpw - 1) / rpw;
    void* ws = nullptr;
    if (int st = workspace_get(gp_workspace_bytes(m, n, k), stream, &ws)) return st;
    GpArgs a{};
    a.X = X;
    a.m = m;
    a.ld = ld;
    a.n = n;
    a.k = k;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.row_offset = row_offset;
    a.rows_per_wg = rpw;
    a.part = (float*)((char*)ws + kTicketBytes);
    a.part_cs = colsum != nullptr ? (double*)((char*)ws + kTicketBytes + (size_t)parts * k * n * 4) : nullptr;
    // grid: row ranges x 512-wide l-ranges x 128-wide column blocks
    const dim3 grid((unsigned)parts, (unsigned)((k + 511) / 512), (unsigned)((n + 127) / 128));
    const bool prof = profiling_on();
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    if (prof) {
        if (int st = profile_event(stream, &e0)) return st;
    }
    if (mfma) {
        // up to 128 columns of Y: 1 or 2 slices of 64, shared by the 8 waves
        // (4 shared slices measured slower than 4 waves with a slice each:
        // 3.9 against 3.6 ms at 2e7 x 128, k = 256)
        const int coop = k <= 64 ? 1 : k <= 128 ? 2 : 0;
        if (bf16) {
            if (coop == 1) hipLaunchKernelGGL((gp_mfma_kernel<true, 1>), grid, dim3(512), 0, stream, a);
            else if (coop == 2) hipLaunchKernelGGL((gp_mfma_kernel<true, 2>), grid, dim3(512), 0, stream, a);
            else hipLaunchKernelGGL((gp_mfma_kernel<true, 0>), grid, dim3(512), 0, stream, a);
        } else {
            if (coop == 1) hipLaunchKernelGGL((gp_mfma_kernel<false, 1>), grid, dim3(512), 0, stream, a);
            else if (coop == 2) hipLaunchKernelGGL((gp_mfma_kernel<false, 2>), grid, dim3(512), 0, stream, a);
            else hipLaunchKernelGGL((gp_mfma_kernel<false, 0>), grid, dim3(512), 0, stream, a);
        }
    } else {
        // up to 128 columns of Y: lanes own one column group and split the rows
        if (k <= 32) hipLaunchKernelGGL(gp_simd_small_kernel<8>, grid, dim3(512), 0, stream, a);
        else if (k <= 64) hipLaunchKernelGGL(gp_simd_small_kernel<16>, grid, dim3(512), 0, stream, a);
        else if (k <= 128) hipLaunchKernelGGL(gp_simd_small_kernel<32>, grid, dim3(512), 0, stream, a);
        else if (k <= 256) hipLaunchKernelGGL((gp_simd_kernel<false, true>), grid, dim3(512), 0, stream, a);
        else if (n % 128 != 0) hipLaunchKernelGGL((gp_simd_kernel<true, true>), grid, dim3(512), 0, stream, a);
        else hipLaunchKernelGGL((gp_simd_kernel<true, false>), grid, dim3(512), 0, stream, a);
    }
    TSNMF_LAUNCH_CHECK();
    const bool prof_all = prof && profiling_all();
    if (prof) {
        if (int st = profile_event(stream, &e1)) return st;
        profile_record(0, e0, e1);
        if (prof_all)
            if (int st = profile_event(stream, &e2)) return st;
    }
    const int64_t outs = (int64_t)k * n;
    hipLaunchKernelGGL(gp_reduce_kernel, dim3(reduce_blocks(outs + (colsum != nullptr ? n : 0))),
                       dim3(kReduceWaves * 64), 0, stream, a.part, parts, k, n, Y, a.part_cs, colsum, yacc);
    TSNMF_LAUNCH_CHECK();
    if (prof_all) {
        if (int st = profile_event(stream, &e3)) return st;
        profile_record(1, e2, e3);
    }
    return TSNMF_OK;
}

}  // namespace tsnmf

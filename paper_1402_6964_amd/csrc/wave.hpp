// Wave64 cross-lane building blocks for the Householder kernels (gfx950).
//
// The Householder step for column j needs, for every trailing column k, the
// dot product of column j with column k over all rows of a block.  Rows are
// spread over the 64 lanes, so each lane first forms its partial sums for up
// to 32 columns and the wave then reduces all of them at once with a
// reduce-scatter butterfly: at every stage a lane keeps half of its values and
// adds its partner's copy of that half, so V values cost about 2 V operations
// instead of 6 V for one all-reduce per value.
//
// Stage order (lane bit -> instruction):
//   bit 5: v_permlane32_swap   (swaps lanes 32..63 of the first operand with
//                                lanes 0..31 of the second; after the add, lanes
//                                with bit 5 clear hold the first value)
//   bit 4: v_permlane16_swap   (odd 16-lane rows of the first operand with even
//                                rows of the second; bit 4 clear -> first value)
//   bit 3: DPP row_mirror      (partner L ^ 15)
//   bit 2: DPP row_half_mirror (partner L ^ 7)
//   bit 1: DPP quad_perm 2301  (partner L ^ 2)
//   bit 0: DPP quad_perm 1032  (partner L ^ 1)
// A pair stage on bit b keeps value "a" in lanes with bit b clear and "b" in
// lanes with it set.  Each partner differs from the lane in bit b and only in
// lower bits, so partial sums stay disjoint and the result is the full 64-lane
// sum.  With V = 2^P values the first P stages pair values and the remaining
// 6 - P stages are plain all-reduce steps.  Value v ends up in every lane L
// whose top P bits, read from bit 5 downward, spell v from its least
// significant bit upward:  v = sum_{s<P} bit_{5-s}(L) 2^s.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsnmf {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// ---- 32-bit views ----------------------------------------------------------
__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__double2loint(x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)__double2hiint(x); }
__device__ __forceinline__ double mk64(uint32_t hi, uint32_t lo) { return __hiloint2double((int)hi, (int)lo); }

// ---- pair stages on bits 5 and 4 ---------------------------------------------
__device__ __forceinline__ float swap32_add(float a, float b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double swap32_add(double a, double b) {
    auto rl = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    auto rh = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
}
__device__ __forceinline__ float swap16_add(float a, float b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double swap16_add(double a, double b) {
    auto rl = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    auto rh = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return mk64(rh[0], rl[0]) + mk64(rh[1], rl[1]);
}

// ---- DPP partner reads (bits 3..0) -------------------------------------------
template <int CTRL> __device__ __forceinline__ float dpp_read(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_read(double x) {
    int l = __builtin_amdgcn_update_dpp(0, (int)lo32(x), CTRL, 0xf, 0xf, false);
    int h = __builtin_amdgcn_update_dpp(0, (int)hi32(x), CTRL, 0xf, 0xf, false);
    return mk64((uint32_t)h, (uint32_t)l);
}
constexpr int kDppRowMirror = 0x140;      // L ^ 15 within a 16-lane row
constexpr int kDppRowHalfMirror = 0x141;  // L ^ 7 within an 8-lane half row
constexpr int kDppXor2 = 0x4E;            // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;            // quad_perm [1,0,3,2]

template <int BIT> struct DppCtrl;
template <> struct DppCtrl<3> { static constexpr int v = kDppRowMirror; };
template <> struct DppCtrl<2> { static constexpr int v = kDppRowHalfMirror; };
template <> struct DppCtrl<1> { static constexpr int v = kDppXor2; };
template <> struct DppCtrl<0> { static constexpr int v = kDppXor1; };

template <int BIT, typename T> __device__ __forceinline__ T pair_stage(T a, T b) {
    if constexpr (BIT == 5) {
        return swap32_add(a, b);
    } else if constexpr (BIT == 4) {
        return swap16_add(a, b);
    } else {
        const bool up = (lane_id() >> BIT) & 1;
        T keep = up ? b : a;
        T send = up ? a : b;
        return keep + dpp_read<DppCtrl<BIT>::v>(send);
    }
}

template <int BIT, typename T> __device__ __forceinline__ T allreduce_stage(T x) {
    if constexpr (BIT == 5) {
        return swap32_add(x, x);
    } else if constexpr (BIT == 4) {
        return swap16_add(x, x);
    } else {
        return x + dpp_read<DppCtrl<BIT>::v>(x);
    }
}

// Loops rather than recursion: at run time a recursive constexpr function
// becomes a real call with a stack frame.
__host__ __device__ constexpr __forceinline__ int ilog2(int v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}
__host__ __device__ constexpr __forceinline__ int pow2ceil(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// One stage over the live values p[0 .. 2^(P - S) - 1]: S is the stage index
// (0 = bit 5).  Pairs (p[2i], p[2i+1]) -> p[i] while values remain, then
// all-reduce.  Values at index >= LIVE are known to be zero (padding up to a
// power of two): a pair of two such values stays zero without instructions.
template <int P, int S, int LIVE, typename T> __device__ __forceinline__ void bfly_stage(T* p) {
    constexpr int BIT = 5 - S;
    if constexpr (S < P) {
        constexpr int HALF = 1 << (P - S - 1);
#pragma unroll
        for (int i = 0; i < HALF; ++i) p[i] = 2 * i < LIVE ? pair_stage<BIT>(p[2 * i], p[2 * i + 1]) : T(0);
    } else {
        p[0] = allreduce_stage<BIT>(p[0]);
    }
}

// Reduce-scatter of V = 2^P values (P <= 5) held in p[0..V-1] (clobbered),
// of which the first LIVE may be nonzero.  Returns the register whose lane L
// holds the wave-wide sum of value bfly_vidx<P>(L).
template <int P, int LIVE = (1 << P), typename T> __device__ __forceinline__ T butterfly(T* p) {
    static_assert(P >= 0 && P <= 5, "at most 32 values per butterfly");
    static_assert(LIVE >= 1 && LIVE <= (1 << P), "live values within the butterfly");
    constexpr int L1 = (LIVE + 1) / 2, L2 = (L1 + 1) / 2, L3 = (L2 + 1) / 2, L4 = (L3 + 1) / 2;
    bfly_stage<P, 0, LIVE>(p);
    bfly_stage<P, 1, L1>(p);
    bfly_stage<P, 2, L2>(p);
    bfly_stage<P, 3, L3>(p);
    bfly_stage<P, 4, L4>(p);
    bfly_stage<P, 5, 1>(p);
    return p[0];
}

// Value index held by lane L after butterfly<P>.
template <int P> __device__ __forceinline__ int bfly_vidx(int L) {
    int v = 0;
#pragma unroll
    for (int s = 0; s < P; ++s) v |= ((L >> (5 - s)) & 1) << s;
    return v;
}
// Lowest lane holding value v after butterfly<P> (compile-time usable).
constexpr int bfly_lane(int v, int P) {
    int L = 0;
    for (int s = 0; s < P; ++s) L |= ((v >> s) & 1) << (5 - s);
    return L;
}

// Full wave sum of one value (6 stages), result in every lane.
template <typename T> __device__ __forceinline__ T wave_sum(T x) {
    x = allreduce_stage<5>(x);
    x = allreduce_stage<4>(x);
    x = allreduce_stage<3>(x);
    x = allreduce_stage<2>(x);
    x = allreduce_stage<1>(x);
    x = allreduce_stage<0>(x);
    return x;
}

// Broadcast of lane `src` (wave-uniform, compile-time or not) to all lanes.
__device__ __forceinline__ float lane_bcast(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ __forceinline__ double lane_bcast(double x, int src) {
    uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)lo32(x), src);
    uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)hi32(x), src);
    return mk64(h, l);
}

// Per-lane gather: value of `x` at lane `src` (any per-lane index 0..63).
__device__ __forceinline__ float lane_gather(float x, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(x)));
}
__device__ __forceinline__ double lane_gather(double x, int src) {
    int l = __builtin_amdgcn_ds_bpermute(src << 2, (int)lo32(x));
    int h = __builtin_amdgcn_ds_bpermute(src << 2, (int)hi32(x));
    return mk64((uint32_t)h, (uint32_t)l);
}

}  // namespace tsnmf

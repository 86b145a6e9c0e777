// Host planning of one TSQR call: leaf launch over row slabs, FP64 tree
// levels over the stacked slab factors, and the finalisation of R.
#include <algorithm>

#include "common.hpp"
#include "tsqr_small.hpp"

namespace tsnmf {

hipError_t launch_small_f32_staged(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32_col(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_staged(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_col(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32w_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32w_col(int n, const StreamArgs& a, hipStream_t s);
int rows_per_lane_f32(int n);
int rows_per_lane_f64(int n);

namespace {

constexpr int kTargetStreams = 2048;   // 256 CUs x 8 resident waves

// R (column-major, n x n) from the root partial (row-major): rows with a
// negative diagonal are negated, the strict lower triangle is zero.
__global__ void finalize_kernel(const double* __restrict__ Rp, const double* __restrict__ csp, int n,
                                double* __restrict__ R, double* __restrict__ colsum) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * n) {
        const int i = t % n, k = t / n;                 // R(i, k), column-major index t
        const double sgn = Rp[i * n + i] < 0.0 ? -1.0 : 1.0;
        R[t] = k >= i ? sgn * Rp[i * n + k] : 0.0;
    }
    if (colsum != nullptr && t < n) colsum[t] = csp[t];
}

enum class Path { F32, F64, F32W };

hipError_t launch_leaf(Path p, int load, int n, const StreamArgs& a, hipStream_t s) {
    switch (p) {
        case Path::F32:
            return load == LOAD_ROW_STAGED ? launch_small_f32_staged(n, a, s)
                   : load == LOAD_COL      ? launch_small_f32_col(n, a, s)
                                           : launch_small_f32_row(n, a, s);
        case Path::F64:
            return load == LOAD_ROW_STAGED ? launch_small_f64_staged(n, a, s)
                   : load == LOAD_COL      ? launch_small_f64_col(n, a, s)
                                           : launch_small_f64_row(n, a, s);
        case Path::F32W:
            return load == LOAD_COL ? launch_small_f32w_col(n, a, s) : launch_small_f32w_row(n, a, s);
    }
    return hipErrorInvalidValue;
}

struct Plan {
    Path path;
    int load;
    int64_t block_rows;
    int64_t slab;
    int64_t streams;
    int arity;
};

Plan make_plan(int64_t m, int n, int64_t ld, uint32_t flags, const tsnmf_tsqr_config* cfg) {
    Plan p{};
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const bool col = (flags & TSNMF_COL_MAJOR) != 0;
    if (dt == TSNMF_F64) p.path = Path::F64;
    else p.path = (flags & TSNMF_LEAF_F64) ? Path::F32W : Path::F32;
    if (col) p.load = LOAD_COL;
    else if (ld == n && p.path != Path::F32W) p.load = LOAD_ROW_STAGED;
    else p.load = LOAD_ROW;
    const int rpl = p.path == Path::F32 ? rows_per_lane_f32(n) : rows_per_lane_f64(n);
    p.block_rows = 64LL * rpl;
    if (cfg != nullptr && cfg->leaf_rows > 0) {
        p.slab = cfg->leaf_rows;
    } else {
        const int64_t blocks = (m + p.block_rows - 1) / p.block_rows;
        const int64_t streams = std::max<int64_t>(1, std::min<int64_t>(blocks, kTargetStreams));
        p.slab = ((blocks + streams - 1) / streams) * p.block_rows;
    }
    p.streams = (m + p.slab - 1) / p.slab;
    p.arity = (cfg != nullptr && cfg->tree_arity >= 2) ? cfg->tree_arity : (n <= 8 ? 32 : 16);
    return p;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t plan_bytes(const Plan& p, int n) {
    const int64_t s1 = (p.streams + p.arity - 1) / p.arity;
    const size_t nn = (size_t)n * n;
    return align256(p.streams * nn * 8) + align256(std::max<int64_t>(s1, 1) * nn * 8) +
           align256(p.streams * (size_t)n * 8) + align256(std::max<int64_t>(s1, 1) * (size_t)n * 8);
}

}  // namespace

size_t tsqr_workspace_bytes(int64_t m, int n) {
    // The default plan has the most streams of any plan without a leaf_rows override.
    const Plan p32 = make_plan(m, n, n, TSNMF_F32, nullptr);
    const Plan p64 = make_plan(m, n, n, TSNMF_F64, nullptr);
    return std::max(plan_bytes(p32, n), plan_bytes(p64, n));
}

int tsqr_r_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R,
                double* colsum, const tsnmf_tsqr_config* cfg, hipStream_t stream) {
    const Plan p = make_plan(m, n, ld, flags, cfg);
    void* ws = nullptr;
    const size_t need = plan_bytes(p, n);
    if (int st = workspace_get(need, stream, &ws)) return st;
    const int64_t s1 = std::max<int64_t>(1, (p.streams + p.arity - 1) / p.arity);
    const size_t nn = (size_t)n * n;
    char* base = (char*)ws;
    double* bufR[2];
    double* bufC[2];
    bufR[0] = (double*)base;
    base += align256(p.streams * nn * 8);
    bufR[1] = (double*)base;
    base += align256(s1 * nn * 8);
    bufC[0] = (double*)base;
    base += align256(p.streams * (size_t)n * 8);
    bufC[1] = (double*)base;

    // Leaves: one wave per slab of rows.
    StreamArgs a{};
    a.X = X;
    a.m = m;
    a.ld = ld;
    a.slab = p.slab;
    a.nstreams = p.streams;
    a.load = p.load;
    a.cs_mode = CS_DATA;
    a.out_R = bufR[0];
    a.out_cs = bufC[0];
    TSNMF_HIP(launch_leaf(p.path, p.load, n, a, stream));

    // FP64 tree: groups of `arity` stacked partial factors.
    int64_t P = p.streams;
    int cur = 0;
    while (P > 1) {
        const int64_t next = (P + p.arity - 1) / p.arity;
        StreamArgs t{};
        t.X = bufR[cur];
        t.m = P * n;
        t.ld = n;
        t.slab = (int64_t)p.arity * n;
        t.nstreams = next;
        t.load = LOAD_ROW;
        t.cs_mode = CS_PARTIALS;
        t.in_cs = bufC[cur];
        t.nin = P;
        t.group = p.arity;
        t.out_R = bufR[cur ^ 1];
        t.out_cs = bufC[cur ^ 1];
        TSNMF_HIP(launch_small_f64_row(n, t, stream));
        cur ^= 1;
        P = next;
    }
    const int threads = 256;
    const int blocks = (n * n + threads - 1) / threads;
    hipLaunchKernelGGL(finalize_kernel, dim3(blocks), dim3(threads), 0, stream, bufR[cur], bufC[cur], n, R,
                       colsum);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

}  // namespace tsnmf

// Host planning of one TSQR call: leaf launch over row slabs, FP64 tree
// levels over the stacked slab factors, and the finalisation of R.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "tsqr_wide.hpp"

namespace tsnmf {

hipError_t launch_small_f32_staged(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32_col(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_staged(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f64_col(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32w_row(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_small_f32w_col(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_coop_leaf_f64(int n, const StreamArgs& a, hipStream_t s);
hipError_t launch_wide_f32_row(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32_col(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f64_row(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f64_col(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32w_row(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32w_col(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32_rowbuf(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32_rowstg(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f64_rowbuf(const WideArgs& a, hipStream_t s);
hipError_t launch_wide_f32w_rowbuf(const WideArgs& a, hipStream_t s);
int rows_per_lane_f32(int n, bool staged);
int rows_per_lane_f64(int n, bool staged);
hipError_t launch_xl_f32_row(const WideArgs& a, hipStream_t s);
hipError_t launch_xl_f32_col(const WideArgs& a, hipStream_t s);
hipError_t launch_xl_f64_row(const WideArgs& a, hipStream_t s);
hipError_t launch_xl_f64_col(const WideArgs& a, hipStream_t s);
hipError_t launch_xl_f32w_row(const WideArgs& a, hipStream_t s);
hipError_t launch_xl_f32w_col(const WideArgs& a, hipStream_t s);
size_t xl_rslot_bytes();
hipError_t launch_wy_f32_col(const WideArgs& a, hipStream_t s);
hipError_t launch_wy_f32_row(const WideArgs& a, hipStream_t s);
int wy_block_rows();
hipError_t launch_small_kron(int q, const StreamArgs& a, hipStream_t s);

namespace {

constexpr int kTargetStreams = 2048;   // 256 CUs x 8 resident waves
// Short FP64 slabs (more than one block, at most 8 x 128 rows), when there
// are at most one per CU: eight waves per slab (tsqr_coop_leaf.hpp).
constexpr int64_t kCoopLeafRows = 1024;
constexpr int64_t kCoopLeafMaxSlabs = 256;

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

hipError_t launch_wide(Path p, int load, const WideArgs& a, hipStream_t s) {
    const bool col = load == LOAD_COL, buf = load == LOAD_ROW_BUF, stg = load == LOAD_ROW_STAGED;
    if (a.n > 128) {
        switch (p) {
            case Path::F32: return col ? launch_xl_f32_col(a, s) : launch_xl_f32_row(a, s);
            case Path::F64: return col ? launch_xl_f64_col(a, s) : launch_xl_f64_row(a, s);
            case Path::F32W: return col ? launch_xl_f32w_col(a, s) : launch_xl_f32w_row(a, s);
        }
        return hipErrorInvalidValue;
    }
    switch (p) {
        case Path::F32:
            return col   ? launch_wide_f32_col(a, s)
                   : stg ? launch_wide_f32_rowstg(a, s)
                   : buf ? launch_wide_f32_rowbuf(a, s)
                         : launch_wide_f32_row(a, s);
        case Path::F64:
            return col ? launch_wide_f64_col(a, s) : buf ? launch_wide_f64_rowbuf(a, s) : launch_wide_f64_row(a, s);
        case Path::F32W:
            return col ? launch_wide_f32w_col(a, s) : buf ? launch_wide_f32w_rowbuf(a, s) : launch_wide_f32w_row(a, s);
    }
    return hipErrorInvalidValue;
}

struct Plan {
    Path path;
    bool wide;
    bool wy;         // blocked compact-WY leaf (FP32 blocks, 33..64 columns)
    bool coop_leaf;  // eight waves per short FP64 slab
    int waves;       // waves per slab
    int load;
    int64_t block_rows;
    int64_t slab;
    int64_t streams;
};

Plan make_plan(int64_t m, int n, int64_t ld, uint32_t flags, const tsnmf_tsqr_config* cfg,
               int64_t max_leaves = kMaxLeaves) {
    Plan p{};
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const bool col = (flags & TSNMF_COL_MAJOR) != 0;
    if (dt == TSNMF_F64) p.path = Path::F64;
    else p.path = (flags & TSNMF_LEAF_F64) ? Path::F32W : Path::F32;
    p.wide = n > 32;
    if (col) p.load = LOAD_COL;
    else if (ld == n && p.path != Path::F32W && !p.wide) p.load = LOAD_ROW_STAGED;
    else p.load = LOAD_ROW;
    // wide: 8 waves above 64 columns; up to 64, 8 for FP32 column-major input
    // (8 columns x 16 rows per lane), else 4 (16 columns per wave)
    const bool f32_8x8 = p.path == Path::F32 && n <= 64 && col;
    p.waves = !p.wide ? 1 : (n > 64 || f32_8x8 ? 8 : 4);
    // wide row-major input with FP64 blocks (FP64 input, or FP32 input with
    // FP64 leaves) goes through buffer resources when the row offsets of a
    // 64-row chunk fit their 32 bits (5 rows per lane), otherwise through
    // per-element loads (4); FP32 blocks are staged below
    const int64_t esize = dt == TSNMF_F64 ? 8 : 4;
    const bool f32 = p.path == Path::F32;
    const int rpl_buf = f32 ? 12 : 5;
    if (p.wide && n <= 128 && p.load == LOAD_ROW && 64LL * ld * esize < ((int64_t)1 << 31))
        p.load = LOAD_ROW_BUF;
    // FP32 blocks of row-major input of 48..128 columns: coalesced loads
    // regrouped through LDS (12 rows per lane), whatever the row stride (the
    // kernels above 128 columns stage FP32 row-major input the same way).
    // Below 48 columns neither load wins throughout (2e7 rows: 33 columns
    // 3.47 ms direct against 3.66 staged, 40 columns 4.34 against 4.07, 44
    // columns 4.07 against 4.34, 48 columns 4.85 against 4.60), and the
    // direct loads are kept.
    if (p.wide && n >= 48 && n <= 128 && f32 && !col) p.load = LOAD_ROW_STAGED;
    // above 128 columns: 8 waves x 32 columns, FP32 4 rows per lane, FP64 2
    // FP32 blocks of 33..64 columns: the blocked compact-WY leaf (8 waves,
    // 512-row blocks) when the configuration asks for it; the unblocked leaf
    // is the default (5e7 x 64 column-major: 11.5 ms against 20.9 ms)
    p.wy = f32 && n >= 33 && n <= 64 && cfg != nullptr && cfg->wy_panel == 16;
    if (p.wy) {
        p.waves = 8;
        p.load = col ? LOAD_COL : LOAD_ROW;
    }
    const int rpl = p.wy ? wy_block_rows() / 64
                    : n > 128 ? (f32 ? 4 : 2)
                    : p.wide ? (p.load == LOAD_ROW_BUF || p.load == LOAD_ROW_STAGED ? rpl_buf
                                : f32 ? (f32_8x8 ? 22 : (n <= 64 && !col ? 12 : 11)) : 4)
                             : (p.path == Path::F32 ? rows_per_lane_f32(n, p.load == LOAD_ROW_STAGED)
                                                    : rows_per_lane_f64(n, p.load == LOAD_ROW_STAGED));
    p.block_rows = 64LL * rpl;
    if (cfg != nullptr && cfg->leaf_rows > 0) {
        p.slab = cfg->leaf_rows;
    } else {
        const int64_t blocks = (m + p.block_rows - 1) / p.block_rows;
        const int64_t streams = std::max<int64_t>(1, std::min<int64_t>(blocks, kTargetStreams / p.waves));
        p.slab = ((blocks + streams - 1) / streams) * p.block_rows;
    }
    // the ticket area (or a fixed scratch buffer) bounds the number of leaves
    if (max_leaves > kMaxLeaves) max_leaves = kMaxLeaves;
    if (max_leaves < 1) max_leaves = 1;
    p.slab = std::max<int64_t>(p.slab, (m + max_leaves - 1) / max_leaves);
    p.streams = (m + p.slab - 1) / p.slab;
    // the FP32 staged loads address a slab through a 32-bit byte range
    if (p.load == LOAD_ROW_STAGED && p.path == Path::F32 && p.slab * n * 4 > kMaxBufSlabBytes) p.load = LOAD_ROW;
    // few short FP64 slabs (a 1,000-row leaf): each slab is one block of the
    // eight waves of a workgroup, n dependent steps instead of n per block
    // (100,000 x 20 in 1,000-row leaves: 93 us for the one-wave leaves)
    p.coop_leaf = p.path == Path::F64 && !p.wide && !col && p.slab > p.block_rows && p.slab <= kCoopLeafRows &&
                  p.streams <= kCoopLeafMaxSlabs;
    return p;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Node storage of a tree over `leaves` factors: the levels of a binary tree
// bound those of any group size, plus the top node (which the wide tree
// stores above a single leaf too).
int64_t tree_nodes(int64_t leaves) {
    int64_t total = 0, c = leaves;
    while (c > 1) {
        total += c;
        c = (c + 1) / 2;
    }
    return total + 2;
}

// Tickets | tree nodes | node column sums | (n > 128) one global R slot per leaf.
size_t tree_bytes(int64_t leaves, int n) {
    const int64_t nodes = tree_nodes(leaves);
    return kTicketBytes + align256(nodes * (size_t)n * n * 8) + align256(nodes * (size_t)n * 8) +
           (n > 128 ? align256((size_t)leaves * xl_rslot_bytes()) : 0);
}

size_t plan_bytes(const Plan& p, int n) { return tree_bytes(p.streams, n); }

// Most leaves whose tree (and R slots) fit `bytes` of workspace.
int64_t fixed_leaves(int n, size_t bytes) {
    int64_t lo = 1, hi = kMaxLeaves;                  // tree_bytes grows with the leaves
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (tree_bytes(mid, n) <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


}  // namespace

// Every default plan (any dtype, layout, leaf precision and row stride) has
// at most kTargetStreams leaves, and at most m: size the tree for that many.
size_t tsqr_workspace_bytes(int64_t m, int n) { return tree_bytes(std::min<int64_t>(m, kTargetStreams), n); }

// ---- allocation-free variant: a fixed scratch array per device ----------------
//
// tsnmf_tsqr_r_noalloc keeps its tickets and tree nodes in this array instead
// of the grown workspace, so it never allocates.  In host code `scratch` is
// only a stand-in for the symbol: its device address (one per GPU) comes from
// hipGetSymbolAddress at the first call on each device and is kept in
// g_scratch; only that address is ever handed to kernels.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch;       // device address of `scratch`, per device

__global__ void zero_words_kernel(int* p, int count) {
    for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < count; i += (int)(gridDim.x * blockDim.x))
        p[i] = 0;
}

// The scratch address of the current device; at its first use the ticket
// area is cleared (by a kernel on `stream`: the array is zero when the code
// object loads, and every call leaves its tickets zero again).
int scratch_get(hipStream_t stream, void** out) {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (g_scratch[dev] == nullptr) {
        void* p = nullptr;
        TSNMF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        hipLaunchKernelGGL(zero_words_kernel, dim3(64), dim3(256), 0, stream, (int*)p,
                           (int)(kTicketBytes / sizeof(int)));
        TSNMF_LAUNCH_CHECK();
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return TSNMF_OK;
}

}  // namespace

int tsqr_r_noalloc_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R, double* colsum,
                        hipStream_t stream) {
    void* ws = nullptr;
    if (int st = scratch_get(stream, &ws)) return st;
    return tsqr_r_impl(X, m, n, ld, flags, R, colsum, nullptr, stream, ws, kScratchBytes);
}

int tsqr_r_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R,
                double* colsum, const tsnmf_tsqr_config* cfg, hipStream_t stream, void* fixed_ws,
                size_t fixed_bytes) {
    // With a fixed buffer the slabs are lengthened until the tree fits it.
    const Plan p = make_plan(m, n, ld, flags, cfg, fixed_ws != nullptr ? fixed_leaves(n, fixed_bytes) : kMaxLeaves);
    void* ws = nullptr;
    if (fixed_ws != nullptr) {
        if (plan_bytes(p, n) > fixed_bytes) return TSNMF_ERR_UNSUPPORTED;
        ws = fixed_ws;
    } else if (int st = workspace_get(plan_bytes(p, n), stream, &ws)) {
        return st;
    }
    const int64_t nodes = tree_nodes(p.streams);
    char* base = (char*)ws;
    TreeArgs tree{};
    tree.tickets = (int*)base;
    tree.nodes = (double*)(base + kTicketBytes);
    tree.node_cs = (double*)(base + kTicketBytes + align256(nodes * (size_t)n * n * 8));
    tree.leaves = p.streams;
    tree.R = R;
    tree.colsum = colsum;
    tree.group = cfg != nullptr && cfg->tree_arity > 0 ? cfg->tree_arity : 0;
    tree.rglob = n > 128 ? (double*)(base + kTicketBytes + align256(nodes * (size_t)n * n * 8) +
                                     align256(nodes * (size_t)n * 8))
                         : nullptr;
    StreamArgs a{};
    a.X = X;
    a.m = m;
    a.ld = ld;
    a.slab = p.slab;
    a.nstreams = p.streams;
    a.tree = tree;
    WideArgs aw{};
    aw.X = X;
    aw.m = m;
    aw.ld = ld;
    aw.slab = p.slab;
    aw.nstreams = p.streams;
    aw.n = n;
    aw.tree = tree;
    const bool prof = profiling_on();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof) {
        if (int st = profile_event(stream, &e0)) return st;
    }
    if (p.wy) {
        TSNMF_HIP(p.load == LOAD_COL ? launch_wy_f32_col(aw, stream) : launch_wy_f32_row(aw, stream));
    } else if (p.wide) {
        TSNMF_HIP(launch_wide(p.path, p.load, aw, stream));
    } else if (p.coop_leaf) {
        TSNMF_HIP(launch_coop_leaf_f64(n, a, stream));
    } else {
        TSNMF_HIP(launch_leaf(p.path, p.load, n, a, stream));
    }
    if (prof) {
        hipEvent_t m0 = nullptr, m1 = nullptr;
        if (profile_take_split(&m0, &m1)) {
            profile_record(0, e0, m0);       // leaf kernel
            if (m1 != nullptr) {
                if (int st = profile_event(stream, &e1)) return st;
                profile_record(1, m1, e1);   // reduction tree
            }
        } else {
            if (int st = profile_event(stream, &e1)) return st;
            profile_record(0, e0, e1);
        }
    }
    return TSNMF_OK;
}

// X = A (x) A (p^2 x q^2) formed in the leaf from A (Sec. 5.2), with the plan
// of an explicit contiguous FP32 X of that shape.
int tsqr_r_kron_impl(const float* A, int64_t p, int q, int64_t lda, double* R, double* colsum, hipStream_t stream) {
    const int n = q * q;
    const int64_t m = p * p;
    Plan pl = make_plan(m, n, n, TSNMF_F32, nullptr);
    if (pl.wide || pl.load != LOAD_ROW_STAGED) return TSNMF_ERR_UNSUPPORTED;   // not reached for q <= 5
    void* ws = nullptr;
    if (int st = workspace_get(plan_bytes(pl, n), stream, &ws)) return st;
    const int64_t nodes = tree_nodes(pl.streams);
    char* base = (char*)ws;
    TreeArgs tree{};
    tree.tickets = (int*)base;
    tree.nodes = (double*)(base + kTicketBytes);
    tree.node_cs = (double*)(base + kTicketBytes + align256(nodes * (size_t)n * n * 8));
    tree.leaves = pl.streams;
    tree.R = R;
    tree.colsum = colsum;
    StreamArgs a{};
    a.X = A;
    a.m = m;
    a.ld = lda;
    a.slab = pl.slab;
    a.nstreams = pl.streams;
    a.tree = tree;
    a.kp = p;
    const bool prof = profiling_on();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof)
        if (int st = profile_event(stream, &e0)) return st;
    TSNMF_HIP(launch_small_kron(q, a, stream));
    if (prof) {
        hipEvent_t m0 = nullptr, m1 = nullptr;
        if (profile_take_split(&m0, &m1)) {
            profile_record(0, e0, m0);
            if (m1 != nullptr) {
                if (int st = profile_event(stream, &e1)) return st;
                profile_record(1, m1, e1);
            }
        }
    }
    return TSNMF_OK;
}

}  // namespace tsnmf

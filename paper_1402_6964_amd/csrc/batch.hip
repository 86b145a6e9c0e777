// Batched TSQR of many independent tall-and-skinny matrices of uneven shape.
//
// The paper's MapReduce runs one map task per row split and reduces the
// stacked R factors (Sec. 3.5); here all row slabs of all matrices of a batch
// form one work list, consumed by a persistent kernel whose workgroups pop
// items with an atomic counter.  The shapes live in device arrays (they may
// change between replays of a captured graph), so the work list is built on
// the device: a one-workgroup planner reads them, orders the matrices by
// their Householder work (m n^2, largest first: the longest-processing-time
// rule), sizes row slabs and tree storage to the reserved workspace and
// resets the counters.  Nothing in the two launches depends on the shapes on
// the host side.
//
// Width classes: n = 16 and n = 32 with ld = n use the one-wave streaming
// kernel (one slab per wave, eight slabs per item); every other n <= 64, and
// n <= 128, use the multi-wave kernel (eight waves per slab).  Row blocks are
// FP32, R is kept in FP64.  The reduction tree of each matrix runs inside the
// same kernel: slabs are grouped, and the workgroup that completes the last
// slab of a group (by ticket) factors the group's stacked R factors in FP64
// and climbs, level by level, as long as it is the last of its next group.
// The workgroup that reaches the single node of the top level writes R
// (rows flipped to a nonnegative diagonal) and the column sums.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "tsqr_coop.hpp"
#include "tsqr_small_inst.hpp"
#include "tsqr_wide.hpp"

namespace tsnmf {
namespace {

enum : int { CLS_NONE = -1, CLS_S16 = 0, CLS_S32 = 1, CLS_W64 = 2, CLS_W128 = 3 };

constexpr int kWaves = 8;                                   // waves per workgroup
// The 64- and 128-column classes read each 64-row chunk with coalesced loads
// and regroup it through LDS (68.3 -> 57.3 ms on the 512-matrix workload,
// against per-element loads and buffer loads); any row stride works.
constexpr int64_t kMaxBatchN = 128;      // widest matrix of the batched call
constexpr int kRplS16 = 8;        // one-wave classes: 512- and 320-row blocks
constexpr int kRplS32 = 5;
constexpr int kRplW64 = 22;       // 8 columns per wave
constexpr int kRplW128 = 12;      // 16 columns per wave
constexpr int kRplM64 = 8;        // FP64 merges, 8 columns per wave
constexpr int kRplM128 = 4;       // FP64 merges, 16 columns per wave
using S16 = Small<float, float, 16, kRplS16>;
using S32 = Small<float, float, 32, kRplS32>;
using W64 = Wide<float, float, 8, kWaves, kRplW64>;
using W128 = Wide<float, float, 16, kWaves, kRplW128>;
using M64 = Wide<double, double, 8, kWaves, kRplM64>;
using M128 = Wide<double, double, 16, kWaves, kRplM128>;
using C16 = CoopTree<16, kWaves>;
using C32 = CoopTree<32, kWaves>;
constexpr int kGroupW64 = 8;      // nodes per FP64 merge (n <= 64): <= 512 rows
constexpr int kGroupW128 = 4;     // nodes per FP64 merge (n <= 128): <= 512 rows

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kLds = cmax(cmax(cmax(S16::lds_bytes(true, kWaves), S32::lds_bytes(true, kWaves)),
                                  cmax(W64::lds_bytes(true), W128::lds_bytes(true))),
                             cmax(cmax(M64::lds_bytes(), M128::lds_bytes()),
                                  cmax(sizeof(CoopTreeLds<16, kWaves>), sizeof(CoopTreeLds<32, kWaves>))));

static_assert(kLds <= 160 * 1024, "LDS of the persistent kernel exceeds a CU's 160 KB");

// ---- slab and tree sizes (shared by the host-side sizing and the planner) ----

__host__ __device__ constexpr int class_of(int64_t n, int64_t ld) {
    return (n == 16 && ld == 16) ? CLS_S16 : (n == 32 && ld == 32) ? CLS_S32 : n <= 64 ? CLS_W64 : CLS_W128;
}
// Rows per block of the class's leaf kernel, and the default slab: about 2 %
// of the slab's bytes go to its n x n FP64 node.
__host__ __device__ constexpr int64_t class_block(int c) {
    return c == CLS_S16 ? S16::BR : c == CLS_S32 ? S32::BR : c == CLS_W64 ? W64::BR : W128::BR;
}
// Slabs are whole numbers of blocks (512, 320, 1408 and 768 rows).
__host__ __device__ constexpr int64_t class_slab(int c) {
    return c == CLS_S16 ? 4096 : c == CLS_S32 ? 4160 : c == CLS_W64 ? 7040 : 16128;
}
static_assert(4096 % S16::BR == 0 && 4160 % S32::BR == 0 && 7040 % W64::BR == 0 && 16128 % W128::BR == 0,
              "default slabs are whole blocks");
// Nodes per tree group.  For the one-wave classes a group must hold whole
// items (multiples of kWaves slabs); 24 and 16 are near the fastest pass sizes.
constexpr int kGroupS16 = 24;
constexpr int kGroupS32 = 16;
static_assert(kGroupS16 % kWaves == 0 && kGroupS32 % kWaves == 0, "groups hold whole items");
static_assert(kGroupS16 <= C16::G && kGroupS32 <= C32::G, "groups fit one pass");
__host__ __device__ constexpr int64_t class_group(int c) {
    return c == CLS_S16 ? kGroupS16 : c == CLS_S32 ? kGroupS32 : c == CLS_W64 ? kGroupW64 : kGroupW128;
}
__host__ __device__ constexpr int class_per_item(int c) { return (c == CLS_S16 || c == CLS_S32) ? kWaves : 1; }

struct Sizes {
    int64_t slab, leaves, items, words, tickets;
};

// `shift` doubles every slab (used when the workspace is short).
__host__ __device__ inline Sizes matrix_sizes(int64_t m, int64_t n, int c, int shift) {
    Sizes s{};
    const int64_t br = class_block(c);
    const int64_t mr = (m + br - 1) / br * br;
    int64_t want = shift >= 40 ? mr : class_slab(c) << shift;
    if (c == CLS_S16 || c == CLS_S32) {
        // the one-wave kernel addresses a slab through a 32-bit byte range
        const int64_t cap = kMaxBufSlabBytes / (n * 4) / br * br;
        want = want < cap ? want : cap;
    }
    s.slab = want < mr ? want : mr;
    s.leaves = (m + s.slab - 1) / s.slab;
    s.items = (s.leaves + class_per_item(c) - 1) / class_per_item(c);
    const int64_t g = class_group(c);
    int64_t nodes = 0, cnt = s.leaves;
    while (cnt > 1) {
        nodes += cnt;
        cnt = (cnt + g - 1) / g;
    }
    nodes += 2;                             // the top node (also above a single leaf)
    s.words = nodes * (n * n + n);          // node R's and node column sums, FP64
    s.tickets = 2 * s.leaves + 2;           // slab groups + tree levels
    return s;
}

struct BatchMat {
    const void* X;
    int64_t m, ld, slab, leaves, group;
    int32_t n, cls;
    int* leaf_tickets;        // one per slab group
    TreeArgs tree;            // nodes, column sums, tree tickets, outputs
};

struct BatchHdr {
    int counter;              // next item
    int nitems;
    int shift;                // slab doubling the planner applied
    int pad_;
};

constexpr int kMaxBatch = TSNMF_MAX_BATCH;
constexpr int kPlanThreads = 1024;

// ---- planner ------------------------------------------------------------------

template <typename V> __device__ V block_exclusive_scan(V v, V* tmp, V* total) {
    const int t = (int)threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < kPlanThreads; off <<= 1) {
        const V a = t >= off ? tmp[t - off] : V(0);
        __syncthreads();
        tmp[t] += a;
        __syncthreads();
    }
    const V incl = tmp[t];
    *total = tmp[kPlanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kPlanThreads)
batch_plan_kernel(int B, const void* const* X, const int64_t* m, const int64_t* n, const int64_t* ld,
                  double* const* R, double* const* colsum, BatchHdr* hdr, BatchMat* mats, int64_t* iprefix,
                  int* tickets, int64_t tcap, double* words, int64_t dcap, int cshift) {
    // per-class slab doubling of the configuration (8 bits per class), on top
    // of the doubling the workspace may force
    auto cls_shift = [cshift](int c) { return (cshift >> (8 * c)) & 0xff; };
    __shared__ float cost[kMaxBatch];
    __shared__ int order[kMaxBatch];
    __shared__ int64_t tmp[kPlanThreads];
    const int t = (int)threadIdx.x;

    // 1. validity and cost; invalid matrices get NaN outputs when their R fits
    for (int i = t; i < B; i += kPlanThreads) {
        const int64_t mi = m[i], ni = n[i], li = ld[i];
        const bool ok = X[i] != nullptr && R[i] != nullptr && ni >= 1 && ni <= kMaxBatchN && mi >= 1 && li >= ni;
        cost[i] = ok ? (float)mi * (float)(ni * ni) : -1.0f;
        if (!ok && R[i] != nullptr && ni >= 1 && ni <= kMaxBatchN) {
            const double nan = __builtin_nan("");
            for (int64_t q = 0; q < ni * ni; ++q) R[i][q] = nan;
            double* cs = colsum != nullptr ? colsum[i] : nullptr;
            if (cs != nullptr)
                for (int64_t q = 0; q < ni; ++q) cs[q] = nan;
        }
    }
    __syncthreads();
    // 2. order by cost, largest first, ties by index (rank by counting)
    for (int i = t; i < B; i += kPlanThreads) {
        const float ci = cost[i];
        int r = 0;
        for (int j = 0; j < B; ++j) {
            const float cj = cost[j];
            r += (cj > ci || (cj == ci && j < i)) ? 1 : 0;
        }
        order[r] = i;
    }
    __syncthreads();
    // 3. slab doubling until the trees fit the workspace
    const int chunk = (B + kPlanThreads - 1) / kPlanThreads;
    const int p0 = min(B, t * chunk), p1 = min(B, p0 + chunk);
    int shift = 0;
    bool overflow = false;
    for (;; ++shift) {
        int64_t w = 0, k = 0;
        for (int p = p0; p < p1; ++p) {
            const int i = order[p];
            if (cost[i] < 0.0f) continue;
            const Sizes s = matrix_sizes(m[i], n[i], class_of(n[i], ld[i]), shift + cls_shift(class_of(n[i], ld[i])));
            w += s.words;
            k += s.tickets;
        }
        int64_t wt = 0, kt = 0;
        (void)block_exclusive_scan(w, tmp, &wt);
        (void)block_exclusive_scan(k, tmp, &kt);
        if ((wt <= dcap && kt <= tcap) || shift >= 40) {
            overflow = wt > dcap || kt > tcap;
            break;
        }
    }
    if (overflow) {
        // The trees do not fit even at the longest slabs: every matrix is
        // skipped and gets NaN outputs (the workspace is never overrun).
        for (int i = t; i < B; i += kPlanThreads) {
            const int64_t ni = n[i];
            if (cost[i] >= 0.0f) {
                const double nan = __builtin_nan("");
                for (int64_t q = 0; q < ni * ni; ++q) R[i][q] = nan;
                double* cs = colsum != nullptr ? colsum[i] : nullptr;
                if (cs != nullptr)
                    for (int64_t q = 0; q < ni; ++q) cs[q] = nan;
            }
        }
        __syncthreads();
        for (int i = t; i < B; i += kPlanThreads) cost[i] = -1.0f;
        __syncthreads();
    }
    // 4. offsets (exclusive scans over the ordered matrices) and descriptors
    int64_t it = 0, w = 0, k = 0;
    for (int p = p0; p < p1; ++p) {
        const int i = order[p];
        if (cost[i] < 0.0f) continue;
        const Sizes s = matrix_sizes(m[i], n[i], class_of(n[i], ld[i]), shift + cls_shift(class_of(n[i], ld[i])));
        it += s.items;
        w += s.words;
        k += s.tickets;
    }
    int64_t it_tot = 0, w_tot = 0, k_tot = 0;
    int64_t ito = block_exclusive_scan(it, tmp, &it_tot);
    int64_t wo = block_exclusive_scan(w, tmp, &w_tot);
    int64_t ko = block_exclusive_scan(k, tmp, &k_tot);
    for (int p = p0; p < p1; ++p) {
        const int i = order[p];
        BatchMat d{};
        iprefix[p] = ito;
        if (cost[i] >= 0.0f) {
            const int c = class_of(n[i], ld[i]);
            const Sizes s = matrix_sizes(m[i], n[i], c, shift + cls_shift(c));
            d.X = X[i];
            d.m = m[i];
            d.ld = ld[i];
            d.n = (int32_t)n[i];
            d.cls = c;
            d.slab = s.slab;
            d.leaves = s.leaves;
            d.group = class_group(c);
            d.leaf_tickets = tickets + ko;
            d.tree.tickets = tickets + ko + (s.leaves + d.group - 1) / d.group;
            d.tree.nodes = words + wo;
            const int64_t nodes = s.words / (n[i] * n[i] + n[i]);
            d.tree.node_cs = words + wo + nodes * n[i] * n[i];
            d.tree.leaves = s.leaves;
            d.tree.group = (int32_t)d.group;
            d.tree.R = R[i];
            d.tree.colsum = colsum != nullptr ? colsum[i] : nullptr;
            ito += s.items;
            wo += s.words;
            ko += s.tickets;
        } else {
            d.cls = CLS_NONE;
        }
        mats[p] = d;
    }
    if (t == 0) {
        iprefix[B] = it_tot;
        hdr->counter = 0;
        hdr->nitems = (int)min(it_tot, (int64_t)0x7fffffff);
        hdr->shift = shift;
    }
    // 5. tickets start at zero
    for (int64_t q = t; q < k_tot; q += kPlanThreads) tickets[q] = 0;
}

// ---- persistent kernel ----------------------------------------------------------

__device__ __forceinline__ int find_matrix(const int64_t* prefix, int cnt, int64_t item) {
    int lo = 0, hi = cnt - 1;                // last i with prefix[i] <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kWaves * 64) batch_kernel(BatchHdr* hdr, const BatchMat* __restrict__ mats,
                                                            const int64_t* __restrict__ iprefix, int B) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int item_sh, go_sh;
    const int tid = (int)threadIdx.x;
    const int wv = tid >> 6;
    const int nitems = hdr->nitems;
    while (true) {
        if (tid == 0) item_sh = __hip_atomic_fetch_add(&hdr->counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= nitems) break;
        const int p = find_matrix(iprefix, B, item);
        const BatchMat& M = mats[p];
        const int cls = M.cls;
        const int64_t s0 = (item - iprefix[p]) * (int64_t)class_per_item(cls);
        const int ns = (int)min((int64_t)class_per_item(cls), M.leaves - s0);
        if (cls == CLS_S16 || cls == CLS_S32) {
            if (wv < ns) {
                const StreamArgs a{M.X, M.m, M.ld, M.slab, M.leaves, M.tree, 0};
                if (cls == CLS_S16) small_slab<float, float, 16, kRplS16, LOAD_ROW_STAGED, kWaves>(a, s0 + wv, smem, wv);
                else small_slab<float, float, 32, kRplS32, LOAD_ROW_STAGED, kWaves>(a, s0 + wv, smem, wv);
            }
        } else {
            const WideArgs a{M.X, M.m, M.ld, M.slab, M.leaves, M.n, 0, M.tree};
            if (cls == CLS_W64) wide_slab<float, float, 8, kWaves, kRplW64, LOAD_ROW_STAGED>(a, s0, smem);
            else wide_slab<float, float, 16, kWaves, kRplW128, LOAD_ROW_STAGED>(a, s0, smem);
        }
        // slab group ticket: every wave releases its node stores first
        grid_release();
        __syncthreads();
        const int64_t g = s0 / M.group;
        const int gsize = (int)min(M.group, M.leaves - g * M.group);
        if (tid == 0) {
            const int old = __hip_atomic_fetch_add(M.leaf_tickets + g, ns, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            const int last = old + ns == gsize;
            if (last) __hip_atomic_store(M.leaf_tickets + g, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            go_sh = last;
        }
        __syncthreads();
        if (go_sh) {
            grid_acquire();
            if (cls == CLS_S16) coop_tree_run<16, kWaves>(M.tree, g, *(CoopTreeLds<16, kWaves>*)smem);
            else if (cls == CLS_S32) coop_tree_run<32, kWaves>(M.tree, g, *(CoopTreeLds<32, kWaves>*)smem);
            else if (cls == CLS_W64) wide_merge_run<8, kWaves, kRplM64, kGroupW64>(M.tree, M.n, g, smem, &go_sh);
            else wide_merge_run<16, kWaves, kRplM128, kGroupW128>(M.tree, M.n, g, smem, &go_sh);
        }
        __syncthreads();     // LDS is reused by the next item
    }
}

// ---- host side --------------------------------------------------------------------

// Layout: header | descriptors[bcap] | item prefix[bcap + 1] | tickets[tcap] |
// FP64 words[dcap].  Grows (outside capture) to the largest need seen.
struct BatchWs {
    void* ptr = nullptr;
    int32_t bcap = 0;
    int64_t tcap = 0, dcap = 0;
    int grid = 0;
    // Buffers replaced by a larger one, kept for graphs captured before the
    // growth until tsnmf_workspace_release() (or the end of the process).
    std::vector<void*> retired;
};
std::mutex g_bws_mu;
std::vector<BatchWs> g_bws;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Smallest tree storage that always fits B matrices of width <= kMaxBatchN
// (one node per matrix after enough slab doubling).
void minimum_need(int B, int64_t* words, int64_t* tickets) {
    const int64_t nm = kMaxBatchN;
    *words = (int64_t)B * (nm * nm + nm);
    *tickets = (int64_t)B * 4;
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

bool fits(const BatchWs& w, int B, int64_t words, int64_t tickets) {
    return w.ptr != nullptr && w.bcap >= B && w.tcap >= tickets && w.dcap >= words;
}

int bws_grow(int dev, int B, int64_t words, int64_t tickets) {
    BatchWs& w = g_bws[dev];
    if (fits(w, B, words, tickets)) return TSNMF_OK;
    // each capacity that grows grows by at least half, so the retired
    // buffers stay within a small multiple of the live one
    auto up = [](int64_t have, int64_t need) { return need <= have ? have : std::max(need, have + have / 2); };
    const int32_t bc = (int32_t)std::min<int64_t>(up(w.bcap, B), TSNMF_MAX_BATCH);
    const int64_t tc = up(w.tcap, tickets), dc = up(w.dcap, words);
    const size_t bytes = align256(sizeof(BatchHdr)) + align256(sizeof(BatchMat) * (size_t)bc) +
                         align256(sizeof(int64_t) * ((size_t)bc + 1)) + align256(sizeof(int) * (size_t)tc) +
                         sizeof(double) * (size_t)dc;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hip_fail(e);
        (void)hipGetLastError();
        return TSNMF_ERR_NOMEM;
    }
    // The old buffer may still be used by enqueued work or by a captured
    // graph: retire it instead of freeing it.
    if (w.ptr != nullptr) w.retired.push_back(w.ptr);
    w.ptr = p;
    w.bcap = bc;
    w.tcap = tc;
    w.dcap = dc;
    return TSNMF_OK;
}

int batch_grid(int dev, int* grid) {
    BatchWs& w = g_bws[dev];
    if (w.grid == 0) {
        if (kLds > 65536)
            TSNMF_HIP(hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)kLds));
        int cus = 0, per = 0;
        TSNMF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        TSNMF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel, kWaves * 64, kLds));
        w.grid = cus * std::max(1, per);
    }
    *grid = w.grid;
    return TSNMF_OK;
}

}  // namespace

int batch_release_retired() {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_bws_mu);
    if ((int)g_bws.size() <= dev || g_bws[dev].retired.empty()) return TSNMF_OK;
    TSNMF_HIP(hipDeviceSynchronize());
    for (void* q : g_bws[dev].retired) TSNMF_HIP(hipFree(q));
    g_bws[dev].retired.clear();
    return TSNMF_OK;
}

int batch_reserve(int32_t max_batch, int64_t max_rows) {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    int64_t w0 = 0, k0 = 0;
    minimum_need(max_batch, &w0, &k0);
    // all rows in matrices of width kMaxBatchN at the default slabs bound the
    // tree storage; the narrowest class's slabs bound the tickets
    const Sizes s = matrix_sizes(max_rows, kMaxBatchN, CLS_W128, 0);
    const int64_t words = w0 + s.words + (int64_t)max_batch * (kMaxBatchN * kMaxBatchN + kMaxBatchN);
    const int64_t tickets = k0 + 2 * (max_rows / class_slab(CLS_S16) + 1) + 2 * (int64_t)max_batch;
    std::lock_guard<std::mutex> lk(g_bws_mu);
    if ((int)g_bws.size() <= dev) g_bws.resize(dev + 1);
    return bws_grow(dev, max_batch, words, tickets);
}

int tsqr_batched_impl(int32_t B, const void* const* X, const int64_t* m, const int64_t* n, const int64_t* ld,
                      double* const* R, double* const* colsum, int cshift, hipStream_t stream) {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_bws_mu);
    if ((int)g_bws.size() <= dev) g_bws.resize(dev + 1);
    int64_t words = 0, tickets = 0;
    minimum_need(B, &words, &tickets);
    if (!capturing(stream)) {
        // outside capture the shapes are read back to size the workspace exactly
        std::vector<int64_t> hm(B), hn(B), hl(B);
        TSNMF_HIP(hipMemcpyAsync(hm.data(), m, sizeof(int64_t) * B, hipMemcpyDeviceToHost, stream));
        TSNMF_HIP(hipMemcpyAsync(hn.data(), n, sizeof(int64_t) * B, hipMemcpyDeviceToHost, stream));
        TSNMF_HIP(hipMemcpyAsync(hl.data(), ld, sizeof(int64_t) * B, hipMemcpyDeviceToHost, stream));
        TSNMF_HIP(hipStreamSynchronize(stream));
        int64_t w = 0, k = 0;
        for (int i = 0; i < B; ++i) {
            if (hn[i] < 1 || hn[i] > kMaxBatchN || hm[i] < 1 || hl[i] < hn[i]) continue;
            const Sizes s = matrix_sizes(hm[i], hn[i], class_of(hn[i], hl[i]), 0);
            w += s.words;
            k += s.tickets;
        }
        words = std::max(words, w);
        tickets = std::max(tickets, k);
        if (int st = bws_grow(dev, B, words, tickets)) return st;
    } else if (!fits(g_bws[dev], B, words, tickets)) {
        return TSNMF_ERR_CAPTURE;
    }
    BatchWs& ws = g_bws[dev];
    int grid = 0;
    if (int st = batch_grid(dev, &grid)) return st;

    char* base = (char*)ws.ptr;
    size_t off = 0;
    auto* hdr = (BatchHdr*)(base + off);
    off += align256(sizeof(BatchHdr));
    auto* mats = (BatchMat*)(base + off);
    off += align256(sizeof(BatchMat) * (size_t)ws.bcap);
    auto* iprefix = (int64_t*)(base + off);
    off += align256(sizeof(int64_t) * ((size_t)ws.bcap + 1));
    auto* tk = (int*)(base + off);
    off += align256(sizeof(int) * (size_t)ws.tcap);
    auto* wd = (double*)(base + off);
    const int64_t tcap = ws.tcap, dcap = ws.dcap;

    const bool prof = profiling_on();
    const bool prof_all = prof && profiling_all();
    hipEvent_t p0 = nullptr, p1 = nullptr, e0 = nullptr, e1 = nullptr;
    if (prof_all)
        if (int st = profile_event(stream, &p0)) return st;
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, stream, (int)B, X, m, n, ld, R, colsum,
                       hdr, mats, iprefix, tk, tcap, wd, dcap, cshift);
    TSNMF_LAUNCH_CHECK();
    if (prof_all) {
        if (int st = profile_event(stream, &p1)) return st;
        profile_record(1, p0, p1);           // planner
    }
    if (prof)
        if (int st = profile_event(stream, &e0)) return st;
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kWaves * 64), kLds, stream, hdr, mats, iprefix, (int)B);
    TSNMF_LAUNCH_CHECK();
    if (prof) {
        if (int st = profile_event(stream, &e1)) return st;
        profile_record(0, e0, e1);           // persistent kernel
    }
    return TSNMF_OK;
}

}  // namespace tsnmf

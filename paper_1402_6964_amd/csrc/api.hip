// C entry points of libtsnmf: argument validation, workspace, status codes.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tsnmf {

namespace {
thread_local int g_last_hip = 0;

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    // Buffers replaced by a larger one.  A graph captured before the growth
    // still names them in its kernel arguments, so they are kept until
    // tsnmf_workspace_release() (or the end of the process).
    std::vector<void*> retired;
};
std::mutex g_ws_mu;
std::vector<Workspace> g_ws;

bool is_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int grow(int dev, size_t bytes) {
    Workspace& w = g_ws[dev];
    if (w.bytes >= bytes) return TSNMF_OK;
    // Growth by at least half the current size keeps the retired buffers
    // below twice the live one.
    size_t sz = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (sz < w.bytes + w.bytes / 2) sz = w.bytes + w.bytes / 2;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        (void)hipGetLastError();
        return TSNMF_ERR_NOMEM;
    }
    e = hipMemset(p, 0, kTicketBytes);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return hip_fail(e);
    }
    // The old buffer may still be in use by enqueued work or by a captured
    // graph: retire it instead of freeing it.
    if (w.ptr != nullptr) w.retired.push_back(w.ptr);
    w.ptr = p;
    w.bytes = sz;
    return TSNMF_OK;
}
struct ProfileStage {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
std::mutex g_prof_mu;
int g_prof_mode = 0;           // 0 off, 1 every stage, 2 the main kernel only
ProfileStage g_prof[2];
}  // namespace

bool profiling_on() { return g_prof_mode != 0; }
bool profiling_all() { return g_prof_mode == 1; }

int profile_event(hipStream_t s, hipEvent_t* ev) {
    TSNMF_HIP(hipEventCreate(ev));
    TSNMF_HIP(hipEventRecord(*ev, s));
    return TSNMF_OK;
}

namespace {
thread_local hipEvent_t g_split[2] = {nullptr, nullptr};
}

void profile_split(hipStream_t s) {
    if (g_prof_mode == 0) return;
    for (int q = 0; q < 2; ++q) {
        hipEvent_t& e = g_split[q];
        if (q == 1 && g_prof_mode != 1) break;   // the second stage is not timed
        if (e != nullptr) (void)hipEventDestroy(e);
        e = nullptr;
        if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, s) != hipSuccess) {
            (void)hipGetLastError();
            if (e != nullptr) (void)hipEventDestroy(e);
            e = nullptr;
        }
    }
}

bool profile_take_split(hipEvent_t* end0, hipEvent_t* begin1) {
    const bool ok = g_split[0] != nullptr && (g_split[1] != nullptr || g_prof_mode == 2);
    if (ok) {
        *end0 = g_split[0];
        *begin1 = g_split[1];
    } else {
        for (auto& e : g_split)
            if (e != nullptr) (void)hipEventDestroy(e);
    }
    g_split[0] = g_split[1] = nullptr;
    return ok;
}

int profile_record(int stage, hipEvent_t start, hipEvent_t stop) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[stage].pending.emplace_back(start, stop);
    return TSNMF_OK;
}

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return TSNMF_ERR_HIP;
}

int workspace_get(size_t bytes, hipStream_t stream, void** out) {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    if (g_ws[dev].bytes < bytes) {
        if (is_capturing(stream)) return TSNMF_ERR_CAPTURE;
        if (int st = grow(dev, bytes)) return st;
    }
    *out = g_ws[dev].ptr;
    return TSNMF_OK;
}

int workspace_release_retired() {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev || g_ws[dev].retired.empty()) return TSNMF_OK;
    TSNMF_HIP(hipDeviceSynchronize());
    for (void* q : g_ws[dev].retired) TSNMF_HIP(hipFree(q));
    g_ws[dev].retired.clear();
    return TSNMF_OK;
}

int workspace_reserve(size_t bytes) {
    int dev = 0;
    TSNMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    return grow(dev, bytes);
}

}  // namespace tsnmf

using namespace tsnmf;

extern "C" {

int tsnmf_tsqr_r_ex(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags, double* R,
                    double* colsum, const tsnmf_tsqr_config* cfg, hipStream_t stream) {
    if (X == nullptr) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const bool col = (flags & TSNMF_COL_MAJOR) != 0;
    if (ld < (col ? m : n)) return -4;
    if ((dt != TSNMF_F32 && dt != TSNMF_F64) ||
        (flags & ~(TSNMF_DTYPE_MASK | TSNMF_COL_MAJOR | TSNMF_LEAF_F64)) != 0)
        return -5;
    if (R == nullptr) return -6;
    if (cfg != nullptr) {
        if (cfg->leaf_rows < 0 || (cfg->tree_arity != 0 && (cfg->tree_arity < 2 || cfg->tree_arity > 64)) ||
            cfg->rows_per_lane != 0 || (cfg->wy_panel != 0 && cfg->wy_panel != 1 && cfg->wy_panel != 16) ||
            cfg->reserved != 0)
            return -8;
    }
    if (n > TSNMF_MAX_N) return TSNMF_ERR_UNSUPPORTED;
    return tsqr_r_impl(X, m, (int)n, ld, flags, R, colsum, cfg, stream);
}

int tsnmf_tsqr_r(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags, double* R,
                 double* colsum, hipStream_t stream) {
    tsnmf_tsqr_config tuned{};
    const bool have = n >= 1 && n <= TSNMF_MAX_N && m >= 1 && tune_lookup(flags, m, (int)n, ld, &tuned);
    return tsnmf_tsqr_r_ex(X, m, n, ld, flags, R, colsum, have ? &tuned : nullptr, stream);
}

int tsnmf_tsqr_r_noalloc(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags, double* R,
                         double* colsum, hipStream_t stream) {
    if (X == nullptr) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const bool col = (flags & TSNMF_COL_MAJOR) != 0;
    if (ld < (col ? m : n)) return -4;
    if ((dt != TSNMF_F32 && dt != TSNMF_F64) ||
        (flags & ~(TSNMF_DTYPE_MASK | TSNMF_COL_MAJOR | TSNMF_LEAF_F64)) != 0)
        return -5;
    if (R == nullptr) return -6;
    if (n > TSNMF_MAX_N) return TSNMF_ERR_UNSUPPORTED;
    return tsqr_r_noalloc_impl(X, m, (int)n, ld, flags, R, colsum, stream);
}

int tsnmf_tsqr_r_kron(const float* A, int64_t p, int32_t q, int64_t lda, double* R, double* colsum,
                      hipStream_t stream) {
    if (A == nullptr) return -1;
    if (p < 1 || p > ((int64_t)1 << 31)) return -2;
    if (q < 1 || q > 5) return -3;
    if (lda < q) return -4;
    if (R == nullptr) return -5;
    return tsqr_r_kron_impl(A, p, q, lda, R, colsum, stream);
}

int tsnmf_tsqr_r_batched(int32_t batch, const void* const* X, const int64_t* m, const int64_t* n,
                         const int64_t* ld, uint32_t flags, double* const* R, double* const* colsum,
                         hipStream_t stream) {
    if (batch < 1 || batch > TSNMF_MAX_BATCH) return -1;
    if (X == nullptr) return -2;
    if (m == nullptr) return -3;
    if (n == nullptr) return -4;
    if (ld == nullptr) return -5;
    if (flags != TSNMF_F32) return -6;
    if (R == nullptr) return -7;
    return tsqr_batched_impl(batch, X, m, n, ld, R, colsum, tune_batch_shift(), stream);
}

int tsnmf_tsqr_r_batched_ex(int32_t batch, const void* const* X, const int64_t* m, const int64_t* n,
                            const int64_t* ld, uint32_t flags, double* const* R, double* const* colsum,
                            const tsnmf_batch_config* cfg, hipStream_t stream) {
    if (batch < 1 || batch > TSNMF_MAX_BATCH) return -1;
    if (X == nullptr) return -2;
    if (m == nullptr) return -3;
    if (n == nullptr) return -4;
    if (ld == nullptr) return -5;
    if (flags != TSNMF_F32) return -6;
    if (R == nullptr) return -7;
    int cshift = tune_batch_shift();
    if (cfg != nullptr) {
        cshift = 0;
        for (int c = 0; c < 4; ++c) {
            if (cfg->slab_shift[c] < 0 || cfg->slab_shift[c] > 8 || cfg->reserved[c] != 0) return -8;
            cshift |= cfg->slab_shift[c] << (8 * c);
        }
    }
    return tsqr_batched_impl(batch, X, m, n, ld, R, colsum, cshift, stream);
}

int tsnmf_reserve_batched(int32_t max_batch, int64_t max_rows) {
    if (max_batch < 1 || max_batch > TSNMF_MAX_BATCH) return -1;
    if (max_rows < 0) return -2;
    return batch_reserve(max_batch, max_rows);
}

int tsnmf_gauss_proj(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags, int32_t k, uint64_t seed,
                     int64_t row_offset, float* Y, double* colsum, hipStream_t stream) {
    if (X == nullptr) return -1;
    if (m < 1) return -2;
    if (n < 1) return -3;
    if (ld < n) return -4;
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const uint32_t mode = flags & (TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32);
    if ((dt != TSNMF_F32 && dt != TSNMF_BF16) || (flags & TSNMF_COL_MAJOR) ||
        mode == (TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32) || (dt == TSNMF_BF16 && mode == TSNMF_GP_SIMD_F32) ||
        (flags & ~(TSNMF_DTYPE_MASK | TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32)) != 0)
        return -5;
    if (k < 4 || k > 4096 || (k % 4) != 0) return -6;
    if (row_offset < 0) return -8;
    if (Y == nullptr) return -9;
    if (n > TSNMF_MAX_N) return TSNMF_ERR_UNSUPPORTED;
    return gauss_proj_impl(X, m, (int)n, ld, flags, k, seed, row_offset, Y, colsum, stream);
}

int tsnmf_gauss_colsum(int64_t m, int32_t k, uint64_t seed, int64_t row_offset, float* s, hipStream_t stream) {
    if (m < 1) return -1;
    if (k < 4 || k > 4096 || (k % 4) != 0) return -2;
    if (row_offset < 0) return -4;
    if (s == nullptr) return -5;
    return gauss_colsum_impl(m, k, seed, row_offset, s, stream);
}

static const int kMaxSmall = 256;   // p, n bound of the n x n solvers
static const int kMaxSpaRows = 4096; // p bound of SPA (the rows of a projection)
static const int kMaxPicks = 64;    // r bound of XRAY and NNLS

int tsnmf_select_spa(const double* M, int32_t p, int32_t n, int32_t ldm, const double* colscale, int32_t r,
                     int32_t* K, double* score, int32_t* info, hipStream_t stream) {
    if (M == nullptr) return -1;
    if (p < 1 || p > kMaxSpaRows) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldm < p) return -4;
    if (r < 1 || r > n) return -6;
    if (K == nullptr) return -7;
    if (info == nullptr) return -9;
    return select_spa_impl(M, p, n, ldm, colscale, r, K, score, info, stream);
}

int tsnmf_select_xray(const double* M, int32_t p, int32_t n, int32_t ldm, int32_t r, int32_t* K, int32_t* info,
                      hipStream_t stream) {
    if (M == nullptr) return -1;
    if (p < 1 || p > kMaxSmall) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldm < p) return -4;
    if (r < 1 || r > n || r > kMaxPicks) return -5;
    if (K == nullptr) return -6;
    if (info == nullptr) return -7;
    return select_xray_impl(M, p, n, ldm, r, K, info, stream);
}

int tsnmf_select_gp(const float* Y, int32_t k, int32_t n, int32_t ldy, const double* colscale, int32_t r,
                    int32_t* K, int32_t* counts, int32_t* info, hipStream_t stream) {
    if (Y == nullptr) return -1;
    if (k < 1 || k > (1 << 20)) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldy < k) return -4;
    if (r < 1 || r > n) return -6;
    if (K == nullptr) return -7;
    if (info == nullptr) return -9;
    return select_gp_impl(Y, k, n, ldy, colscale, r, K, counts, info, stream);
}

int tsnmf_nnls(const double* M, int32_t p, int32_t n, int32_t ldm, const int32_t* K, int32_t r, double* H,
               int32_t ldh, double* resid2, int32_t* info, hipStream_t stream) {
    if (M == nullptr) return -1;
    if (p < 1 || p > kMaxSmall) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldm < p) return -4;
    if (K == nullptr) return -5;
    if (r < 1 || r > n || r > kMaxPicks) return -6;
    if (H == nullptr) return -7;
    if (ldh < r) return -8;
    return nnls_impl(M, p, n, ldm, K, r, H, ldh, resid2, info, stream);
}

int tsnmf_residual(const double* M, int32_t p, int32_t n, int32_t ldm, const int32_t* K, int32_t r, const double* H,
                   int32_t ldh, double* relerr, hipStream_t stream) {
    if (M == nullptr) return -1;
    if (p < 1 || p > kMaxSmall) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldm < p) return -4;
    if (K == nullptr) return -5;
    if (r < 1 || r > n) return -6;
    if (H == nullptr) return -7;
    if (ldh < r) return -8;
    if (relerr == nullptr) return -9;
    return residual_impl(M, p, n, ldm, K, r, H, ldh, relerr, stream);
}

int tsnmf_rsvd(const double* R, int32_t n, int32_t ldr, double* S, double* V, int32_t ldv, double* U, int32_t ldu,
               int32_t* info, hipStream_t stream) {
    if (R == nullptr) return -1;
    if (n < 1 || n > kMaxSmall) return -2;
    if (ldr < n) return -3;
    if (S == nullptr) return -4;
    if (V == nullptr) return -5;
    if (ldv < n) return -6;
    if (U != nullptr && ldu < n) return -8;
    return rsvd_impl(R, n, ldr, S, V, ldv, U, ldu, info, stream);
}

int tsnmf_rank_sweep(const double* R, int32_t p, int32_t n, int32_t ldr, const double* colscale, int32_t rmax,
                     int32_t* K, double* H, int32_t ldh, double* resid, int32_t* info, hipStream_t stream) {
    if (R == nullptr) return -1;
    if (p < 1 || p > kMaxSmall) return -2;
    if (n < 1 || n > kMaxSmall) return -3;
    if (ldr < p) return -4;
    if (rmax < 1 || rmax > n || rmax > kMaxPicks) return -6;
    if (K == nullptr) return -7;
    if (H == nullptr) return -8;
    if (ldh < rmax) return -9;
    if (resid == nullptr) return -10;
    if (info == nullptr) return -11;
    return rank_sweep_impl(R, p, n, ldr, colscale, rmax, K, H, ldh, resid, info, stream);
}

int tsnmf_reserve(int64_t max_m, int32_t max_n, int32_t max_k) {
    if (max_m < 0) return -1;
    if (max_n < 0 || max_n > TSNMF_MAX_N) return -2;
    if (max_k < 0 || max_k > 4096) return -3;
    size_t b = 0;
    if (max_m > 0 && max_n > 0) b = tsqr_workspace_bytes(max_m, max_n);
    if (max_m > 0 && max_n > 0 && max_k > 0) {
        const size_t g = gp_workspace_bytes(max_m, max_n, max_k);
        b = b > g ? b : g;
    }
    return workspace_reserve(b);
}

int tsnmf_workspace_release(void) {
    if (int st = workspace_release_retired()) return st;
    return batch_release_retired();
}

int tsnmf_profile_enable(int on) {
    g_prof_mode = on == 2 ? 2 : (on != 0 ? 1 : 0);
    return TSNMF_OK;
}

int tsnmf_profile_query(int stage, double* total_ms, int64_t* calls) {
    if (stage < 0 || stage > 1) return -1;
    if (total_ms == nullptr) return -2;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        ev.swap(g_prof[stage].pending);
    }
    double sum = 0.0;
    int st = TSNMF_OK;
    for (auto& pr : ev) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(pr.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess && st == TSNMF_OK) st = hip_fail(e);
        sum += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    *total_ms = sum;
    if (calls != nullptr) *calls = (int64_t)ev.size();
    return st;
}

const char* tsnmf_status_string(int status) {
    if (status < 0) return "invalid argument";
    switch (status) {
        case TSNMF_OK: return "success";
        case TSNMF_ERR_HIP: return "HIP runtime error";
        case TSNMF_ERR_NOMEM: return "workspace allocation failed";
        case TSNMF_ERR_CAPTURE: return "workspace too small while the stream is capturing";
        case TSNMF_ERR_UNSUPPORTED: return "unsupported shape";
        default: return "unknown status";
    }
}

int tsnmf_last_hip_error(void) { return g_last_hip; }

int tsnmf_version(void) { return 200; }

}  // extern "C"

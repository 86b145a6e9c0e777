// One pass over a tall matrix delivered in consecutive row blocks, possibly
// from host memory and larger than the device (the 286 GB and 2 TB matrices
// of Sec. 4 and Sec. 5.1 are read once from disk).  Each block gets the same
// work as a whole matrix would: its R factor and column sums (tsqr_r_impl)
// and, with k > 0, its share of G^T X with the rows of G that its global row
// indices select (gauss_proj_impl with row_offset = rows before it, FP64
// accumulation), so TSQR and the projection consume the block together
// (Sec. 3.5).  The block's R joins the running R through one more FP64 tree
// node: the QR of the 2n x n stack [running R; block R].
//
// The running state is small (O(n^2 + k n) doubles) and is the whole
// resumable state of the pass.  Host input goes through two device blocks:
// the copy of one (on a copy stream owned by the state) overlaps the work on
// the other (on the caller's stream), ordered by events; pinned input of a
// state without projection is read in place by the leaf kernels instead.
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "common.hpp"

struct tsnmf_onepass_s {
    int n = 0, k = 0;
    uint32_t flags = 0;        // input dtype | layout | leaf precision
    uint32_t gp_flags = 0;     // flags of the projection
    uint64_t seed = 0;
    int64_t rows = 0;          // rows pushed so far
    size_t elem = 0;           // bytes per input element
    int64_t block_rows = 0;    // rows per device block of host input
    double* S = nullptr;       // 2n x n column-major (ld 2n): running R on top, block R below
    double* Rb = nullptr;      // n x n: R of the last block, then the merged R
    double* cs = nullptr;      // running column sums
    double* csb = nullptr;     // column sums of the last block
    double* Y = nullptr;       // k x n column-major FP64 G^T X
    void* dev[2] = {nullptr, nullptr};   // device blocks of host input
    void* pin[2] = {nullptr, nullptr};   // pinned staging of pageable host input
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};   // the block's host-to-device copy is done
    hipEvent_t used[2] = {nullptr, nullptr};     // the work on the block is done
};

namespace tsnmf {

namespace {

constexpr size_t kBlockBytes = (size_t)64 << 20;   // device block of host input
constexpr char kMagic[8] = {'T', 'S', 'N', 'M', 'F', 'O', 'P', '1'};

struct SavedHeader {
    char magic[8];
    int32_t n, k;
    uint32_t flags, gp_flags;
    uint64_t seed;
    int64_t rows;
};

// The block's R below the running R in the stack; the running column sums
// take the block's.
__global__ void place_block_kernel(const double* __restrict__ Rb, const double* __restrict__ csb, double* S, int n,
                                   double* cs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)n * n) {
        const int64_t r = t % n, c = t / n;
        S[c * 2 * n + n + r] = Rb[t];
    }
    if (t < n) cs[t] += csb[t];
}

// The merged R becomes the running R (top of the stack).
__global__ void keep_merged_kernel(const double* __restrict__ Rm, double* S, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)n * n) {
        const int64_t r = t % n, c = t / n;
        S[c * 2 * n + r] = Rm[t];
    }
}

__global__ void result_kernel(const double* __restrict__ S, int n, const double* __restrict__ cs, const double* Yacc,
                              int k, double* R, double* colsum, float* Y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)n * n) {
        const int64_t r = t % n, c = t / n;
        R[t] = S[c * 2 * n + r];
    }
    if (colsum != nullptr && t < n) colsum[t] = cs[t];
    if (Y != nullptr && t < (int64_t)k * n) Y[t] = (float)Yacc[t];
}

unsigned blocks_for(int64_t count) { return (unsigned)std::max<int64_t>(1, (count + 255) / 256); }

// One block in device memory: projection share, block R and column sums, merge.
int process_block(tsnmf_onepass_s* p, const void* X, int64_t rows, int64_t ld, hipStream_t stream) {
    const int n = p->n;
    if (p->k > 0)
        if (int st = gauss_proj_impl(X, rows, n, ld, p->gp_flags, p->k, p->seed, p->rows, nullptr, nullptr, stream,
                                     p->Y))
            return st;
    if (int st = tsqr_r_impl(X, rows, n, ld, p->flags, p->Rb, p->csb, nullptr, stream)) return st;
    hipLaunchKernelGGL(place_block_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, stream, p->Rb, p->csb,
                       p->S, n, p->cs);
    TSNMF_LAUNCH_CHECK();
    if (int st = tsqr_r_impl(p->S, 2 * (int64_t)n, n, 2 * (int64_t)n, TSNMF_F64 | TSNMF_COL_MAJOR, p->Rb, nullptr,
                             nullptr, stream))
        return st;
    hipLaunchKernelGGL(keep_merged_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, stream, p->Rb, p->S, n);
    TSNMF_LAUNCH_CHECK();
    p->rows += rows;
    return TSNMF_OK;
}

bool host_pinned(const void* ptr) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess) {
        (void)hipGetLastError();     // pageable memory may report an error: clear it
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

// Rows [0, rows) of a host matrix with row stride ld (elements) into a
// contiguous buffer, split over a few host threads for large blocks.
void gather_rows(void* dst, const void* src, int64_t rows, int64_t ld, size_t rowbytes, size_t elem) {
    const size_t total = (size_t)rows * rowbytes;
    const int nt = total >= ((size_t)8 << 20) ? 8 : 1;
    auto part = [&](int t) {
        const int64_t r0 = rows * t / nt, r1 = rows * (t + 1) / nt;
        if ((size_t)ld * elem == rowbytes) {
            memcpy((char*)dst + r0 * rowbytes, (const char*)src + r0 * rowbytes, (size_t)(r1 - r0) * rowbytes);
        } else {
            for (int64_t r = r0; r < r1; ++r)
                memcpy((char*)dst + r * rowbytes, (const char*)src + r * ld * elem, rowbytes);
        }
    };
    if (nt == 1) {
        part(0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(part, t);
    part(0);
    for (auto& x : th) x.join();
}

void destroy_state(tsnmf_onepass_s* p) {
    for (int b = 0; b < 2; ++b) {
        if (p->dev[b]) (void)hipFree(p->dev[b]);
        if (p->pin[b]) (void)hipHostFree(p->pin[b]);
        if (p->copied[b]) (void)hipEventDestroy(p->copied[b]);
        if (p->used[b]) (void)hipEventDestroy(p->used[b]);
    }
    if (p->copy) (void)hipStreamDestroy(p->copy);
    for (double* d : {p->S, p->Rb, p->cs, p->csb, p->Y})
        if (d) (void)hipFree(d);
    delete p;
}

int create_impl(int n, uint32_t flags, int k, uint64_t seed, tsnmf_onepass_s** out) {
    auto* p = new tsnmf_onepass_s();
    p->n = n;
    p->k = k;
    p->flags = flags & (TSNMF_DTYPE_MASK | TSNMF_COL_MAJOR | TSNMF_LEAF_F64);
    p->gp_flags = TSNMF_F32 | (flags & (TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32));
    p->seed = seed;
    p->elem = (flags & TSNMF_DTYPE_MASK) == TSNMF_F64 ? 8 : 4;
    p->block_rows = std::max<int64_t>(1, (int64_t)(kBlockBytes / ((size_t)n * p->elem)));
    auto fail = [&](hipError_t e) {
        const int st = e == hipErrorOutOfMemory ? TSNMF_ERR_NOMEM : hip_fail(e);
        destroy_state(p);
        return st;
    };
    hipError_t e;
    const size_t nn = (size_t)n * n * 8;
    if ((e = hipMalloc((void**)&p->S, 2 * nn)) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void**)&p->Rb, nn)) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void**)&p->cs, (size_t)n * 8)) != hipSuccess) return fail(e);
    if ((e = hipMalloc((void**)&p->csb, (size_t)n * 8)) != hipSuccess) return fail(e);
    if (k > 0 && (e = hipMalloc((void**)&p->Y, (size_t)k * n * 8)) != hipSuccess) return fail(e);
    if ((e = hipMemset(p->S, 0, 2 * nn)) != hipSuccess) return fail(e);
    if ((e = hipMemset(p->cs, 0, (size_t)n * 8)) != hipSuccess) return fail(e);
    if (k > 0 && (e = hipMemset(p->Y, 0, (size_t)k * n * 8)) != hipSuccess) return fail(e);
    if ((e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking)) != hipSuccess) return fail(e);
    for (int b = 0; b < 2; ++b) {
        if ((e = hipEventCreateWithFlags(&p->copied[b], hipEventDisableTiming)) != hipSuccess) return fail(e);
        if ((e = hipEventCreateWithFlags(&p->used[b], hipEventDisableTiming)) != hipSuccess) return fail(e);
    }
    *out = p;
    return TSNMF_OK;
}

int push_host_impl(tsnmf_onepass_s* p, const void* X, int64_t rows, int64_t ld, hipStream_t stream) {
    const size_t rowbytes = (size_t)p->n * p->elem;
    const int64_t br = p->block_rows;
    for (int b = 0; b < 2; ++b)
        if (p->dev[b] == nullptr) {
            hipError_t e = hipMalloc(&p->dev[b], (size_t)br * rowbytes);
            if (e != hipSuccess) return e == hipErrorOutOfMemory ? TSNMF_ERR_NOMEM : hip_fail(e);
        }
    const bool pinned = host_pinned(X);
    // Pinned input without a projection: the leaf kernels read the blocks
    // over the host link directly (each element once), no copy at all.
    void* mapped = nullptr;
    if (pinned && p->k == 0) {
        if (hipHostGetDevicePointer(&mapped, const_cast<void*>(X), 0) != hipSuccess) {
            (void)hipGetLastError();
            mapped = nullptr;
        }
    }
    if (mapped != nullptr) {
        for (int64_t r0 = 0; r0 < rows; r0 += br) {
            const int64_t nb = std::min(br, rows - r0);
            if (int st = process_block(p, (const char*)mapped + (size_t)r0 * ld * p->elem, nb, ld, stream)) return st;
        }
        TSNMF_HIP(hipStreamSynchronize(stream));     // the kernels read X: done before X may be reused
        return TSNMF_OK;
    }
    if (!pinned)
        for (int b = 0; b < 2; ++b)
            if (p->pin[b] == nullptr) {
                hipError_t e = hipHostMalloc(&p->pin[b], (size_t)br * rowbytes, hipHostMallocDefault);
                if (e != hipSuccess) return e == hipErrorOutOfMemory ? TSNMF_ERR_NOMEM : hip_fail(e);
            }
    int64_t blk = 0;
    for (int64_t r0 = 0; r0 < rows; r0 += br, ++blk) {
        const int b = (int)(blk & 1);
        const int64_t nb = std::min(br, rows - r0);
        const char* src = (const char*)X + (size_t)r0 * ld * p->elem;
        // device block b is free once the work on its previous contents is done
        TSNMF_HIP(hipStreamWaitEvent(p->copy, p->used[b], 0));
        if (pinned && (size_t)ld * p->elem == rowbytes) {
            TSNMF_HIP(hipMemcpyAsync(p->dev[b], src, (size_t)nb * rowbytes, hipMemcpyHostToDevice, p->copy));
        } else if (pinned) {
            TSNMF_HIP(hipMemcpy2DAsync(p->dev[b], rowbytes, src, (size_t)ld * p->elem, rowbytes, (size_t)nb,
                                       hipMemcpyHostToDevice, p->copy));
        } else {
            TSNMF_HIP(hipEventSynchronize(p->copied[b]));   // staging b has been copied out
            gather_rows(p->pin[b], src, nb, ld, rowbytes, p->elem);
            TSNMF_HIP(hipMemcpyAsync(p->dev[b], p->pin[b], (size_t)nb * rowbytes, hipMemcpyHostToDevice, p->copy));
        }
        TSNMF_HIP(hipEventRecord(p->copied[b], p->copy));
        TSNMF_HIP(hipStreamWaitEvent(stream, p->copied[b], 0));
        if (int st = process_block(p, p->dev[b], nb, p->n, stream)) return st;
        TSNMF_HIP(hipEventRecord(p->used[b], stream));
    }
    // pinned input is read by the copy engine: wait for the last copies so
    // that the caller may reuse X on return
    if (pinned)
        for (int b = 0; b < 2; ++b) TSNMF_HIP(hipEventSynchronize(p->copied[b]));
    return TSNMF_OK;
}

size_t state_bytes(const tsnmf_onepass_s* p) {
    return sizeof(SavedHeader) + ((size_t)p->n * p->n + p->n + (size_t)p->k * p->n) * 8;
}

}  // namespace
}  // namespace tsnmf

using namespace tsnmf;

extern "C" {

int tsnmf_onepass_create(int32_t n, uint32_t flags, int32_t k, uint64_t seed, tsnmf_onepass_t* out) {
    if (n < 1 || n > TSNMF_MAX_N) return -1;
    const uint32_t dt = flags & TSNMF_DTYPE_MASK;
    const uint32_t mode = flags & (TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32);
    if ((dt != TSNMF_F32 && dt != TSNMF_F64) || mode == (TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32) ||
        (flags & ~(TSNMF_DTYPE_MASK | TSNMF_COL_MAJOR | TSNMF_LEAF_F64 | TSNMF_GP_MFMA_BF16 | TSNMF_GP_SIMD_F32)) != 0)
        return -2;
    if (k != 0 && (k < 4 || k > 4096 || (k % 4) != 0 || dt != TSNMF_F32 || (flags & TSNMF_COL_MAJOR))) return -3;
    if (out == nullptr) return -5;
    return create_impl(n, flags, k, seed, out);
}

int tsnmf_onepass_push(tsnmf_onepass_t p, const void* X, int64_t rows, int64_t ld, hipStream_t stream) {
    if (p == nullptr) return -1;
    if (X == nullptr) return -2;
    if (rows < 1) return -3;
    if (ld < ((p->flags & TSNMF_COL_MAJOR) ? rows : p->n)) return -4;
    return process_block(p, X, rows, ld, stream);
}

int tsnmf_onepass_push_host(tsnmf_onepass_t p, const void* X, int64_t rows, int64_t ld, hipStream_t stream) {
    if (p == nullptr) return -1;
    if (X == nullptr) return -2;
    if (rows < 1) return -3;
    if (ld < p->n) return -4;
    if (p->flags & TSNMF_COL_MAJOR) return TSNMF_ERR_UNSUPPORTED;
    return push_host_impl(p, X, rows, ld, stream);
}

int tsnmf_onepass_block_rows(tsnmf_onepass_t p, int64_t* rows) {
    if (p == nullptr) return -1;
    if (rows == nullptr) return -2;
    *rows = p->block_rows;
    return TSNMF_OK;
}

int tsnmf_onepass_rows(tsnmf_onepass_t p, int64_t* rows) {
    if (p == nullptr) return -1;
    if (rows == nullptr) return -2;
    *rows = p->rows;
    return TSNMF_OK;
}

int tsnmf_onepass_result(tsnmf_onepass_t p, double* R, double* colsum, float* Y, hipStream_t stream) {
    if (p == nullptr) return -1;
    if (R == nullptr) return -2;
    const int64_t cnt = std::max<int64_t>((int64_t)p->n * p->n, (int64_t)p->k * p->n);
    hipLaunchKernelGGL(result_kernel, dim3(blocks_for(cnt)), dim3(256), 0, stream, p->S, p->n, p->cs, p->Y, p->k, R,
                       colsum, p->k > 0 ? Y : nullptr);
    TSNMF_LAUNCH_CHECK();
    return TSNMF_OK;
}

int tsnmf_onepass_state_bytes(tsnmf_onepass_t p, size_t* bytes) {
    if (p == nullptr) return -1;
    if (bytes == nullptr) return -2;
    *bytes = state_bytes(p);
    return TSNMF_OK;
}

int tsnmf_onepass_save(tsnmf_onepass_t p, void* host, size_t bytes, hipStream_t stream) {
    if (p == nullptr) return -1;
    if (host == nullptr) return -2;
    if (bytes < state_bytes(p)) return -3;
    TSNMF_HIP(hipStreamSynchronize(stream));
    SavedHeader h{};
    memcpy(h.magic, kMagic, sizeof(kMagic));
    h.n = p->n;
    h.k = p->k;
    h.flags = p->flags;
    h.gp_flags = p->gp_flags;
    h.seed = p->seed;
    h.rows = p->rows;
    memcpy(host, &h, sizeof(h));
    double* d = (double*)((char*)host + sizeof(h));
    const size_t n = (size_t)p->n;
    TSNMF_HIP(hipMemcpy2D(d, n * 8, p->S, 2 * n * 8, n * 8, n, hipMemcpyDeviceToHost));
    TSNMF_HIP(hipMemcpy(d + n * n, p->cs, n * 8, hipMemcpyDeviceToHost));
    if (p->k > 0) TSNMF_HIP(hipMemcpy(d + n * n + n, p->Y, (size_t)p->k * n * 8, hipMemcpyDeviceToHost));
    return TSNMF_OK;
}

int tsnmf_onepass_load(tsnmf_onepass_t p, const void* host, size_t bytes, hipStream_t stream) {
    if (p == nullptr) return -1;
    if (host == nullptr) return -2;
    if (bytes < state_bytes(p)) return -3;
    SavedHeader h;
    memcpy(&h, host, sizeof(h));
    if (memcmp(h.magic, kMagic, sizeof(kMagic)) != 0 || h.n != p->n || h.k != p->k || h.flags != p->flags ||
        h.gp_flags != p->gp_flags || h.seed != p->seed || h.rows < 0)
        return -2;
    TSNMF_HIP(hipStreamSynchronize(stream));
    const double* d = (const double*)((const char*)host + sizeof(h));
    const size_t n = (size_t)p->n;
    TSNMF_HIP(hipMemcpy2D(p->S, 2 * n * 8, d, n * 8, n * 8, n, hipMemcpyHostToDevice));
    TSNMF_HIP(hipMemcpy(p->cs, d + n * n, n * 8, hipMemcpyHostToDevice));
    if (p->k > 0) TSNMF_HIP(hipMemcpy(p->Y, d + n * n + n, (size_t)p->k * n * 8, hipMemcpyHostToDevice));
    p->rows = h.rows;
    return TSNMF_OK;
}

int tsnmf_onepass_destroy(tsnmf_onepass_t p) {
    if (p == nullptr) return -1;
    (void)hipDeviceSynchronize();
    destroy_state(p);
    return TSNMF_OK;
}

}  // extern "C"

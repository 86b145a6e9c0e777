// Host-side shared declarations of libtsnmf (status handling, workspace).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tsnmf.h"

namespace tsnmf {

// Record a HIP failure for tsnmf_last_hip_error() and map it to a status.
int hip_fail(hipError_t e);

#define TSNMF_HIP(call)                                 \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return ::tsnmf::hip_fail(e_); \
    } while (0)

#define TSNMF_LAUNCH_CHECK() TSNMF_HIP(hipGetLastError())

// The first kTicketBytes of every device workspace hold the reduction-tree
// tickets; they are zeroed when the workspace is allocated and every call
// leaves them zero again.
constexpr size_t kTicketBytes = 64 * 1024;
constexpr int64_t kMaxLeaves = (int64_t)(kTicketBytes / sizeof(int));

// Grow-only per-device workspace.  `bytes` is the size needed; returns a
// device pointer aligned to 256 bytes or a status (TSNMF_ERR_CAPTURE when the
// stream is capturing and the workspace is too small, TSNMF_ERR_NOMEM).
int workspace_get(size_t bytes, hipStream_t stream, void** out);
int workspace_reserve(size_t bytes);
// Free the buffers that growth retired (waits for the device first).
int workspace_release_retired();
int batch_release_retired();

// Bytes of workspace one TSQR call of this shape needs (for tsnmf_reserve).
size_t tsqr_workspace_bytes(int64_t m, int n);
size_t gp_workspace_bytes(int64_t m, int n, int k);

// Profiling (see tsnmf_profile_enable): profile_event creates and records an
// event on the stream; profile_record files a (start, stop) pair under a stage.
bool profiling_on();
bool profiling_all();    // also the stages after the main kernel
int profile_record(int stage, hipEvent_t start, hipEvent_t stop);
int profile_event(hipStream_t s, hipEvent_t* ev);
// Called by launch helpers between a leaf kernel and its tree kernel: while
// profiling, records two events there (end of stage 0, start of stage 1) for
// the caller to take with profile_take_split.
void profile_split(hipStream_t s);
bool profile_take_split(hipEvent_t* end0, hipEvent_t* begin1);

// Entry of the loaded autotune table for this call, if any.
bool tune_lookup(uint32_t flags, int64_t m, int n, int64_t ld, tsnmf_tsqr_config* out);
// Per-class slab shifts of the batched call from the loaded table (8 bits per
// class), 0 when the table has no "batch" line.
int tune_batch_shift();

// Implementations behind the C entry points (arguments already validated).
int select_spa_impl(const double* M, int p, int n, int ldm, const double* colscale, int r, int* K, double* score,
                    int* info, hipStream_t stream);
int select_gp_impl(const float* Y, int k, int n, int ldy, const double* colscale, int r, int* K, int* counts,
                   int* info, hipStream_t stream);
int select_xray_impl(const double* M, int p, int n, int ldm, int r, int* K, int* info, hipStream_t stream);
int nnls_impl(const double* M, int p, int n, int ldm, const int* K, int r, double* H, int ldh, double* resid2,
              int* info, hipStream_t stream);
int residual_impl(const double* M, int p, int n, int ldm, const int* K, int r, const double* H, int ldh,
                  double* relerr, hipStream_t stream);
int gauss_proj_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, int k, uint64_t seed,
                    int64_t row_offset, float* Y, double* colsum, hipStream_t stream, double* yacc = nullptr);
int tsqr_r_kron_impl(const float* A, int64_t p, int q, int64_t lda, double* R, double* colsum, hipStream_t stream);
int rsvd_impl(const double* R, int n, int ldr, double* S, double* V, int ldv, double* U, int ldu, int* info,
              hipStream_t stream);
int rank_sweep_impl(const double* R, int p, int n, int ldr, const double* colscale, int rmax, int* K, double* H,
                    int ldh, double* resid, int* info, hipStream_t stream);
int gauss_colsum_impl(int64_t m, int k, uint64_t seed, int64_t row_offset, float* out, hipStream_t stream);
int tsqr_batched_impl(int32_t B, const void* const* X, const int64_t* m, const int64_t* n, const int64_t* ld,
                      double* const* R, double* const* colsum, int cshift, hipStream_t stream);
int batch_reserve(int32_t max_batch, int64_t max_rows);
int tsqr_r_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R,
                double* colsum, const tsnmf_tsqr_config* cfg, hipStream_t stream, void* fixed_ws = nullptr,
                size_t fixed_bytes = 0);
int tsqr_r_noalloc_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R, double* colsum,
                        hipStream_t stream);

}  // namespace tsnmf

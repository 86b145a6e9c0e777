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

// Grow-only per-device workspace.  `bytes` is the size needed; returns a
// device pointer aligned to 256 bytes or a status (TSNMF_ERR_CAPTURE when the
// stream is capturing and the workspace is too small, TSNMF_ERR_NOMEM).
int workspace_get(size_t bytes, hipStream_t stream, void** out);
int workspace_reserve(size_t bytes);

// Bytes of workspace one TSQR call of this shape needs (for tsnmf_reserve).
size_t tsqr_workspace_bytes(int64_t m, int n);
size_t gp_workspace_bytes(int64_t m, int n, int k);

// Implementations behind the C entry points (arguments already validated).
int tsqr_r_impl(const void* X, int64_t m, int n, int64_t ld, uint32_t flags, double* R,
                double* colsum, const tsnmf_tsqr_config* cfg, hipStream_t stream);

}  // namespace tsnmf

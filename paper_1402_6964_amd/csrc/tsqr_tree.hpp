// Shared pieces of the FP64 reduction tree: the workspace layout handed to
// the kernels, wave-level LDS ordering and agent-scope fences for tickets.
#pragma once
#include "wave.hpp"

namespace tsnmf {
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
}  // namespace tsnmf

namespace tsnmf {

struct TreeArgs {
    double* nodes;       // level-major node storage: [level offset + index][n][n]
    double* node_cs;     // [level offset + index][n]
    int* tickets;        // one per pair and level, zero between calls
    int64_t leaves;      // nodes at level 0
    double* R;           // final R, n x n column-major
    double* colsum;      // final column sums or nullptr
    int32_t group;       // nodes per tree group (n <= 32 trees); 0 = the default
    int32_t pad_;
    double* rglob;       // running R of every workgroup of the wide kernels whose R
                         // does not fit in LDS (n > 128), one slot per workgroup
};

__device__ __forceinline__ void grid_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void grid_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

}  // namespace tsnmf

// Entry points whose kernels are not in this build yet: they validate nothing
// and report TSNMF_ERR_UNSUPPORTED.
#include "common.hpp"

extern "C" {
int tsnmf_batch_plan_create(int32_t, const tsnmf_matrix_desc*, uint32_t, tsnmf_batch_plan*) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_tsqr_r_batched(tsnmf_batch_plan, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_batch_plan_destroy(tsnmf_batch_plan) { return TSNMF_ERR_UNSUPPORTED; }
}

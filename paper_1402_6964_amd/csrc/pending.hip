// Entry points whose kernels are not in this build yet: they validate nothing
// and report TSNMF_ERR_UNSUPPORTED.
#include "common.hpp"

extern "C" {
int tsnmf_batch_plan_create(int32_t, const tsnmf_matrix_desc*, uint32_t, tsnmf_batch_plan*) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_tsqr_r_batched(tsnmf_batch_plan, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_batch_plan_destroy(tsnmf_batch_plan) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_select_spa(const double*, int32_t, int32_t, int32_t, const double*, int32_t, int32_t*, double*, int32_t*, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_select_xray(const double*, int32_t, int32_t, int32_t, int32_t, int32_t*, int32_t*, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_select_gp(const float*, int32_t, int32_t, int32_t, const double*, int32_t, int32_t*, int32_t*, int32_t*, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_nnls(const double*, int32_t, int32_t, int32_t, const int32_t*, int32_t, double*, int32_t, double*, int32_t*, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
int tsnmf_residual(const double*, int32_t, int32_t, int32_t, const int32_t*, int32_t, const double*, int32_t, double*, hipStream_t) { return TSNMF_ERR_UNSUPPORTED; }
}

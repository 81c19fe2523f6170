// Adjoint of the accelerated forward path (filled in below).
#include "accel_common.h"

namespace rcscm {

void launch_backward(hipStream_t s, int nt, int bpl, int nrows, const int* row_list,
                     const RowInfo* rows, const RowConstF* rcf, const RowConstD* rcd,
                     const float2* x, const float4* tsig, const float* nu, const float* ckpt_rh,
                     const float* ckpt_ru, const float* ckpt_lam, long long ckpt_stride_bins,
                     int ckpt_stride_rows, int K, float alpha, float beta, const float2* grad_s,
                     float2* grad_x, float* grad_rh0, float* grad_lam0, unsigned* status) {
  (void)s; (void)nt; (void)bpl; (void)nrows; (void)row_list; (void)rows; (void)rcf; (void)rcd;
  (void)x; (void)tsig; (void)nu; (void)ckpt_rh; (void)ckpt_ru; (void)ckpt_lam;
  (void)ckpt_stride_bins; (void)ckpt_stride_rows; (void)K; (void)alpha; (void)beta; (void)grad_s;
  (void)grad_x; (void)grad_rh0; (void)grad_lam0; (void)status;
}

}  // namespace rcscm

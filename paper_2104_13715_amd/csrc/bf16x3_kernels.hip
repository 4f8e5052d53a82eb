// Batched split-precision (bf16 x 3) implicit-GEMM evaluation (not built yet: every
// request for it is rejected at argument checking).
#include "bf16x3.h"

namespace dia {

int bf16x3_partial_rows(int, int, int, int n_ep) { return n_ep; }
size_t bf16x3_scratch_bytes(int, int) { return 0; }
int bf16x3_check_epoch(const dia_epoch&, const dia_epoch&, int) { return DIA_E_ARG; }
Bf16x3Args bf16x3_args(char* scratch, const dia_image& R, const dia_epoch*, int n, int m, const dia_objective&,
                       const float* theta0, long long theta_stride, const int* done0, long long done_stride,
                       double* partial) {
    Bf16x3Args g = {};
    g.R = R.data;
    g.n_ep = n;
    g.m = m;
    g.theta0 = theta0;
    g.theta_stride = theta_stride;
    g.done0 = done0;
    g.done_stride = done_stride;
    g.partial = partial;
    g.scratch = scratch;
    return g;
}
hipError_t bf16x3_launch_eval(const Bf16x3Args&, hipStream_t) { return hipErrorNotSupported; }

}  // namespace dia

// Batched split-precision (bf16 x 3) implicit-GEMM evaluation over epochs that share
// one reference crop: forward M[p][e] = sum_t A[p][t] K[t][e] + B0[e] and
// dL/dK[t][e] = sum_p A[p][t] g[p][e] on BF16 matrix cores, A = im2col(R) never stored.
#pragma once

#include "dia_common.h"

namespace dia {

struct Bf16x3Args {
    const float* R;         // shared reference at the epochs' common offset
    long long ldR;
    int rows, cols, m, n_ep;
    const float* const* I;  // device array of n_ep target pointers
    long long ldI;
    const float* theta0;    // epoch e's parameters at byte offset e * theta_stride
    long long theta_stride;
    const int* done0;       // epoch e's done flag at byte offset e * done_stride (nullptr: none)
    long long done_stride;
    ObjParams obj;
    double* partial;        // [n_ep][rows_per_epoch][m*m + 2]
    char* scratch;
};

int bf16x3_partial_rows(int m, int rows, int cols, int n_ep);
size_t bf16x3_scratch_bytes(int m, int n_ep);
int bf16x3_check_epoch(const dia_epoch& first, const dia_epoch& x, int m);
Bf16x3Args bf16x3_args(char* scratch, const dia_image& R, const dia_epoch* ep, int n, int m, const dia_objective& obj,
                       const float* theta0, long long theta_stride, const int* done0, long long done_stride,
                       double* partial);
hipError_t bf16x3_launch_eval(const Bf16x3Args& g, hipStream_t s);

}  // namespace dia

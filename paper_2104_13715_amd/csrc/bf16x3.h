// Batched split-precision (bf16 x 3) implicit-GEMM evaluation over epochs that share one
// reference window:
//   forward   M[e][p]  = sum_t K_e[t] X[t][p] + B0_e          (X = im2col(R), never stored)
//   backward  dL/dK_e[t] = sum_p g_e[p] X[t][p],  dL/dB0_e = sum_p g_e[p]
// on BF16 matrix cores.  Each operand x is split as x = hi + lo (both bf16) and a product
// is hi*hi + hi*lo + lo*hi, accumulated in FP32 per tile and in FP64 across tiles.
#pragma once

#include "dia_common.h"

namespace dia {

struct Bf16x3Args {
    const float* R;                // shared reference at the epochs' common window
    long long ldR;
    int rows, cols, m, n_ep;
    const float* const* I;         // device array of n_ep target pointers
    const float* const* W;         // device arrays of per-epoch weights / flat / mask (entries may be null)
    const float* const* F;
    const uint8_t* const* Mk;
    long long ldI;
    const float* theta0;           // epoch e's parameters at byte offset e * theta_stride
    long long theta_stride;
    ObjParams obj;                 // scalars (the per-epoch arrays above replace its pointers)
    double* partial;               // row (e * wpb + w) holds workgroup w's [dK (m*m), dB0, loss] for epoch e
    int wpb;                       // workgroups per block of 32 epochs
};

bool bf16x3_supported(int m);
int bf16x3_partial_rows(int m, int rows, int cols, int n_ep);
size_t bf16x3_scratch_bytes(int m, int n_ep);
int bf16x3_check_epoch(const dia_epoch& first, const dia_epoch& x, int m);
// Uploads the per-epoch pointer arrays into scratch (synchronises s) and fills *out.
int bf16x3_prepare(char* scratch, const dia_image& R, const dia_epoch* ep, int n, int m, const dia_objective& obj,
                   const float* theta0, long long theta_stride, double* partial, hipStream_t s, Bf16x3Args* out);
hipError_t bf16x3_launch_eval(const Bf16x3Args& g, hipStream_t s);

}  // namespace dia

// Batched split-precision (bf16 x 3) implicit-GEMM evaluation over epochs that share one
// reference window:
//   forward   M[e][p]  = sum_t K_e[t] X[t][p] + B0_e          (X = im2col(R), never stored)
//   backward  dL/dK_e[t] = sum_p g_e[p] X[t][p],  dL/dB0_e = sum_p g_e[p]
// on BF16 matrix cores.  Each operand x is split as x = hi + lo (both bf16) and a product
// is hi*hi + hi*lo + lo*hi, accumulated in FP32 per tile and in FP64 across tiles.
#pragma once

#include <vector>

#include "dia_common.h"

namespace dia {

constexpr int kBf16x3Block = 32;  // epochs per launch (one MFMA row block)

// Arguments of one launch: one block of up to 32 epochs.  The per-epoch pointers travel in the
// kernel arguments (nothing is uploaded per call).
struct Bf16x3Args {
    const float* R;                // shared reference at the epochs' common window
    long long ldR;
    int rows, cols, m, n_ep;       // n_ep: epochs in the whole batch
    int ep[kBf16x3Block];          // epoch index of each of the launch's 32 slots (-1: empty)
    const float* I[kBf16x3Block];  // per-slot arrays (null in empty slots; W / F / Mk
    const float* W[kBf16x3Block];  // entries may be null, and has_w / has_f / has_m say whether any
    const float* F[kBf16x3Block];  // epoch of the batch has one)
    const uint8_t* Mk[kBf16x3Block];
    int has_w, has_f, has_m;
    long long ldI;
    const float* theta0;           // epoch e's parameters at byte offset e * theta_stride
    long long theta_stride;
    ObjParams obj;                 // scalars (the per-epoch arrays above replace its pointers)
    double* partial;               // row (e * wpb + w) holds workgroup w's [dK (m*m), dB0, loss] for epoch e
    int wpb;                       // workgroups per block of 32 epochs
    const int* done;               // fits: epoch e's done flag at byte offset e * done_stride (else null);
    long long done_stride;         // a launch whose epochs are all done returns at once
};

bool bf16x3_supported(int m);
int bf16x3_partial_rows(int m, int rows, int cols, int n_ep);
int bf16x3_check_epoch(const dia_epoch& first, const dia_epoch& x, int m);
// Fills one argument block per 32 epochs of `live` (every epoch when null), in order (host only;
// no device work).
int bf16x3_prepare(const dia_image& R, const dia_epoch* ep, int n, int m, const dia_objective& obj,
                   const float* theta0, long long theta_stride, double* partial, std::vector<Bf16x3Args>* out,
                   const int* done = nullptr, long long done_stride = 0, const std::vector<int>* live = nullptr);
hipError_t bf16x3_launch_eval(const std::vector<Bf16x3Args>& blocks, hipStream_t s);

}  // namespace dia

// Kernel-kernel block of the Hessian of the loss (the observed Fisher information of
// Section 2.5 when the loss is a negative log-likelihood).  M is affine in theta, so
//     d2L / dK_t1 dK_t2 = sum_p h_p R_(p+t1) R_(p+t2),   h_p = d2l/dM2 at pixel p:
// a dense SYRK over im2col(R) with the pixels as the contraction dimension, on the FP64 matrix
// cores (v_mfma_f64_16x16x4_f64, D[16x16] += A[16x4] B[4x16]; lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16], and D[4 r + l / 16][l % 16] in register r).  FP64 throughout (FP32 reference
// values widen exactly).
//
// Work split: the taps are cut into regions of 64; a workgroup (4 waves) owns one pair of regions
// r1 <= r2 and a contiguous range of 8 x 32 pixel tiles (split-K over the image); wave w owns the
// 32 x 32 sub-block (w / 2, w % 2) as 2 x 2 MFMA tiles.  Per pixel tile the reference window
// (FP64) and h sit in LDS; a contraction step is 4 consecutive pixels of one tile row.  Pixels
// outside the valid region carry h = 0; taps past m*m read tap 0 and their rows / columns are
// dropped at assembly.
#pragma once

#include "dia_common.h"

namespace dia {

constexpr int kHessThreads = 256;
constexpr int kHessTY = 8, kHessTX = 32;
constexpr int kHessRegion = 64;
static_assert(kHessRegion * kHessRegion == kHessBlockElems, "partial block size");
constexpr int kHessTargetBlocks = 1024;

template <int M>
struct HessGeo {
    static constexpr int T = M * M;
    static constexpr int NR = (T + kHessRegion - 1) / kHessRegion;  // tap regions
    static constexpr int NPB = NR * (NR + 1) / 2;                   // region pairs r1 <= r2
    static constexpr int RH = kHessTY + M - 1;
    static constexpr int RW = kHessTX + M - 1;
    static constexpr int RS = RW | 1;                               // doubles
};

typedef double hess_f64x4 __attribute__((ext_vector_type(4)));

template <int M>
__global__ __launch_bounds__(kHessThreads) void hess_kernel(HessArgs a) {
    using G = HessGeo<M>;
    __shared__ double Rs[G::RH * G::RS];
    __shared__ double hs[kHessTY * kHessTX];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i16 = lane & 15, k4 = lane >> 4;

    // region pair of this workgroup
    int r1 = 0, rem = blockIdx.x;
    while (rem >= G::NR - r1) {
        rem -= G::NR - r1;
        ++r1;
    }
    const int r2 = r1 + rem;

    // this lane's taps in its A tiles (rows) and B tiles (columns), as LDS offsets in the window
    int offA[2], offB[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int t1 = r1 * kHessRegion + (w >> 1) * 32 + 16 * q + i16;
        const int t2 = r2 * kHessRegion + (w & 1) * 32 + 16 * q + i16;
        const int c1 = t1 < G::T ? t1 : 0, c2 = t2 < G::T ? t2 : 0;
        offA[q] = (c1 / M) * G::RS + c1 % M;
        offB[q] = (c2 / M) * G::RS + c2 % M;
    }
    hess_f64x4 acc[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = hess_f64x4{0.0, 0.0, 0.0, 0.0};

    const int Hv = a.rows - M + 1, Wv = a.cols - M + 1;
    const int ntx = (Wv + kHessTX - 1) / kHessTX, nty = (Hv + kHessTY - 1) / kHessTY;
    const int ntiles = ntx * nty;
    const int t_begin = (int)((long long)ntiles * blockIdx.y / gridDim.y);
    const int t_end = (int)((long long)ntiles * (blockIdx.y + 1) / gridDim.y);
    for (int t = t_begin; t < t_end; ++t) {
        const int ty0 = (t / ntx) * kHessTY, tx0 = (t % ntx) * kHessTX;
        __syncthreads();  // the previous tile's readers are done
        for (int idx = tid; idx < G::RH * G::RW; idx += kHessThreads) {
            const int r = idx / G::RW, c = idx - r * G::RW;
            const int gr = ty0 + r, gc = tx0 + c;
            Rs[r * G::RS + c] = (gr < a.rows && gc < a.cols) ? (double)a.R[(long long)gr * a.ldR + gc] : 0.0;
        }
        for (int idx = tid; idx < kHessTY * kHessTX; idx += kHessThreads) {
            const int r = idx / kHessTX, c = idx - r * kHessTX;
            const int gr = ty0 + r, gc = tx0 + c;
            hs[idx] = (gr < Hv && gc < Wv) ? a.h[(long long)gr * Wv + gc] : 0.0;
        }
        __syncthreads();
        for (int py = 0; py < kHessTY; ++py) {
#pragma unroll 2
            for (int c = 0; c < kHessTX / 4; ++c) {
                const int px = 4 * c + k4;  // this lane's pixel of the step
                const double hv = hs[py * kHessTX + px];
                const double* rp = Rs + py * G::RS + px;
                const double a0 = hv * rp[offA[0]], a1 = hv * rp[offA[1]];
                const double b0 = rp[offB[0]], b1 = rp[offB[1]];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
    }
    // this split's 64 x 64 block of the region pair, row-major
    double* out = a.partial + ((long long)blockIdx.y * G::NPB + blockIdx.x) * (kHessRegion * kHessRegion);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (w >> 1) * 32 + 16 * p + 4 * r + k4, col = (w & 1) * 32 + 16 * q + i16;
                out[row * kHessRegion + col] = acc[p][q][r];
            }
}

template <int M>
struct HessOps {
    static int pair_blocks() { return HessGeo<M>::NPB; }
    static int splits(int rows, int cols) {
        const int Hv = rows - M + 1, Wv = cols - M + 1;
        const int ntiles = ((Hv + kHessTY - 1) / kHessTY) * ((Wv + kHessTX - 1) / kHessTX);
        int s = (kHessTargetBlocks + HessGeo<M>::NPB - 1) / HessGeo<M>::NPB;
        return s < ntiles ? s : ntiles;
    }
    static hipError_t launch(const HessArgs& a, hipStream_t s) {
        hipLaunchKernelGGL((hess_kernel<M>), dim3(HessGeo<M>::NPB, splits(a.rows, a.cols)), dim3(kHessThreads), 0, s,
                           a);
        return hipGetLastError();
    }
};

}  // namespace dia

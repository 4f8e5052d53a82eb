// Kernel-kernel block of the Hessian of the loss (the observed Fisher information of
// Section 2.5 when the loss is a negative log-likelihood).  M is affine in theta, so
//     d2L / dK_t1 dK_t2 = sum_p h_p R_(p+t1) R_(p+t2),   h_p = d2l/dM2 at pixel p.
// FP64 throughout (FP32 reference values widen exactly).
//
// Work split: thread <-> a block of 4 x 8 tap pairs (t1 in kernel row a1, columns b1..b1+3;
// t2 in kernel row a2 >= a1, columns b2..b2+7); workgroups along y split the pixel tiles
// (split-K).  Per pixel tile the reference (with halo) and h sit in LDS; a thread walks the
// tile's rows eight pixels at a time with sliding register windows of R.
#pragma once

#include "dia_common.h"

namespace dia {

constexpr int kHessThreads = 256;
constexpr int kHessTY = 16, kHessTX = 64;
constexpr int kHessB1 = 4, kHessB2 = 8;
constexpr int kHessTargetBlocks = 1024;

template <int M>
struct HessGeo {
    static constexpr int NB1 = (M + kHessB1 - 1) / kHessB1;
    static constexpr int NB2 = (M + kHessB2 - 1) / kHessB2;
    static constexpr int NPB = M * (M + 1) / 2 * NB1 * NB2;  // pair blocks with a1 <= a2
    static constexpr int RH = kHessTY + M - 1;
    static constexpr int EXT = (NB1 * kHessB1 > NB2 * kHessB2 ? NB1 * kHessB1 : NB2 * kHessB2) + kHessB2;
    static constexpr int RW = kHessTX + EXT;
    static constexpr int RS = RW | 1;
};

template <int M>
__global__ __launch_bounds__(kHessThreads) void hess_kernel(HessArgs a) {
    using G = HessGeo<M>;
    __shared__ float Rs[G::RH * G::RS];
    __shared__ double hs[kHessTY * kHessTX];
    const int tid = threadIdx.x;
    const int pb = blockIdx.x * kHessThreads + tid;
    const bool active = pb < G::NPB;

    // decode the pair block: (a1 <= a2) row pair, then the column blocks
    const int per_pa = G::NB1 * G::NB2;
    int pa = (active ? pb : 0) / per_pa;
    const int bb = (active ? pb : 0) % per_pa;
    const int b1_0 = (bb / G::NB2) * kHessB1, b2_0 = (bb % G::NB2) * kHessB2;
    int a1 = 0;
    while (pa >= M - a1) {
        pa -= M - a1;
        ++a1;
    }
    const int a2 = a1 + pa;

    double acc[kHessB1][kHessB2];
#pragma unroll
    for (int k1 = 0; k1 < kHessB1; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < kHessB2; ++k2) acc[k1][k2] = 0.0;

    const int Hv = a.rows - M + 1, Wv = a.cols - M + 1;
    const int ntx = (Wv + kHessTX - 1) / kHessTX, nty = (Hv + kHessTY - 1) / kHessTY;
    const int ntiles = ntx * nty;
    for (int t = blockIdx.y; t < ntiles; t += gridDim.y) {
        const int ty0 = (t / ntx) * kHessTY, tx0 = (t % ntx) * kHessTX;
        for (int idx = tid; idx < G::RH * G::RW; idx += kHessThreads) {
            const int r = idx / G::RW, c = idx - r * G::RW;
            const int gr = ty0 + r, gc = tx0 + c;
            Rs[r * G::RS + c] = (gr < a.rows && gc < a.cols) ? a.R[(long long)gr * a.ldR + gc] : 0.0f;
        }
        for (int idx = tid; idx < kHessTY * kHessTX; idx += kHessThreads) {
            const int r = idx / kHessTX, c = idx - r * kHessTX;
            const int gr = ty0 + r, gc = tx0 + c;
            hs[idx] = (gr < Hv && gc < Wv) ? a.h[(long long)gr * Wv + gc] : 0.0;
        }
        __syncthreads();
        if (active) {
            for (int i = 0; i < kHessTY; ++i) {
                const float* r1 = Rs + (i + a1) * G::RS + b1_0;
                const float* r2 = Rs + (i + a2) * G::RS + b2_0;
                const double* hr = hs + i * kHessTX;
                for (int j0 = 0; j0 < kHessTX; j0 += 8) {
                    double w1[8 + kHessB1 - 1], w2[8 + kHessB2 - 1], hv[8];
#pragma unroll
                    for (int k = 0; k < 8 + kHessB1 - 1; ++k) w1[k] = (double)r1[j0 + k];
#pragma unroll
                    for (int k = 0; k < 8 + kHessB2 - 1; ++k) w2[k] = (double)r2[j0 + k];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) hv[jj] = hr[j0 + jj];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
#pragma unroll
                        for (int k1 = 0; k1 < kHessB1; ++k1) {
                            const double hw = hv[jj] * w1[jj + k1];
#pragma unroll
                            for (int k2 = 0; k2 < kHessB2; ++k2) acc[k1][k2] = fma(hw, w2[jj + k2], acc[k1][k2]);
                        }
                }
            }
        }
        __syncthreads();
    }
    if (active) {
        double* out = a.partial + ((long long)blockIdx.y * G::NPB + pb) * (kHessB1 * kHessB2);
#pragma unroll
        for (int k1 = 0; k1 < kHessB1; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < kHessB2; ++k2) out[k1 * kHessB2 + k2] = acc[k1][k2];
    }
}

template <int M>
struct HessOps {
    static int pair_blocks() { return HessGeo<M>::NPB; }
    static int splits(int rows, int cols) {
        const int Hv = rows - M + 1, Wv = cols - M + 1;
        const int ntiles = ((Hv + kHessTY - 1) / kHessTY) * ((Wv + kHessTX - 1) / kHessTX);
        const int gx = (HessGeo<M>::NPB + kHessThreads - 1) / kHessThreads;
        int s = (kHessTargetBlocks + gx - 1) / gx;
        return s < ntiles ? s : ntiles;
    }
    static hipError_t launch(const HessArgs& a, hipStream_t s) {
        const int gx = (HessGeo<M>::NPB + kHessThreads - 1) / kHessThreads;
        hipLaunchKernelGGL((hess_kernel<M>), dim3(gx, splits(a.rows, a.cols)), dim3(kHessThreads), 0, s, a);
        return hipGetLastError();
    }
};

}  // namespace dia

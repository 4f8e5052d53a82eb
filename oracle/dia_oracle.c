/*
 * FP64 CPU oracle for the DIA kernel fit: the two direct-loop correlations.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code with the HIP path.
 *
 * Both loops are written straight from the model of Section 2.1,
 * eq. (model_image_delta_basis):
 *
 *     M_ij = sum_{a,b} K_ab R_{(i+a)(j+b)} + B0
 *
 * indexed on the valid region (the "N_data" pixels of Section 2.1: a pixel of
 * the target enters only when the whole m x m footprint lies inside R), so
 * valid output (i, j) sits at target pixel (i + h, j + h), h = (m - 1) / 2.
 * Because M is linear in K, the gradient of any per-pixel objective is
 *
 *     dL/dK_ab = sum_{i,j} g_ij R_{(i+a)(j+b)},   g_ij = d l_ij / d M_ij.
 *
 * Arithmetic is IEEE double, compiled without fast-math.  Work is split over
 * fixed row blocks; each block's partial gradient is summed in block order,
 * so results do not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_ROW_BLOCK 16

/* M[i*Wv + j] = B0 + sum_{a<m, b<m} K[a*m+b] * R[(i+a)*ldR + (j+b)],  i < H-m+1, j < W-m+1 */
int oracle_model(const double* R, int64_t H, int64_t W, int64_t ldR,
                 const double* K, int64_t m, double B0, double* M) {
    if (m < 1 || H < m || W < m) return -1;
    const int64_t Hv = H - m + 1, Wv = W - m + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < Hv; ++i) {
        for (int64_t j = 0; j < Wv; ++j) {
            double s = 0.0;
            for (int64_t a = 0; a < m; ++a)
                for (int64_t b = 0; b < m; ++b)
                    s += K[a * m + b] * R[(i + a) * ldR + (j + b)];
            M[i * Wv + j] = s + B0;
        }
    }
    return 0;
}

/* dK[a*m+b] = sum_{i<Hv, j<Wv} g[i*Wv + j] * R[(i+a)*ldR + (j+b)] */
int oracle_grad_kernel(const double* R, int64_t H, int64_t W, int64_t ldR,
                       const double* g, int64_t m, double* dK) {
    if (m < 1 || H < m || W < m) return -1;
    const int64_t Hv = H - m + 1, Wv = W - m + 1;
    const int64_t nblk = (Hv + ORACLE_ROW_BLOCK - 1) / ORACLE_ROW_BLOCK;
    const int64_t nt = m * m;
    double* part = (double*)calloc((size_t)(nblk * nt), sizeof(double));
    if (!part) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nblk; ++blk) {
        double* p = part + blk * nt;
        const int64_t i1 = (blk + 1) * ORACLE_ROW_BLOCK < Hv ? (blk + 1) * ORACLE_ROW_BLOCK : Hv;
        for (int64_t a = 0; a < m; ++a)
            for (int64_t b = 0; b < m; ++b) {
                double s = 0.0;
                for (int64_t i = blk * ORACLE_ROW_BLOCK; i < i1; ++i)
                    for (int64_t j = 0; j < Wv; ++j)
                        s += g[i * Wv + j] * R[(i + a) * ldR + (j + b)];
                p[a * m + b] = s;
            }
    }
    for (int64_t t = 0; t < nt; ++t) {
        double s = 0.0;
        for (int64_t blk = 0; blk < nblk; ++blk) s += part[blk * nt + t];
        dK[t] = s;
    }
    free(part);
    return 0;
}

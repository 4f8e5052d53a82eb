// Exact-Hessian Newton steps (the Newton form of eq. newtonupdate) and the observed
// Fisher information of Section 2.5, in FP64:
//   * assemble H from the kernel-kernel pair blocks and the curvature-weighted correlation row;
//   * factor H = L L^T (blocked right-looking Cholesky over many workgroups; column k of L is
//     kept in row k of the storage, so every column read is coalesced) and solve H d = -g;
//   * trial points theta + alpha d, in FP64 for the fused pass and rounded to FP32.
#include <algorithm>

#include "newton.h"

namespace dia {

constexpr int kCholThreads = 1024;

// H[t1][t2] for the kernel taps from the split partials (fixed order; element (min, max) of the
// region-pair blocks of 64 x 64, so H is exactly symmetric), the background rows from hv: row k
// (stride n + 1) holds [sum h P_k R_(p+t) (t < m*m), sum h P_k P_l (l < nb)], P_k the k-th
// background term at the pixel (1 for the scalar B0); the background block takes element
// (min(k, l), max(k, l)), so it is exactly symmetric too.
// Entry (u, v) of L L, L the kernel-pixel Laplacian (Section 2.7, eq. laplacian; pixels sharing a
// side are adjacent): sum over w of L_uw L_wv.  On the grid: deg^2 + deg on the diagonal, -(deg u +
// deg v) for neighbours (they share no neighbour), the number of common neighbours at distance two.
__device__ __forceinline__ double lap2_entry(int u, int v, int m) {
    const int au = u / m, bu = u - au * m, av = v / m, bv = v - av * m;
    auto deg = [m](int a, int b) { return (a > 0) + (a + 1 < m) + (b > 0) + (b + 1 < m); };
    const int da = au > av ? au - av : av - au, db = bu > bv ? bu - bv : bv - bu;
    if (da + db == 0) {
        const int d = deg(au, bu);
        return (double)(d * d + d);
    }
    if (da + db == 1) return -(double)(deg(au, bu) + deg(av, bv));
    if (da + db == 2) return (da == 1) ? 2.0 : 1.0;
    return 0.0;
}

__global__ __launch_bounds__(256) void hess_assemble_kernel(const double* partial, int splits, int npb, int m,
                                                            int nb, const double* hv, double* H, double reg,
                                                            double damp) {
    constexpr int RG = 64;
    const int T = m * m, n = T + nb;
    const int nr = (T + RG - 1) / RG;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < (long long)T * T) {
        const int t1 = (int)(gid / T), t2 = (int)(gid % T);
        const int lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
        const int ra = lo / RG, rb = hi / RG;
        const int pb = ra * nr - ra * (ra - 1) / 2 + (rb - ra);
        const int k = (lo - ra * RG) * RG + (hi - rb * RG);
        double s = 0.0;
        for (int sp = 0; sp < splits; ++sp) s += partial[((long long)sp * npb + pb) * (RG * RG) + k];
        if (reg > 0.0) s += 2.0 * reg * lap2_entry(t1, t2, m);  // Hessian of the smoothness penalty
        if (t1 == t2) s *= 1.0 + damp;
        H[(long long)t1 * n + t2] = s;
    }
    if (gid < (long long)nb * n) {
        const int k = (int)(gid / n), t = (int)(gid % n);
        if (t < T) {
            const double b = hv[(long long)k * (n + 1) + t];
            H[(long long)t * n + (T + k)] = b;
            H[(long long)(T + k) * n + t] = b;
        } else {
            const int l = t - T;
            const int lo = k < l ? k : l, hi = k < l ? l : k;
            double b = hv[(long long)lo * (n + 1) + T + hi];
            if (k == l) b *= 1.0 + damp;
            H[(long long)(T + k) * n + t] = b;
        }
    }
}

__device__ double chol_block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kCholThreads / 64; ++w) s += sh[w];
    return s;
}

__device__ double chol_block_max(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kCholThreads / 64; ++w) s = fmax(s, sh[w]);
    return s;
}

// A (n x n, row-major, symmetric) -> column k of L stored in row k (A[k*n + i] = L[i][k], i >= k)
// when factor != 0; then d = -(L L^T)^-1 g.  info[0] = 1 if A was not positive definite,
// info[1] = -g.d (the Newton decrement squared), info[2] = max|d_i| / max|th_i|,
// info[3] = max_i |d_i| / (FP32 spacing at th_i).
// Blocked right-looking Cholesky A = L L^T in place, column k of L into row k of A
// (A[k*n + i] = L[i][k], i >= k; A symmetric on entry, so that row holds column k of the lower
// triangle).  Panels of kCB columns: the diagonal block is factored in LDS by one workgroup, the
// rows below it are solved against it one row per thread, and the trailing lower triangle takes
// the rank-kCB update in 32 x 32 tiles across many workgroups.  flag (device double): 0 on
// success, 1 when a pivot is not positive (A is not positive definite); later kernels of the
// same factorisation see it and return.
constexpr int kCB = 32;

__global__ __launch_bounds__(256) void chol_diag_kernel(double* A, int n, int k0, double* flag) {
    __shared__ double D[kCB][kCB + 1];
    const int tid = threadIdx.x;
    if (k0 == 0) {
        if (tid == 0) *flag = 0.0;
    } else if (*flag != 0.0) {
        return;
    }
    const int bw = n - k0 < kCB ? n - k0 : kCB;
    for (int e = tid; e < kCB * kCB; e += 256) {
        const int c = e / kCB, r = e % kCB;
        D[r][c] = (r < bw && c < bw && r >= c) ? A[(long long)(k0 + c) * n + k0 + r] : 0.0;
    }
    __syncthreads();
    bool ok = true;
    for (int c = 0; c < bw; ++c) {
        const double p = D[c][c];  // the same value in every thread: the exit is uniform
        if (!(p > 0.0)) {
            ok = false;
            break;
        }
        const double sq = sqrt(p);
        __syncthreads();
        if (tid == 0) D[c][c] = sq;
        for (int r = c + 1 + tid; r < bw; r += 256) D[r][c] /= sq;
        __syncthreads();
        const int rem = bw - c - 1;
        for (int e = tid; e < rem * rem; e += 256) {
            const int r = c + 1 + e / rem, q = c + 1 + e % rem;
            if (q <= r) D[r][q] -= D[r][c] * D[q][c];
        }
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) *flag = 1.0;
        return;
    }
    for (int e = tid; e < kCB * kCB; e += 256) {
        const int c = e / kCB, r = e % kCB;
        if (r < bw && c < bw && r >= c) A[(long long)(k0 + c) * n + k0 + r] = D[r][c];
    }
}

// Rows i >= k0 + kCB of the panel: L[i][k0 .. k0+kCB) solves L11 l^T = a^T (forward substitution).
__global__ __launch_bounds__(256) void chol_trsm_kernel(double* A, int n, int k0, const double* flag) {
    __shared__ double Ls[kCB][kCB + 1];
    if (*flag != 0.0) return;
    const int tid = threadIdx.x;
    for (int e = tid; e < kCB * kCB; e += 256) {
        const int c = e / kCB, r = e % kCB;
        Ls[r][c] = (c <= r) ? A[(long long)(k0 + c) * n + k0 + r] : 0.0;
    }
    __syncthreads();
    const int i = k0 + kCB + blockIdx.x * 256 + tid;
    if (i >= n) return;
    double x[kCB];
#pragma unroll
    for (int c = 0; c < kCB; ++c) x[c] = A[(long long)(k0 + c) * n + i];
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
        double v = x[c];
#pragma unroll
        for (int q = 0; q < c; ++q) v -= Ls[c][q] * x[q];
        x[c] = v / Ls[c][c];
    }
#pragma unroll
    for (int c = 0; c < kCB; ++c) A[(long long)(k0 + c) * n + i] = x[c];
}

// Trailing update A22 -= L21 L21^T on the lower triangle of rows and columns >= k0 + kCB: one
// 32 x 32 tile (ti >= tj) per workgroup, the linear block index mapped to (ti, tj).
__global__ __launch_bounds__(256) void chol_syrk_kernel(double* A, int n, int k0, const double* flag) {
    __shared__ double Li[kCB][kCB + 1];
    __shared__ double Lj[kCB][kCB + 1];
    if (*flag != 0.0) return;
    const int b = blockIdx.x;
    int ti = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    const int tj = b - ti * (ti + 1) / 2;
    const int k1 = k0 + kCB;
    const int i0 = k1 + ti * kCB, j0 = k1 + tj * kCB;
    const int tid = threadIdx.x;
    for (int e = tid; e < kCB * kCB; e += 256) {
        const int c = e / kCB, r = e % kCB;
        Li[r][c] = (i0 + r < n) ? A[(long long)(k0 + c) * n + i0 + r] : 0.0;
        Lj[r][c] = (j0 + r < n) ? A[(long long)(k0 + c) * n + j0 + r] : 0.0;
    }
    __syncthreads();
    const int tx = tid % kCB, ty = tid / kCB;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (int c = 0; c < kCB; ++c) {
        const double a = Li[tx][c];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += a * Lj[ty + 8 * q][c];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + tx, j = j0 + ty + 8 * q;
        if (i < n && j < n && i >= j) A[(long long)j * n + i] -= acc[q];
    }
}

hipError_t launch_chol_factor(double* A, int n, double* flag, hipStream_t s) {
    for (int k0 = 0; k0 < n; k0 += kCB) {
        hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, A, n, k0, flag);
        const int below = n - k0 - kCB;
        if (below > 0) {
            hipLaunchKernelGGL(chol_trsm_kernel, dim3((below + 255) / 256), dim3(256), 0, s, A, n, k0,
                               (const double*)flag);
            const int T = (below + kCB - 1) / kCB;
            hipLaunchKernelGGL(chol_syrk_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, s, A, n, k0,
                               (const double*)flag);
        }
    }
    return hipGetLastError();
}

// A double from lane l of the wave (l the same in every lane).
__device__ __forceinline__ double lane_value(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Newton step d = -A^-1 g from the factor in A (launch_chol_factor), with info[0] its flag:
// info = [not positive definite, decrement -g.d, max |d| / max |th|, max |d| in FP32 spacings of th].
// Blocked substitutions, kSolveBlock rows at a time: the first wave solves the block's triangle (lane j
// holding row j of it in registers, each step's quotient passed to the other lanes by readlane), then
// every thread updates its rows outside the block with the block's solved values.
constexpr int kSolveBlock = 32;

__global__ __launch_bounds__(kCholThreads) void chol_solve_kernel(const double* A, int n, const double* g,
                                                                  const double* th, double* d, double* info) {
    constexpr int B = kSolveBlock;
    __shared__ double col[kMaxTheta];  // the right-hand side being reduced
    __shared__ double sol[kMaxTheta];  // y, then x
    __shared__ double sh[32];
    const int tid = threadIdx.x, lane = tid & 63;
    if (info[0] != 0.0) {
        __syncthreads();
        if (tid == 0) {
            info[0] = 1.0;
            info[1] = 0.0;
            info[2] = 0.0;
            info[3] = 0.0;
        }
        return;
    }
    // forward: L y = -g, blocks top down (column k of L is row k of A: L[i][k] = A[k*n + i], i >= k)
    for (int i = tid; i < n; i += kCholThreads) col[i] = -g[i];
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += B) {
        const int bs = n - k0 < B ? n - k0 : B;
        if (tid < 64) {
            double lr[B];  // lane j: L[k0 + j][k0 + k], k <= j
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < B; ++k) lr[k] = 0.0;
            if (lane < bs) {
                v = col[k0 + lane];
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (k <= lane) lr[k] = A[(long long)(k0 + k) * n + k0 + lane];
            }
#pragma unroll
            for (int k = 0; k < B; ++k) {
                if (k < bs) {
                    const double yk = lane_value(v, k) / lane_value(lr[k], k);
                    if (lane == k) sol[k0 + k] = yk;
                    if (lane > k && lane < bs) v -= lr[k] * yk;
                }
            }
        }
        __syncthreads();
        for (int i = k0 + bs + tid; i < n; i += kCholThreads) {
            double s = col[i];
            for (int k = 0; k < bs; ++k) s -= A[(long long)(k0 + k) * n + i] * sol[k0 + k];
            col[i] = s;
        }
        __syncthreads();
    }
    // backward: L^T x = y, blocks bottom up (L[k][i] = A[i*n + k], i <= k), y reduced in col[], x into sol[]
    for (int i = tid; i < n; i += kCholThreads) col[i] = sol[i];
    __syncthreads();
    for (int k0 = ((n - 1) / B) * B; k0 >= 0; k0 -= B) {
        const int bs = n - k0 < B ? n - k0 : B;
        if (tid < 64) {
            double lr[B];  // lane j: L[k0 + k][k0 + j] = A[(k0 + j)*n + k0 + k], k >= j
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < B; ++k) lr[k] = 0.0;
            if (lane < bs) {
                v = col[k0 + lane];
                const double* row = A + (long long)(k0 + lane) * n + k0;
#pragma unroll
                for (int k = 0; k < B; ++k)
                    if (k >= lane && k < bs) lr[k] = row[k];
            }
#pragma unroll
            for (int k = B - 1; k >= 0; --k) {
                if (k < bs) {
                    const double xk = lane_value(v, k) / lane_value(lr[k], k);
                    if (lane == k) sol[k0 + k] = xk;
                    if (lane < k) v -= lr[k] * xk;
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < k0; i += kCholThreads) {
            const double* row = A + (long long)i * n + k0;
            double s = col[i];
            for (int k = 0; k < bs; ++k) s -= row[k] * sol[k0 + k];
            col[i] = s;
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += kCholThreads) col[i] = sol[i];
    __syncthreads();
    double dec = 0.0, dmax = 0.0, tmax = 0.0, qmax = 0.0;
    for (int i = tid; i < n; i += kCholThreads) {
        d[i] = col[i];
        dec -= g[i] * col[i];
        dmax = fmax(dmax, fabs(col[i]));
        tmax = fmax(tmax, fabs(th[i]));
        // the step in units of the FP32 spacing at th_i (the parameters are stored in FP32)
        const float tf = (float)th[i];
        const double ulp = tf != 0.0f ? ldexp(1.0, ilogbf(tf) - 23) : 1.4e-45;
        qmax = fmax(qmax, fabs(col[i]) / ulp);
    }
    dec = chol_block_sum(dec, sh);
    dmax = chol_block_max(dmax, sh);
    tmax = chol_block_max(tmax, sh);
    qmax = chol_block_max(qmax, sh);
    if (tid == 0) {
        info[0] = 0.0;
        info[1] = dec;
        info[2] = tmax > 0.0 ? dmax / tmax : dmax;
        info[3] = qmax;
    }
}

// ---------------------------------------------------------------- covariance (Section 2.5)
// Sigma = F^-1 for the observed Fisher information F = L L^T: W = L^-1 (lower triangular), then
// Sigma = W^T W.  info[0] = 1 when F (hence Sigma) is positive definite, the paper's validity
// test of Sigma (a positive definite matrix has every eigenvalue and its determinant positive);
// info[1] = ln det Sigma = -2 sum_k ln L_kk; info[2] = the smallest pivot L_kk^2.  When F is not
// positive definite the outputs are NaN.
__global__ __launch_bounds__(kCholThreads) void chol_info_kernel(const double* A, int n, const double* flag,
                                                                 double* info) {
    __shared__ double sh[32];
    const bool ok = *flag == 0.0;
    double ld = 0.0, inv_pmin = 0.0;  // the smallest pivot through the largest reciprocal (all positive)
    if (ok)
        for (int k = threadIdx.x; k < n; k += kCholThreads) {
            const double l = A[(long long)k * n + k];
            ld += log(l);
            inv_pmin = fmax(inv_pmin, 1.0 / (l * l));
        }
    ld = chol_block_sum(ld, sh);
    inv_pmin = chol_block_max(inv_pmin, sh);
    if (threadIdx.x == 0) {
        info[0] = ok ? 1.0 : 0.0;
        info[1] = ok ? -2.0 * ld : __builtin_nan("");
        info[2] = ok ? 1.0 / inv_pmin : __builtin_nan("");
    }
}

// Column j of W = L^-1 (one workgroup per column), row-major W[i*n + j], zero above the diagonal:
// w_k = (delta_jk - sum_{j <= l < k} L[k][l] w_l) / L[k][k] for k = j, j+1, ... (the running sums
// are updated as each w_k is found).
__global__ __launch_bounds__(256) void tri_inverse_kernel(const double* A, int n, double* W, const double* info) {
    __shared__ double acc[kMaxTheta];
    const int j = blockIdx.x, tid = threadIdx.x;
    if (info[0] != 1.0) {
        for (int i = tid; i < n; i += 256) W[(long long)i * n + j] = __builtin_nan("");
        return;
    }
    for (int i = tid; i < n; i += 256) {
        acc[i] = 0.0;
        if (i < j) W[(long long)i * n + j] = 0.0;
    }
    __syncthreads();
    for (int k = j; k < n; ++k) {
        const double wk = ((k == j ? 1.0 : 0.0) - acc[k]) / A[(long long)k * n + k];
        if (tid == 0) W[(long long)k * n + j] = wk;
        for (int i = k + 1 + tid; i < n; i += 256) acc[i] += A[(long long)k * n + i] * wk;
        __syncthreads();
    }
}

// Sigma[i][j] = sum_k W[k][i] W[k][j] (W lower triangular, so k >= max(i, j)); 32 x 32 output
// tiles, k in chunks of 32 staged in LDS.
constexpr int kCovTile = 32;
__global__ __launch_bounds__(256) void cov_syrk_kernel(const double* W, int n, double* S) {
    __shared__ double wa[kCovTile][kCovTile + 1];
    __shared__ double wb[kCovTile][kCovTile + 1];
    const int i0 = blockIdx.y * kCovTile, j0 = blockIdx.x * kCovTile;
    const int tx = threadIdx.x % kCovTile, ty = threadIdx.x / kCovTile;  // ty in 0..7: 4 rows each
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = (i0 > j0 ? i0 : j0); k0 < n; k0 += kCovTile) {
        for (int r = ty; r < kCovTile; r += 8) {
            const int k = k0 + r;
            wa[r][tx] = (k < n && i0 + tx < n) ? W[(long long)k * n + i0 + tx] : 0.0;
            wb[r][tx] = (k < n && j0 + tx < n) ? W[(long long)k * n + j0 + tx] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < kCovTile; ++r) {
            const double b = wb[r][tx];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += wa[r][ty + 8 * q] * b;
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = i0 + ty + 8 * q, j = j0 + tx;
        if (i < n && j < n) S[(long long)i * n + j] = acc[q];
    }
}

// sigma_p = sqrt(Sigma_pp); sigma_P^2 = 1^T Sigma_KK 1 = sum_k (sum_{i < nk} W[k][i])^2 (the kernel
// block of Sigma = W^T W, the first nk parameters), summed in a fixed order.
__global__ __launch_bounds__(256) void cov_finish_kernel(const double* S, const double* W, int n, int nk,
                                                         double* sigma, double* sigma_P, const double* info) {
    __shared__ double sh[4];
    const int tid = threadIdx.x;
    const bool ok = info[0] == 1.0;
    for (int i = tid; i < n; i += 256) sigma[i] = ok ? sqrt(S[(long long)i * n + i]) : __builtin_nan("");
    double part = 0.0;
    if (ok)
        for (int k = tid; k < n; k += 256) {
            double v = 0.0;
            for (int i = 0; i < nk && i <= k; ++i) v += W[(long long)k * n + i];
            part += v * v;
        }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((tid & 63) == 0) sh[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) *sigma_P = ok ? sqrt((sh[0] + sh[1]) + (sh[2] + sh[3])) : __builtin_nan("");
}

// theta_t = th + alpha d, stored as the FP32 parameters (and their FP64 widening) to evaluate.
// Trial point th + alpha d.  The fused pass reads the FP64 copy, so the line search sees the loss
// at the unrounded iterate: in an ill-conditioned fit the loss change from rounding the stiff
// parameters to FP32 can exceed the whole decrease still available along the soft directions.
__global__ void newton_trial_kernel(const double* th, const double* d, double alpha, float* theta, double* theta64,
                                    int n) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) {
        const double t = th[i] + alpha * d[i];
        theta[i] = (float)t;
        theta64[i] = t;
    }
}

// x = u(theta) (see the optimiser's coordinates) and the loss at that point.
__global__ __launch_bounds__(256) void set_x_kernel(FitState* st, FitVecs v, const double* th, int n, double L) {
    __shared__ double sh[8];
    const double c = st->ref_scale, s = st->ref_shift;
    const int nk = st->nk;
    double ks = 0.0;
    for (int i = threadIdx.x; i < nk; i += 256) {
        v.x[i] = c * th[i];
        ks += th[i];
    }
    for (int i = nk + 1 + threadIdx.x; i < n; i += 256) v.x[i] = th[i];
    for (int off = 32; off > 0; off >>= 1) ks += __shfl_xor(ks, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ks;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        v.x[nk] = th[nk] + s * tot;
        st->L = L;
    }
}

// theta (FP32 and FP64 copies) from the optimiser point x.
__global__ __launch_bounds__(256) void theta_from_x_kernel(const FitState* st, FitVecs v, int n) {
    __shared__ double sh[8];
    const double c = st->ref_scale, s = st->ref_shift;
    const int nk = st->nk;
    double ks = 0.0;
    for (int i = threadIdx.x; i < nk; i += 256) {
        const double k = v.x[i] / c;
        const float kf = (float)k;
        v.theta_eval[i] = kf;
        v.theta_eval64[i] = (double)kf;
        ks += k;
    }
    for (int i = nk + 1 + threadIdx.x; i < n; i += 256) {
        const float bf = (float)v.x[i];
        v.theta_eval[i] = bf;
        v.theta_eval64[i] = (double)bf;
    }
    for (int off = 32; off > 0; off >>= 1) ks += __shfl_xor(ks, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ks;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        const float bf = (float)(v.x[nk] - s * tot);
        v.theta_eval[nk] = bf;
        v.theta_eval64[nk] = (double)bf;
    }
}

hipError_t launch_hess_assemble(const double* partial, int splits, int npb, int m, int nb, const double* hv,
                                double* H, double reg, double damp, hipStream_t s) {
    const long long work = std::max<long long>((long long)m * m * m * m, (long long)nb * (m * m + nb));
    const int blocks = (int)((work + 255) / 256);
    hipLaunchKernelGGL(hess_assemble_kernel, dim3(blocks), dim3(256), 0, s, partial, splits, npb, m, nb, hv, H, reg,
                       damp);
    return hipGetLastError();
}

hipError_t launch_chol_solve(double* A, int n, int factor, const double* g, const double* th, double* d, double* info,
                             hipStream_t s) {
    if (factor && launch_chol_factor(A, n, info, s) != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(kCholThreads), 0, s, (const double*)A, n, g, th, d, info);
    return hipGetLastError();
}

hipError_t launch_covariance(double* A, int n, int nk, double* W, double* S, double* sigma, double* sigma_P,
                             double* info, hipStream_t s) {
    // W's first element holds the factorisation's flag until chol_info_kernel has read it
    if (launch_chol_factor(A, n, W, s) != hipSuccess) return hipGetLastError();
    hipLaunchKernelGGL(chol_info_kernel, dim3(1), dim3(kCholThreads), 0, s, (const double*)A, n, (const double*)W,
                       info);
    hipLaunchKernelGGL(tri_inverse_kernel, dim3(n), dim3(256), 0, s, (const double*)A, n, W, (const double*)info);
    const int nt = (n + kCovTile - 1) / kCovTile;
    hipLaunchKernelGGL(cov_syrk_kernel, dim3(nt, nt), dim3(256), 0, s, (const double*)W, n, S);
    hipLaunchKernelGGL(cov_finish_kernel, dim3(1), dim3(256), 0, s, (const double*)S, (const double*)W, n, nk, sigma,
                       sigma_P, (const double*)info);
    return hipGetLastError();
}

hipError_t launch_newton_trial(const double* th, const double* d, double alpha, float* theta, double* theta64, int n,
                               hipStream_t s) {
    hipLaunchKernelGGL(newton_trial_kernel, dim3((n + 255) / 256), dim3(256), 0, s, th, d, alpha, theta, theta64, n);
    return hipGetLastError();
}

hipError_t launch_set_x(FitState* st, FitVecs v, const double* th, int n, double L, hipStream_t s) {
    hipLaunchKernelGGL(set_x_kernel, dim3(1), dim3(256), 0, s, st, v, th, n, L);
    return hipGetLastError();
}

hipError_t launch_theta_from_x(const FitState* st, FitVecs v, int n, hipStream_t s) {
    hipLaunchKernelGGL(theta_from_x_kernel, dim3(1), dim3(256), 0, s, st, v, n);
    return hipGetLastError();
}

}  // namespace dia

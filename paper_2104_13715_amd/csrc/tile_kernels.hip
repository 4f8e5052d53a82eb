// Tiled direct-correlation kernels for gfx950: the fused forward + objective +
// backward pass of the DIA fit, the model image, and the reweight/clip pass.
//
// One persistent workgroup walks a fixed list of output tiles.  Per tile:
//   1. the reference tile with its (m-1) halo is staged in LDS once (row-coalesced);
//   2. forward (eq. model_image_delta_basis): each thread forms RB x 8 model values
//      in registers, sliding down the LDS rows; kernel taps are wave-uniform and
//      come through the scalar cache;
//   3. the per-pixel objective gives l and g = dl/dM in registers (FP64 running
//      sums of l and g); g goes to an LDS tile — the residual never reaches HBM;
//   4. backward: dL/dK_ab = sum g_ij R_(i+a)(j+b) — thread (a, strip) correlates the
//      g tile with the same LDS reference tile into m FP32 accumulators, flushed
//      into FP64 after every tile.
// At the end each workgroup reduces its m*m + 2 sums in a fixed order and
// writes one row of partials; a separate kernel adds the rows in FP64.
#include "dia_common.h"

namespace dia {

template <int M, int MODE>
__global__ __launch_bounds__(Geo<M>::NT) void tile_kernel(TileArgs a) {
    using G = Geo<M>;
    constexpr int S = G::S, NS = G::NS, NT = G::NT, RB = G::RB;
    constexpr int TX = G::TX, TY = G::TY, RW = G::RW, RS = G::RS, RH = G::RH;
    constexpr int SEG = S + M - 1;
    constexpr int H = (M - 1) / 2;
    constexpr int NPP = M * M + 2;

    __shared__ float Rs[RH * RS];
    __shared__ float gs[MODE == MODE_EVAL ? TY * TX : 1];

    if (a.done != nullptr && *a.done != 0) return;

    const int tid = threadIdx.x;
    const int q = tid / NS;   // forward: row group; backward: kernel row a
    const int cs = tid % NS;  // column strip
    const bool active = tid < G::NA;

    const int Hv = a.rows - M + 1, Wv = a.cols - M + 1;
    const int ntx = (Wv + TX - 1) / TX, nty = (Hv + TY - 1) / TY;
    const int ntiles = ntx * nty;

    // XCD-aware static schedule: workgroups are dispatched round-robin over the
    // 8 XCDs, so workgroup b runs on XCD b % 8; each XCD gets a contiguous band of
    // tiles (neighbouring tiles share halo rows in that XCD's L2).
    const int nb = gridDim.x;
    const int ngrp = nb < 8 ? nb : 8;
    const int grp = blockIdx.x % ngrp;
    const int mem = blockIdx.x / ngrp;
    const int nmem = (nb - grp + ngrp - 1) / ngrp;
    const int t_begin = (int)((long long)ntiles * grp / ngrp);
    const int t_end = (int)((long long)ntiles * (grp + 1) / ngrp);

    const float* __restrict__ K = a.theta;
    const float B0 = a.theta[M * M];

    double dk64[M];
    float dk32[M];
#pragma unroll
    for (int b = 0; b < M; ++b) dk64[b] = 0.0;
    double loss64 = 0.0, db064 = 0.0;

    for (int t = t_begin + mem; t < t_end; t += nmem) {
        const int ty0 = (t / ntx) * TY;
        const int tx0 = (t % ntx) * TX;

        // 1. stage the reference tile (zero outside the image)
        for (int idx = tid; idx < RH * RW; idx += NT) {
            const int r = idx / RW, c = idx - r * RW;
            const int gr = ty0 + r, gc = tx0 + c;
            Rs[r * RS + c] = (gr < a.rows && gc < a.cols) ? a.R[(long long)gr * a.ldR + gc] : 0.0f;
        }
        __syncthreads();

        if (active) {
            // 2. forward: acc[i][j] = B0 + sum_{ka,b} K[ka][b] * R[row + i + ka][col + j + b]
            float acc[RB][S];
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < S; ++j) acc[i][j] = B0;
            const float* rbase = Rs + (q * RB) * RS + cs * S;
            for (int r = 0; r < RB + M - 1; ++r) {
                float seg[SEG];
#pragma unroll
                for (int k = 0; k < SEG; ++k) seg[k] = rbase[r * RS + k];
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const int ka = r - i;
                    if (ka >= 0 && ka < M) {
#pragma unroll
                        for (int b = 0; b < M; ++b) {
                            const float kv = K[ka * M + b];
#pragma unroll
                            for (int j = 0; j < S; ++j) acc[i][j] = fmaf(kv, seg[j + b], acc[i][j]);
                        }
                    }
                }
            }

            // 3. per-pixel step
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int ly = q * RB + i;
                const int oy = ty0 + ly;
#pragma unroll
                for (int j = 0; j < S; ++j) {
                    const int lx = cs * S + j;
                    const int ox = tx0 + lx;
                    const bool valid = (oy < Hv) && (ox < Wv);
                    const long long pix = (long long)(oy + H) * a.ldI + (ox + H);
                    if (MODE == MODE_MODEL) {
                        if (valid) a.out[(long long)oy * a.ld_out + ox] = acc[i][j];
                    } else if (MODE == MODE_EVAL) {
                        float g = 0.0f;
                        if (valid) {
                            const bool use = (a.obj.mask == nullptr) || (a.obj.mask[pix] != 0);
                            if (use) {
                                const float w = a.obj.weights ? a.obj.weights[pix] : 1.0f;
                                const float F = a.obj.flat ? a.obj.flat[pix] : 1.0f;
                                float l;
                                pixel_objective(a.obj, a.I[pix], acc[i][j], w, F, l, g);
                                loss64 += (double)l;
                                db064 += (double)g;
                            }
                        }
                        gs[ly * TX + lx] = g;
                    } else {  // MODE_CLIP
                        if (valid) {
                            const uint8_t old = a.obj.mask ? a.obj.mask[pix] : (uint8_t)1;
                            const float F = a.obj.flat ? a.obj.flat[pix] : 1.0f;
                            const float v = model_variance(a.obj, acc[i][j], F);
                            const float z = (a.I[pix] - acc[i][j]) / sqrtf(v);
                            const uint8_t keep = (a.kappa > 0.0f && fabsf(z) > a.kappa) ? (uint8_t)0 : old;
                            a.w_out[pix] = 1.0f / v;
                            a.mask_out[pix] = keep;
                            if (old && !keep) atomicAdd(a.clip_count, 1);
                        }
                    }
                }
            }
        }

        if (MODE == MODE_EVAL) {
            __syncthreads();
            if (active) {
                // 4. backward: dk[b] += sum_i sum_j g[i][j] * R[i + q][j + b] over this strip
#pragma unroll
                for (int b = 0; b < M; ++b) dk32[b] = 0.0f;
                const float* gb = gs + cs * S;
                const float* rbase = Rs + q * RS + cs * S;
                for (int i = 0; i < TY; ++i) {
                    float gv[S];
#pragma unroll
                    for (int j = 0; j < S; ++j) gv[j] = gb[i * TX + j];
                    float seg[SEG];
#pragma unroll
                    for (int k = 0; k < SEG; ++k) seg[k] = rbase[i * RS + k];
#pragma unroll
                    for (int b = 0; b < M; ++b)
#pragma unroll
                        for (int j = 0; j < S; ++j) dk32[b] = fmaf(gv[j], seg[j + b], dk32[b]);
                }
#pragma unroll
                for (int b = 0; b < M; ++b) dk64[b] += (double)dk32[b];
            }
        }
        __syncthreads();
    }

    if (MODE != MODE_EVAL) return;

    // Block reduction in a fixed order.  dK: sum over the NS strips of each kernel row.
    double* red = reinterpret_cast<double*>(Rs);
    constexpr int CAP = (RH * RS / 2) / NT;  // kernel columns per round
    static_assert(CAP >= 1, "LDS too small for the reduction");
    double* prow = a.partial + (long long)blockIdx.x * NPP;
    for (int b0 = 0; b0 < M; b0 += CAP) {
        const int nbr = (M - b0) < CAP ? (M - b0) : CAP;
#pragma unroll
        for (int b = 0; b < M; ++b)
            if (b >= b0 && b < b0 + CAP) red[(b - b0) * NT + tid] = active ? dk64[b] : 0.0;
        __syncthreads();
        for (int o = tid; o < M * nbr; o += NT) {
            const int ka = o / nbr, kb = o - ka * nbr;
            double s = 0.0;
            for (int c = 0; c < NS; ++c) s += red[kb * NT + ka * NS + c];
            prow[ka * M + b0 + kb] = s;
        }
        __syncthreads();
    }
    // loss and dL/dB0: wave tree then waves in order
    for (int off = 32; off > 0; off >>= 1) {
        loss64 += __shfl_xor(loss64, off);
        db064 += __shfl_xor(db064, off);
    }
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) {
        red[2 * wave] = db064;
        red[2 * wave + 1] = loss64;
    }
    __syncthreads();
    if (tid == 0) {
        double sb = 0.0, sl = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            sb += red[2 * w];
            sl += red[2 * w + 1];
        }
        prow[M * M] = sb;
        prow[M * M + 1] = sl;
    }
}

// ---------------------------------------------------------------------------- dispatch
#define DIA_FOR_EACH_M(X) \
    X(1) X(3) X(5) X(7) X(9) X(11) X(13) X(15) X(17) X(19) X(21) X(23) X(25) \
    X(27) X(29) X(31) X(33) X(35) X(37) X(39) X(41) X(43) X(45) X(47) X(49)

int tile_grid_tiles(int m, int rows, int cols) {
    int tx = 0, ty = 0;
    switch (m) {
#define X(MM)                \
    case MM:                 \
        tx = Geo<MM>::TX;    \
        ty = Geo<MM>::TY;    \
        break;
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return -1;
    }
    const int Hv = rows - m + 1, Wv = cols - m + 1;
    return ((Hv + ty - 1) / ty) * ((Wv + tx - 1) / tx);
}

int tile_block_threads(int m) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return Geo<MM>::NT;
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return -1;
    }
}

template <int M>
static int max_blocks_for() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tile_kernel<M, MODE_EVAL>, Geo<M>::NT, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

int tile_max_blocks_per_cu(int m) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return max_blocks_for<MM>();
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return 1;
    }
}

template <int M>
static hipError_t launch_m(int mode, int grid, const TileArgs& a, hipStream_t s) {
    dim3 blk(Geo<M>::NT), grd(grid);
    if (mode == MODE_EVAL)
        hipLaunchKernelGGL((tile_kernel<M, MODE_EVAL>), grd, blk, 0, s, a);
    else if (mode == MODE_MODEL)
        hipLaunchKernelGGL((tile_kernel<M, MODE_MODEL>), grd, blk, 0, s, a);
    else
        hipLaunchKernelGGL((tile_kernel<M, MODE_CLIP>), grd, blk, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tile(int mode, int m, int grid, const TileArgs& a, hipStream_t s) {
    switch (m) {
#define X(MM) \
    case MM:  \
        return launch_m<MM>(mode, grid, a, s);
        DIA_FOR_EACH_M(X)
#undef X
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace dia

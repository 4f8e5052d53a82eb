// Tiled direct-correlation kernels for gfx950 (templates; instantiated per kernel size
// in tile_inst.hip): the fused forward + objective +
// backward pass of the DIA fit, the model image, the reweight/clip pass, and the
// batched work-queue form of the fused pass.
//
// Per tile (TY x TX valid outputs):
//   1. the reference tile with its (m-1) halo is staged in LDS once (row-coalesced);
//   2. forward (eq. model_image_delta_basis): each thread forms RB x 8 model values
//      in registers, sliding down the LDS rows; kernel taps are wave-uniform and
//      come through the scalar cache;
//   3. the per-pixel objective gives l and g = dl/dM in registers (FP64 running
//      sums of l and g); g goes to an LDS tile — the residual never reaches HBM;
//   4. backward: dL/dK_ab = sum g_ij R_(i+a)(j+b) — thread (a, strip) correlates the
//      g tile with the same LDS reference tile into m FP64 accumulators that persist
//      across the workgroup's tiles.
// The shapes for small images that split the kernel rows (Geo::KSPLIT) give steps 2 and 4 to two
// halves of the threads: the second half's forward sums reach the first through the g tile, the
// first half runs step 3, and each half correlates half of the g rows.
// A workgroup reduces its m*m + nb + 1 sums in a fixed order and writes one row of
// partials; a separate kernel adds the rows in FP64.  With a polynomial background
// (POLY, Section 2.6) the forward starts each pixel at B(eta, xi) and the objective step
// adds g eta^a xi^b into one FP64 sum per background term.
#pragma once

#include "tile_ops.h"

namespace dia {

template <int M, int RBV>
struct Smem {
    using G = Geo<M, RBV>;
    float Rs[G::RH * G::RS];
    double gs[G::TY * G::GS];
};

// Kernel tap (ka, b) in FP64: the widened copy in the fused pass, the FP32 value otherwise.
template <int MODE>
__device__ __forceinline__ double ktap(const TileArgs& a, int idx) {
    if (MODE == MODE_EVAL) return a.theta64[idx];
    return (double)a.theta[idx];
}

// Polynomial background at normalised coordinates (eta, xi): sum over a of eta^a c_a(xi), each
// c_a(xi) = sum_b b_ab xi^b by Horner's rule (coefficients read from theta after the m*m taps).
template <int M, int MODE>
__device__ __forceinline__ double bg_value(const TileArgs& a, double eta, double xi) {
    const int d = a.bg_deg;
    double B = 0.0, ep = 1.0;
    for (int p = 0; p <= d; ++p) {
        double c = 0.0;
        for (int b = d - p; b >= 0; --b) c = fma(c, xi, ktap<MODE>(a, M * M + bg_index(p, b, d)));
        B = fma(c, ep, B);
        ep *= eta;
    }
    return B;
}

// bg[slot of (a, b)] += g eta^a xi^b for every term of the degree-d background.  The slots follow
// the highest degree's order, so every register index is a compile-time constant.
__device__ __forceinline__ void bg_accumulate(double (&bg)[kMaxBgTerms], double g, double eta, double xi, int d) {
    double ep = g;
#pragma unroll
    for (int p = 0; p <= kMaxBgDegree; ++p) {
        double t = ep;
#pragma unroll
        for (int b = 0; b <= kMaxBgDegree - p; ++b) {
            if (p + b <= d) bg[bg_index(p, b, kMaxBgDegree)] += t;
            t *= xi;
        }
        ep *= eta;
    }
}

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

// Reference tile (with its m-1 halo) straight from global memory into LDS (zero outside the image).
template <int M, int RBV>
__device__ __forceinline__ void stage_tile(const TileArgs& a, int ty0, int tx0, float* Rs) {
    using G = Geo<M, RBV>;
    for (int idx = threadIdx.x; idx < G::RH * G::RW; idx += G::NT) {
        const int r = idx / G::RW, c = idx - r * G::RW;
        const int gr = ty0 + r, gc = tx0 + c;
        Rs[r * G::RS + G::rcol(c)] = (gr < a.rows && gc < a.cols) ? a.R[(long long)gr * a.ldR + gc] : 0.0f;
    }
}

// 3. The per-pixel step on a thread's RB x 8 model values: the objective's l and g = dl/dM (FP64
// running sums of l and g, g into the LDS tile), the curvature, the model image or the clip test.
template <int M, int RBV, int MODE, bool POLY>
__device__ __forceinline__ void tile_pixels(const TileArgs& a, const double (&acc)[Geo<M, RBV>::RB][Geo<M, RBV>::S],
                                            int q, int cs, int ty0, int tx0, double* gs, double& loss64,
                                            double& db064, double (&bg)[kMaxBgTerms]) {
    using G = Geo<M, RBV>;
    constexpr int S = G::S, RB = G::RB, GS = G::GS, GP = G::GP;
    constexpr int H = (M - 1) / 2;
    const int Hv = a.rows - M + 1, Wv = a.cols - M + 1;
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
                if (valid) a.out[(long long)oy * a.ld_out + ox] = (float)acc[i][j];
            } else if (MODE == MODE_EVAL) {
                double g = 0.0;
                if (valid) {
                    const bool use = (a.obj.mask == nullptr) || (a.obj.mask[pix] != 0);
                    if (use) {
                        const float w = a.obj.weights ? a.obj.weights[pix] : 1.0f;
                        const float F = a.obj.flat ? a.obj.flat[pix] : 1.0f;
                        double l;
                        pixel_objective_d(a.obj, (double)a.I[pix], acc[i][j], w, F, l, g);
                        loss64 += l;
                        if constexpr (POLY)
                            bg_accumulate(bg, g, a.eta0 + (double)ox * a.deta, a.xi0 + (double)oy * a.dxi,
                                          a.bg_deg);
                        else
                            db064 += g;
                    }
                }
                gs[ly * GS + cs * GP + j] = g;
            } else if (MODE == MODE_CURV) {
                double hh = 0.0;
                if (valid) {
                    const bool use = (a.obj.mask == nullptr) || (a.obj.mask[pix] != 0);
                    if (use) {
                        const float w = a.obj.weights ? a.obj.weights[pix] : 1.0f;
                        const float F = a.obj.flat ? a.obj.flat[pix] : 1.0f;
                        hh = pixel_curvature_d(a.obj, (double)a.I[pix], acc[i][j], w, F, a.curv_exact != 0);
                    }
                    if constexpr (POLY) {
                        if (a.curv_a == 0 && a.curv_b == 0) a.h_out[(long long)oy * Wv + ox] = hh;
                        const double eta = a.eta0 + (double)ox * a.deta, xi = a.xi0 + (double)oy * a.dxi;
                        hh *= ipow(eta, a.curv_a) * ipow(xi, a.curv_b);
                        bg_accumulate(bg, hh, eta, xi, a.bg_deg);
                    } else {
                        a.h_out[(long long)oy * Wv + ox] = hh;
                        db064 += hh;
                    }
                }
                gs[ly * GS + cs * GP + j] = hh;
            } else {  // MODE_CLIP
                if (valid) {
                    const uint8_t old = a.obj.mask ? a.obj.mask[pix] : (uint8_t)1;
                    const float F = a.obj.flat ? a.obj.flat[pix] : 1.0f;
                    const float Mf = (float)acc[i][j];
                    const float v = model_variance(a.obj, Mf, F);
                    const float z = (float)((double)a.I[pix] - acc[i][j]) / sqrtf(v);
                    const uint8_t keep = (a.kappa > 0.0f && fabsf(z) > a.kappa) ? (uint8_t)0 : old;
                    a.w_out[pix] = 1.0f / v;
                    a.mask_out[pix] = keep;
                    if (old && !keep) atomicAdd(a.clip_count, 1);
                }
            }
        }
    }
}

// One tile whose reference window is already staged in LDS: forward, per-pixel step, and
// (MODE_EVAL / MODE_CURV) backward into dk64.  With two thread sets, nsets = 1 runs a half tile: the
// first set's rows only, the second set's threads idle.  With the kernel rows split (KS = 2), the
// second half of the threads hands its forward sums to the first through the g tile; the first half
// runs the per-pixel step; each half correlates its own g rows in the backward pass.
// FP32 data (exactly widened), FP64 products and sums: on gfx950 an FP64 FMA issues at the
// rate of a non-packed FP32 FMA.
template <int M, int RBV, int MODE, bool POLY = false>
__device__ __forceinline__ void tile_body(const TileArgs& a, double B0, int ty0, int tx0, float* Rs, double* gs,
                                          double (&dk64)[M], double& loss64, double& db064,
                                          double (&bg)[kMaxBgTerms], int nsets = Geo<M, RBV>::TS) {
    using G = Geo<M, RBV>;
    constexpr int S = G::S, NS = G::NS, RB = G::RB;
    constexpr int RS = G::RS, SP = G::SP, GP = G::GP;
    constexpr int GS = G::GS;
    constexpr int SEG = S + M - 1;
    const int tid = threadIdx.x;
    const int ks = G::KSPLIT ? tid / (M * NS) : 0;  // kernel-row half
    const int tk = G::KSPLIT ? tid - ks * (M * NS) : tid;
    const int q = tk / NS;   // forward: row group; backward: kernel row a
    const int cs = tk % NS;  // column strip
    const bool active = tid < G::NA && q / M < nsets;  // q / M: the thread's set
    // kernel rows of this thread's forward sums
    const int klo = G::KSPLIT ? (ks == 0 ? 0 : G::KA0) : 0;
    const int khi = G::KSPLIT ? (ks == 0 ? G::KA0 : M) : M;

    double acc[RB][S];
    if (active) {
        // 2. forward: acc[i][j] = B0 + sum_{ka,b} K[ka][b] * R[row + i + ka][col + j + b]
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if constexpr (POLY) {
                    const double xi = a.xi0 + (double)(ty0 + q * RB + i) * a.dxi;
                    const double eta = a.eta0 + (double)(tx0 + cs * S + j) * a.deta;
                    acc[i][j] = ks == 0 ? bg_value<M, MODE>(a, eta, xi) : 0.0;
                } else {
                    acc[i][j] = ks == 0 ? B0 : 0.0;
                }
            }
        const float* rbase = Rs + (q * RB) * RS + cs * SP;
        for (int r = klo; r < khi + RB - 1; ++r) {
            double seg[SEG];
#pragma unroll
            for (int k = 0; k < SEG; ++k) seg[k] = (double)rbase[r * RS + G::rcol(k)];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const int ka = r - i;
                if (ka >= klo && ka < khi) {
#pragma unroll
                    for (int b = 0; b < M; ++b) {
                        const double kv = ktap<MODE>(a, ka * M + b);
#pragma unroll
                        for (int j = 0; j < S; ++j) acc[i][j] = fma(kv, seg[j + b], acc[i][j]);
                    }
                }
            }
        }
        if constexpr (!G::KSPLIT) tile_pixels<M, RBV, MODE, POLY>(a, acc, q, cs, ty0, tx0, gs, loss64, db064, bg);
    }
    if constexpr (G::KSPLIT) {
        if (active && ks == 1)
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < S; ++j) gs[(q * RB + i) * GS + cs * GP + j] = acc[i][j];
        __syncthreads();
        if (active && ks == 0) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < S; ++j) acc[i][j] += gs[(q * RB + i) * GS + cs * GP + j];
            tile_pixels<M, RBV, MODE, POLY>(a, acc, q, cs, ty0, tx0, gs, loss64, db064, bg);
        }
    }

    if (MODE == MODE_EVAL || MODE == MODE_CURV) {
        __syncthreads();
        if (active) {
            // 4. backward: dk[b] += sum_i sum_j g[i][j] * R[i + a][j + b] over this strip, thread q = (set, a)
            // taking the g rows of its set (of its half of them with the kernel rows split)
            constexpr int TYS = G::TYS;
            const int set = q / M, ka = q - set * M;
            const int ilo = G::KSPLIT ? (ks == 0 ? 0 : TYS - TYS / 2) : set * TYS;
            const int ihi = G::KSPLIT ? (ks == 0 ? TYS - TYS / 2 : TYS) : (set + 1) * TYS;
            const double* gb = gs + cs * GP;
            const float* rbase = Rs + ka * RS + cs * SP;
            for (int i = ilo; i < ihi; ++i) {
                double gv[S];
#pragma unroll
                for (int j = 0; j < S; ++j) gv[j] = gb[i * GS + j];
                double seg[SEG];
#pragma unroll
                for (int k = 0; k < SEG; ++k) seg[k] = (double)rbase[i * RS + G::rcol(k)];
#pragma unroll
                for (int b = 0; b < M; ++b)
#pragma unroll
                    for (int j = 0; j < S; ++j) dk64[b] = fma(gv[j], seg[j + b], dk64[b]);
            }
        }
    }
    __syncthreads();
}

// Fixed-order workgroup reduction of the per-thread sums into one partial row:
// prow[a*m + b] = dL/dK_ab, prow[m*m] = dL/dB0, prow[m*m + 1] = loss; with a polynomial background
// (POLY, degree d, nb terms) prow[m*m + k] = dL/db_k for k < nb and prow[m*m + nb] = loss.
template <int M, int RBV, bool POLY = false>
__device__ __forceinline__ void write_partials(const double (&dk64)[M], double loss64, double db064,
                                               double (&bg)[kMaxBgTerms], int d, float* Rs, double* prow) {
    using G = Geo<M, RBV>;
    constexpr int NS = G::NS, NT = G::NT;
    const int tid = threadIdx.x;
    const bool active = tid < G::NA;
    double* red = reinterpret_cast<double*>(Rs);
    constexpr int CAP = (G::RH * G::RS / 2) / NT;  // kernel columns per round
    static_assert(CAP >= 1, "LDS too small for the reduction");
    for (int b0 = 0; b0 < M; b0 += CAP) {
        const int nbr = (M - b0) < CAP ? (M - b0) : CAP;
#pragma unroll
        for (int b = 0; b < M; ++b)
            if (b >= b0 && b < b0 + CAP) red[(b - b0) * NT + tid] = active ? dk64[b] : 0.0;
        __syncthreads();
        for (int o = tid; o < M * nbr; o += NT) {
            const int ka = o / nbr, kb = o - ka * nbr;
            double s = 0.0;
            for (int set = 0; set < G::TS * G::KS; ++set)  // thread sets, or kernel-row halves
                for (int c = 0; c < NS; ++c) s += red[kb * NT + (set * M + ka) * NS + c];
            prow[ka * M + b0 + kb] = s;
        }
        __syncthreads();
    }
    const int lane = tid & 63, wave = tid >> 6;
    if constexpr (POLY) {
        // one slot per background term of the highest degree, then the loss
        constexpr int NSL = kMaxBgTerms + 1;
#pragma unroll
        for (int k = 0; k < kMaxBgTerms; ++k)
            for (int off = 32; off > 0; off >>= 1) bg[k] += __shfl_xor(bg[k], off);
        for (int off = 32; off > 0; off >>= 1) loss64 += __shfl_xor(loss64, off);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kMaxBgTerms; ++k) red[NSL * wave + k] = bg[k];
            red[NSL * wave + kMaxBgTerms] = loss64;
        }
        __syncthreads();
        if (tid == 0) {
            for (int p = 0; p <= d; ++p)
                for (int b = 0; b <= d - p; ++b) {
                    double sb = 0.0;
                    for (int w = 0; w < NT / 64; ++w) sb += red[NSL * w + bg_index(p, b, kMaxBgDegree)];
                    prow[M * M + bg_index(p, b, d)] = sb;
                }
            double sl = 0.0;
            for (int w = 0; w < NT / 64; ++w) sl += red[NSL * w + kMaxBgTerms];
            prow[M * M + bg_terms(d)] = sl;
        }
    } else {
        for (int off = 32; off > 0; off >>= 1) {
            loss64 += __shfl_xor(loss64, off);
            db064 += __shfl_xor(db064, off);
        }
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
    __syncthreads();
}

// Single pair: a persistent grid walks a static, XCD-aware list of tiles.
template <int M, int MODE, int RBV, bool POLY = false>
__global__ __launch_bounds__((Geo<M, RBV>::NT)) __attribute__((amdgpu_waves_per_eu(Geo<M, RBV>::WAVES_PER_EU)))
void tile_kernel(TileArgs a) {
    using G = Geo<M, RBV>;
    __shared__ Smem<M, RBV> sm;
    if (a.done != nullptr && *a.done != 0) return;

    const int Hv = a.rows - M + 1, Wv = a.cols - M + 1;
    const int ntx = (Wv + G::TX - 1) / G::TX, nty = (Hv + G::TY - 1) / G::TY;
    const int ntiles = ntx * nty;

    // Workgroups are dispatched round-robin over the 8 XCDs, so workgroup b runs on
    // XCD b % 8; each XCD gets a contiguous band of tiles (neighbouring tiles share
    // halo rows in that XCD's L2), as many as its share of the workgroups (when the grid is
    // not a multiple of 8 the first nb % 8 XCDs have one workgroup more; equal bands would then
    // give some workgroup of the others a second tile while workgroups elsewhere have one).
    const int nb = gridDim.x;
    const int ngrp = nb < 8 ? nb : 8;
    const int grp = blockIdx.x % ngrp;
    const int mem = blockIdx.x / ngrp;
    const int q8 = nb / ngrp, r8 = nb - q8 * ngrp;
    const int nmem = q8 + (grp < r8 ? 1 : 0);
    const long long w0 = (long long)grp * q8 + (grp < r8 ? grp : r8);  // workgroups of the XCDs before
    const int t_begin = (int)((long long)ntiles * w0 / nb);
    const int t_end = (int)((long long)ntiles * (w0 + nmem) / nb);

    const double B0 = POLY ? 0.0 : ktap<MODE>(a, M * M);
    double dk64[M];
#pragma unroll
    for (int b = 0; b < M; ++b) dk64[b] = 0.0;
    double loss64 = 0.0, db064 = 0.0;
    double bg[kMaxBgTerms];
#pragma unroll
    for (int k = 0; k < kMaxBgTerms; ++k) bg[k] = 0.0;

    // Each member takes every nmem-th tile of its band.  With two thread sets, when the band's last
    // round leaves at least half of the members idle, its tiles are split into half tiles (the rows of
    // one set each), so that the round takes about half as long.
    const int rounds = (t_end - t_begin) / nmem;
    const int rest = t_end - t_begin - rounds * nmem;
    const bool halves = G::TS == 2 && 2 * rest <= nmem;
    const int n_items = rounds + ((halves ? mem < 2 * rest : mem < rest) ? 1 : 0);
    for (int k = 0; k < n_items; ++k) {
        int t = t_begin + mem + k * nmem, row_shift = 0, nsets = G::TS;
        if (k == rounds) {  // the last, partial round
            t = t_begin + rounds * nmem + (halves ? mem / 2 : mem);
            row_shift = halves ? (mem % 2) * G::TYS : 0;
            nsets = halves ? 1 : G::TS;
        }
        const int ty0 = (t / ntx) * G::TY + row_shift, tx0 = (t % ntx) * G::TX;
        stage_tile<M, RBV>(a, ty0, tx0, sm.Rs);
        __syncthreads();
        tile_body<M, RBV, MODE, POLY>(a, B0, ty0, tx0, sm.Rs, sm.gs, dk64, loss64, db064, bg, nsets);
    }

    if (MODE == MODE_EVAL || MODE == MODE_CURV) {
        const long long npp = POLY ? (M * M + bg_terms(a.bg_deg) + 1) : (M * M + 2);
        write_partials<M, RBV, POLY>(dk64, loss64, db064, bg, a.bg_deg, sm.Rs, a.partial + (long long)blockIdx.x * npp);
    }
}

// Batched fused pass: a persistent grid pops chunks (runs of tiles of one epoch)
// from a work queue.  Each chunk has its own partial row, so the result does not
// depend on which workgroup ran it.  Chunks of converged epochs are skipped.
template <int M, int RBV>
__global__ __launch_bounds__((Geo<M, RBV>::NT)) __attribute__((amdgpu_waves_per_eu(Geo<M, RBV>::WAVES_PER_EU)))
void batched_eval_kernel(BatchedArgs b) {
    using G = Geo<M, RBV>;
    __shared__ Smem<M, RBV> sm;
    __shared__ int chunk_sh;
    for (;;) {
        if (threadIdx.x == 0) chunk_sh = atomicAdd(b.queue, 1);
        __syncthreads();
        const int c = chunk_sh;
        __syncthreads();
        if (c >= b.n_chunks) break;
        const ChunkDev ch = b.chunks[c];
        const EpochDev e = b.ep[ch.epoch];
        if (*e.done != 0) continue;
        TileArgs a;
        a.R = e.R;
        a.ldR = b.ldR;
        a.I = e.I;
        a.ldI = e.ldI;
        a.rows = e.rows;
        a.cols = e.cols;
        a.theta = e.theta;
        a.theta64 = e.theta64;
        a.obj = b.obj;
        a.obj.weights = e.weights;
        a.obj.flat = e.flat;
        a.obj.mask = e.mask;
        const double B0 = e.theta64[M * M];
        double dk64[M];
#pragma unroll
        for (int k = 0; k < M; ++k) dk64[k] = 0.0;
        double loss64 = 0.0, db064 = 0.0;
        double bg[kMaxBgTerms];  // unused: the batched fits have the scalar background
        for (int t = ch.t_begin; t < ch.t_end; ++t) {
            stage_tile<M, RBV>(a, (t / e.ntx) * G::TY, (t % e.ntx) * G::TX, sm.Rs);
            __syncthreads();
            tile_body<M, RBV, MODE_EVAL>(a, B0, (t / e.ntx) * G::TY, (t % e.ntx) * G::TX, sm.Rs, sm.gs, dk64, loss64,
                                         db064, bg);
        }
        write_partials<M, RBV>(dk64, loss64, db064, bg, 0, sm.Rs, b.partial + (long long)c * (M * M + 2));
    }
}

// ---------------------------------------------------------------------------- per-size entry points
template <int M, int RBV, bool BATCHED>
static int occupancy_for() {
    int n = 0;
    hipError_t e;
    if constexpr (BATCHED)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batched_eval_kernel<M, RBV>, Geo<M, RBV>::NT, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, tile_kernel<M, MODE_EVAL, RBV>, Geo<M, RBV>::NT, 0);
    if (e != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

template <int M, int RBV>
static hipError_t launch_eval_v(int grid, const TileArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((tile_kernel<M, MODE_EVAL, RBV>), dim3(grid), dim3(Geo<M, RBV>::NT), 0, s, a);
    return hipGetLastError();
}

template <int M, int RBV>
static hipError_t launch_bv(int grid, const BatchedArgs& b, hipStream_t s) {
    hipLaunchKernelGGL((batched_eval_kernel<M, RBV>), dim3(grid), dim3(Geo<M, RBV>::NT), 0, s, b);
    return hipGetLastError();
}

template <int M>
hipError_t TileOps<M>::launch(int mode, int grid, const TileArgs& a, hipStream_t s, int v) {
    dim3 blk(Geo<M, 0>::NT), grd(grid);
    if (a.bg_deg > 0) {
        // polynomial background: the default tile shape; no reweight/clip pass
        if (v != 0 || a.bg_deg > kMaxBgDegree || a.nb != bg_terms(a.bg_deg)) return hipErrorInvalidValue;
        if (mode == MODE_EVAL)
            hipLaunchKernelGGL((tile_kernel<M, MODE_EVAL, 0, true>), grd, blk, 0, s, a);
        else if (mode == MODE_CURV)
            hipLaunchKernelGGL((tile_kernel<M, MODE_CURV, 0, true>), grd, blk, 0, s, a);
        else if (mode == MODE_MODEL)
            hipLaunchKernelGGL((tile_kernel<M, MODE_MODEL, 0, true>), grd, blk, 0, s, a);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (v == 0 || mode != MODE_EVAL) {
        if (mode == MODE_EVAL)
            hipLaunchKernelGGL((tile_kernel<M, MODE_EVAL, 0>), grd, blk, 0, s, a);
        else if (mode == MODE_CURV)
            hipLaunchKernelGGL((tile_kernel<M, MODE_CURV, 0>), grd, blk, 0, s, a);
        else if (mode == MODE_MODEL)
            hipLaunchKernelGGL((tile_kernel<M, MODE_MODEL, 0>), grd, blk, 0, s, a);
        else
            hipLaunchKernelGGL((tile_kernel<M, MODE_CLIP, 0>), grd, blk, 0, s, a);
        return hipGetLastError();
    }
    if constexpr (HasVariants<M>::value) {
        if (v == 1) return launch_eval_v<M, 1>(grid, a, s);
        if (v == 2) return launch_eval_v<M, 2>(grid, a, s);
        if (v == 3) return launch_eval_v<M, 4>(grid, a, s);
        if (v == 4) return launch_eval_v<M, 17>(grid, a, s);
        if (v == 6) return launch_eval_v<M, variant_rbv<M>(6)>(grid, a, s);
        if (v == 7) return launch_eval_v<M, variant_rbv<M>(7)>(grid, a, s);
        if (v == 8) return launch_eval_v<M, variant_rbv<M>(8)>(grid, a, s);
        return launch_eval_v<M, 9>(grid, a, s);
    }
    return hipErrorInvalidValue;
}

template <int M>
hipError_t TileOps<M>::launch_batched(int grid, const BatchedArgs& b, hipStream_t s, int v) {
    if (v == 0) return launch_bv<M, 0>(grid, b, s);
    if constexpr (HasVariants<M>::value) {
        if (v == 1) return launch_bv<M, 1>(grid, b, s);
        if (v == 2) return launch_bv<M, 2>(grid, b, s);
        if (v == 3) return launch_bv<M, 4>(grid, b, s);
        if (v == 4) return launch_bv<M, 17>(grid, b, s);
    }
    return hipErrorInvalidValue;  // the batched forms use the wide shapes, variants 0 - 4
}

template <int M>
int TileOps<M>::occupancy(int v, bool batched) {
    if (batched) {
        if (v == 0) return occupancy_for<M, 0, true>();
        if constexpr (HasVariants<M>::value) {
            if (v == 1) return occupancy_for<M, 1, true>();
            if (v == 2) return occupancy_for<M, 2, true>();
            if (v == 3) return occupancy_for<M, 4, true>();
            if (v == 4) return occupancy_for<M, 17, true>();
        }
        return 1;
    }
    if (v == 0) return occupancy_for<M, 0, false>();
    if constexpr (HasVariants<M>::value) {
        if (v == 1) return occupancy_for<M, 1, false>();
        if (v == 2) return occupancy_for<M, 2, false>();
        if (v == 3) return occupancy_for<M, 4, false>();
        if (v == 4) return occupancy_for<M, 17, false>();
        if (v == 6) return occupancy_for<M, variant_rbv<M>(6), false>();
        if (v == 7) return occupancy_for<M, variant_rbv<M>(7), false>();
        if (v == 8) return occupancy_for<M, variant_rbv<M>(8), false>();
        return occupancy_for<M, 9, false>();
    }
    return 1;
}

}  // namespace dia

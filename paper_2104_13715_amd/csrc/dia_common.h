// Internal declarations shared by the HIP kernels and the C-ABI layer of libdia.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dia.h"

namespace dia {

// Per-pixel objective parameters as the kernels see them (float, host-converted).
struct ObjParams {
    int rho;
    int var;
    double s0sq;       // sigma0^2
    double inv_gain;   // 1 / G
    double excess;     // E
    double var_floor;  // lower bound on sigma^2
    double c;          // Huber / Cauchy scale
    double inv_c2;     // 1 / c^2
    const float* weights;
    const float* flat;
    const uint8_t* mask;
};

// Spatially varying background (Section 2.6, eq. polybackground): B(x, y) = sum b_ab eta^a xi^b over
// a + b <= d, in the normalised coordinates of eq. normcoords.  theta holds the kernel (m*m values),
// then the coefficients in the equation's summation order (a = 0..d outer, b = 0..d-a inner), so b_00
// sits where the scalar B0 does and d = 0 is the scalar background.
constexpr int kMaxBgDegree = DIA_MAX_BG_DEGREE;
constexpr int kMaxBgTerms = (kMaxBgDegree + 1) * (kMaxBgDegree + 2) / 2;
__host__ __device__ constexpr int bg_terms(int d) { return (d + 1) * (d + 2) / 2; }
// position of eta^a xi^b among the coefficients of a degree-d background
__host__ __device__ constexpr int bg_index(int a, int b, int d) { return a * (d + 1) - a * (a - 1) / 2 + b; }

// What one launch of the tiled kernel does with the forward result.
enum TileMode { MODE_EVAL = 0, MODE_MODEL = 1, MODE_CLIP = 2, MODE_CURV = 3 };

struct TileArgs {
    const float* R;
    long long ldR;
    const float* I;
    long long ldI;     // also the leading dimension of weights, flat, mask, w_out, mask_out
    int rows, cols;
    const float* theta;    // K (m*m, row-major) then the nb background coefficients
    const double* theta64; // MODE_EVAL / MODE_CURV: the same values in FP64
    ObjParams obj;
    double* partial;     // MODE_EVAL / MODE_CURV: [gridDim.x][m*m + nb + 1]: dL/dK, dL/db, loss
    float* out;          // MODE_MODEL: valid model
    long long ld_out;
    float* w_out;        // MODE_CLIP: 1/v(M) on the target grid
    uint8_t* mask_out;   // MODE_CLIP: updated mask on the target grid
    float kappa;         // MODE_CLIP: clip |z| > kappa (0 = keep every pixel)
    int* clip_count;     // MODE_CLIP: pixels newly clipped (integer atomics)
    const int* done;     // if non-null and *done != 0 the launch does nothing
    double* h_out;       // MODE_CURV: per-pixel curvature d2l/dM2 on the valid region, row stride Wv
    int curv_exact;      // MODE_CURV: 1 = exact d2l/dM2, 0 = the positive Gauss-Newton / IRLS form
    // background: nb coefficients after the kernel (1 = the scalar B0); degree bg_deg >= 1 selects the
    // polynomial form, with eta = eta0 + ox * deta at valid column ox and xi = xi0 + oy * dxi at valid row oy
    int nb, bg_deg;
    double eta0, deta, xi0, dxi;
    // MODE_CURV with a polynomial background: the pass weights each pixel's curvature by the monomial
    // eta^curv_a xi^curv_b (its partial row is then that background term's row of the Hessian); h_out is
    // written by the unweighted pass (curv_a = curv_b = 0) only
    int curv_a, curv_b;
};

// Geometry of the tiled kernel for an m x m kernel (all compile-time).
//  - backward: thread (a, cs) owns kernel row a and column strip cs (S pixels wide),
//    so m * NS threads cover the m x m taps of one tile;
//  - forward: thread (rg, cs) owns RB output rows x S output columns.
//  - tile = TY x TX outputs; the reference tile (with its m-1 halo) and the g tile live in LDS.
// LDS layout: every run of 8 columns (one thread's strip) is stored with a pitch of SP floats
// (reference) or GP doubles (g tile), and the reference row stride RS is 2 mod 64 words.  With
// plain rows the strips of neighbouring lanes start 8 words apart and pile onto a few banks;
// with this skew the lanes of a wave read distinct banks (backward, g tile) or at most two-way
// shared ones (forward).
// RBV selects the rows per forward thread (0 = the largest of 4, 2, 1 whose LDS fits the budget);
// the autotuner chooses among the variants that are compiled.  RBV >= 16 asks for two thread sets
// (TS = 2) of RBV - 16 forward rows per thread: twice the threads and tile rows of the same
// per-thread work, each set correlating its own half of the g tile in the backward pass, so a
// workgroup is 8 waves and two workgroups per CU give 4 waves per SIMD.
template <int M, int RBV = 0>
struct Geo {
    static constexpr int kLdsBudget = 80 * 1024;         // two workgroups per CU
    static constexpr int S = 8;
    static constexpr int SP = 10;                        // reference strip pitch (floats per 8 columns)
    static constexpr int GP = 9;                         // g strip pitch (doubles per 8 columns)
    // RBV >= 8 asks for the narrow shape (RBV - 8 forward rows per thread): about one wave of column
    // strips per workgroup, so that images too small to fill the chip with wide tiles still do
    static constexpr bool NARROW = RBV >= 8 && RBV < 16;
    // RBV >= 32: two thread sets of one forward row and RBV - 32 column strips (a short tile of fewer
    // threads, for images too small to keep the chip busy with the wide two-set shape).
    // RBV >= 64: one forward row and RBV - 64 column strips, with the kernel rows split over two halves
    // of the threads (KS = 2): each half forms the forward sums over its kernel rows and correlates
    // its half of the g rows, so a thread does half the work of the unsplit shape (for small images,
    // whose passes are bound by the latency of one tile)
    static constexpr bool EXPLICIT_NS = RBV >= 32;
    static constexpr bool KSPLIT = RBV >= 64;
    static constexpr int KS = KSPLIT ? 2 : 1;            // kernel-row halves
    static constexpr int TS = (RBV >= 16 && !KSPLIT) ? 2 : 1;  // thread sets
    static constexpr int RBR = EXPLICIT_NS ? 1 : (NARROW ? RBV - 8 : (TS == 2 ? RBV - 16 : RBV));
    static constexpr int NS = EXPLICIT_NS ? RBV - (KSPLIT ? 64 : 32)
                            : (NARROW ? ((64 / M) > 1 ? (64 / M) : 1) : ((256 / M) < 32 ? (256 / M) : 32));
    static constexpr int KA0 = (M + 1) / 2;              // kernel rows of the first half (KS = 2)
    static constexpr int NA = KS * TS * M * NS;          // active threads
    static constexpr int NT = ((NA + 63) / 64) * 64;     // launched threads (whole waves)
    static constexpr int TX = NS * S;
    static constexpr int RW = TX + M - 1;                // reference tile width (columns)
    static constexpr int RS0 = (RW + 7) / 8 * SP;        // words needed per reference row
    static constexpr int RS = RS0 + ((2 - RS0) % 64 + 64) % 64;  // row stride, = 2 (mod 64)
    static constexpr int GS = NS * GP;                   // g tile row stride (doubles)
    // FP32 reference tile + FP64 g tile
    static constexpr int lds_bytes(int rb) { return 4 * (TS * M * rb + M - 1) * RS + 8 * TS * M * rb * GS; }
    static constexpr int RB_AUTO = lds_bytes(4) <= kLdsBudget ? 4 : (lds_bytes(2) <= kLdsBudget ? 2 : 1);
    static constexpr int RB = (RBR > 0 && lds_bytes(RBR) <= kLdsBudget) ? RBR : RB_AUTO;
    static constexpr int TY = TS * M * RB;
    static constexpr int TYS = M * RB;                   // g rows of one thread set
    static constexpr int RH = TY + M - 1;                // reference tile height
    // waves per SIMD that the LDS allows (160 KB per CU); the kernels are compiled for it
    // (rounded up for the explicit-strip shapes, whose workgroups need not divide evenly over the SIMDs)
    static constexpr int WAVES_PER_EU0 = (((160 * 1024) / lds_bytes(RB)) * (NT / 64) + (EXPLICIT_NS ? 3 : 0)) / 4;
    // (at most 4 for the explicit-strip shapes, 3 with the kernel rows split: their loops need about 128
    // and 168 registers)
    static constexpr int WAVES_PER_EU1 = EXPLICIT_NS && WAVES_PER_EU0 > (KSPLIT ? 3 : 4) ? (KSPLIT ? 3 : 4) : WAVES_PER_EU0;
    static constexpr int WAVES_PER_EU = WAVES_PER_EU1 < 1 ? 1 : (WAVES_PER_EU1 > 8 ? 8 : WAVES_PER_EU1);
    // word offset of column c within a reference row / double offset within a g row
    static __host__ __device__ constexpr int rcol(int c) { return (c >> 3) * SP + (c & 7); }
    static __host__ __device__ constexpr int gcol(int c) { return (c >> 3) * GP + (c & 7); }
};
static_assert(Geo<49>::lds_bytes(Geo<49>::RB) <= Geo<49>::kLdsBudget, "LDS budget at m = 49");

// One epoch of a batched fit as the kernels see it.
struct EpochDev {
    const float* R;        // shared reference, already offset to this epoch's crop
    const float* I;
    long long ldI;
    int rows, cols;
    const float* theta;    // the point being evaluated (m*m + 1 floats)
    const double* theta64; // the same values widened to FP64
    const float* weights;
    const float* flat;
    const uint8_t* mask;
    const int* done;       // this epoch's done flag
    int ntx;               // tiles across the valid region
    int pad;
};

// A run of consecutive tiles of one epoch, processed by one workgroup into one partial row.
struct ChunkDev {
    int epoch, t_begin, t_end, pad;
};

struct BatchedArgs {
    const EpochDev* ep;
    const ChunkDev* chunks;
    int n_chunks;
    long long ldR;
    ObjParams obj;     // shared scalars; weights / flat / mask come from the epoch
    double* partial;   // [n_chunks][m*m + 2]
    int* queue;        // work-queue head (reset by the reduce kernel)
};

// rho(z) and psi(z) = rho'(z) for the three loss shapes.
__device__ __forceinline__ void rho_psi(const ObjParams& o, float z, float& rho, float& psi) {
    if (o.rho == DIA_RHO_GAUSS) {
        rho = 0.5f * z * z;
        psi = z;
    } else if (o.rho == DIA_RHO_HUBER) {
        const float c = (float)o.c;
        const float az = fabsf(z);
        if (az <= c) {
            rho = 0.5f * z * z;
            psi = z;
        } else {
            rho = c * (az - 0.5f * c);
            psi = copysignf(c, z);
        }
    } else {
        const float c = (float)o.c;
        const float q = z * z * (float)o.inv_c2;
        rho = 0.5f * c * c * log1pf(q);
        psi = z / (1.0f + q);
    }
}

// Loss l and g = dl/dM for one valid pixel (Iv = target value, M = model value).
__device__ __forceinline__ void pixel_objective(const ObjParams& o, float Iv, float M, float w, float F,
                                                float& l, float& g) {
    const float r = Iv - M;
    float rho, psi;
    if (o.var == DIA_VAR_WEIGHTS) {
        const float sw = sqrtf(w);
        rho_psi(o, r * sw, rho, psi);
        l = rho;
        g = -psi * sw;
        return;
    }
    const bool model = (o.var == DIA_VAR_CCD_MODEL || o.var == DIA_VAR_EMCCD_MODEL);
    const float X = model ? M : Iv;
    float raw, slope;
    const float floor_v = (float)o.var_floor;
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL) {
        slope = (float)o.inv_gain / F;
        raw = (float)o.s0sq / (F * F) + fmaxf(X, 0.0f) * slope;
    } else {
        slope = (float)(o.excess * o.inv_gain) / F;
        raw = fmaxf(X, 0.0f) * slope;
    }
    const float v = fmaxf(raw, floor_v);
    const float inv_s = 1.0f / sqrtf(v);
    rho_psi(o, r * inv_s, rho, psi);
    if (!model) {
        l = rho;
        g = -psi * inv_s;
    } else {
        const float dv = (X > 0.0f && raw > floor_v) ? slope : 0.0f;
        const float inv_v = inv_s * inv_s;
        l = rho + 0.5f * logf(v);
        g = -psi * inv_s * (1.0f + 0.5f * r * dv * inv_v) + 0.5f * dv * inv_v;
    }
}

// FP64 forms used by the fused pass (FP32 inputs widen exactly; the model value and the
// residual I - M are carried in FP64, so the gradient keeps FP64 accuracy).
__device__ __forceinline__ void rho_psi_d(const ObjParams& o, double z, double& rho, double& psi) {
    if (o.rho == DIA_RHO_GAUSS) {
        rho = 0.5 * z * z;
        psi = z;
    } else if (o.rho == DIA_RHO_HUBER) {
        const double c = o.c;
        const double az = fabs(z);
        if (az <= c) {
            rho = 0.5 * z * z;
            psi = z;
        } else {
            rho = c * (az - 0.5 * c);
            psi = copysign(c, z);
        }
    } else {
        const double c = o.c;
        const double q = z * z / (c * c);
        rho = 0.5 * c * c * log1p(q);
        psi = z / (1.0 + q);
    }
}

__device__ __forceinline__ void pixel_objective_d(const ObjParams& o, double Iv, double M, float w, float F,
                                                  double& l, double& g) {
    const double r = Iv - M;
    double rho, psi;
    if (o.var == DIA_VAR_WEIGHTS) {
        const double sw = sqrt((double)w);
        rho_psi_d(o, r * sw, rho, psi);
        l = rho;
        g = -psi * sw;
        return;
    }
    const bool model = (o.var == DIA_VAR_CCD_MODEL || o.var == DIA_VAR_EMCCD_MODEL);
    const double X = model ? M : Iv;
    const double Fd = (double)F;
    double raw, slope;
    // F = 1 (no flat field): the divisions by F are exact, so they are skipped
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL) {
        slope = F == 1.0f ? o.inv_gain : o.inv_gain / Fd;
        raw = (F == 1.0f ? o.s0sq : o.s0sq / (Fd * Fd)) + fmax(X, 0.0) * slope;
    } else {
        slope = F == 1.0f ? o.excess * o.inv_gain : o.excess * o.inv_gain / Fd;
        raw = fmax(X, 0.0) * slope;
    }
    const double v = fmax(raw, o.var_floor);
    const double inv_s = 1.0 / sqrt(v);
    rho_psi_d(o, r * inv_s, rho, psi);
    if (!model) {
        l = rho;
        g = -psi * inv_s;
    } else {
        const double dv = (X > 0.0 && raw > o.var_floor) ? slope : 0.0;
        const double inv_v = inv_s * inv_s;
        l = rho + 0.5 * log(v);
        g = -psi * inv_s * (1.0 + 0.5 * r * dv * inv_v) + 0.5 * dv * inv_v;
    }
}

// Per-pixel curvature h = d2l/dM2 (the Hessian of the loss is X^T diag(h) X because M is affine
// in theta).  With exact = 0 the positive form used for Newton steps is returned: the Cauchy
// curvature psi' is replaced by the IRLS weight psi(z)/z and negative values are clipped to 0.
__device__ __forceinline__ double pixel_curvature_d(const ObjParams& o, double Iv, double M, float w, float F,
                                                   bool exact) {
    const double r = Iv - M;
    auto dpsi = [&](double z) -> double {
        if (o.rho == DIA_RHO_GAUSS) return 1.0;
        const double c = o.c;
        if (o.rho == DIA_RHO_HUBER) return fabs(z) <= c ? 1.0 : 0.0;
        const double q = 1.0 + z * z / (c * c);
        return exact ? (2.0 - q) / (q * q) : 1.0 / q;
    };
    if (o.var == DIA_VAR_WEIGHTS) {
        const double sw = sqrt((double)w);
        return dpsi(r * sw) * (double)w;
    }
    const bool model = (o.var == DIA_VAR_CCD_MODEL || o.var == DIA_VAR_EMCCD_MODEL);
    const double X = model ? M : Iv;
    const double Fd = (double)F;
    double raw, slope;
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL) {
        slope = o.inv_gain / Fd;
        raw = o.s0sq / (Fd * Fd) + fmax(X, 0.0) * slope;
    } else {
        slope = o.excess * o.inv_gain / Fd;
        raw = fmax(X, 0.0) * slope;
    }
    const double v = fmax(raw, o.var_floor);
    const double sg = sqrt(v);
    const double z = r / sg;
    if (!model) return dpsi(z) / v;
    double rho, psi;
    rho_psi_d(o, z, rho, psi);
    const double dv = (X > 0.0 && raw > o.var_floor) ? slope : 0.0;
    const double z1 = -1.0 / sg - r * dv / (2.0 * v * sg);
    const double z2 = dv / (v * sg) + 0.75 * r * dv * dv / (v * v * sg);
    const double h = dpsi(z) * z1 * z1 + psi * z2 - dv * dv / (2.0 * v * v);
    return exact ? h : fmax(h, 0.0);
}

// Model variance v(M) (the CCD or EMCCD form of obj.var, evaluated on the model).
__device__ __forceinline__ float model_variance(const ObjParams& o, float M, float F) {
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL)
        return fmaxf((float)o.s0sq / (F * F) + fmaxf(M, 0.0f) * (float)o.inv_gain / F, (float)o.var_floor);
    return fmaxf((float)(o.excess * o.inv_gain) * fmaxf(M, 0.0f) / F, (float)o.var_floor);
}

// Launchers for the tiled kernels (tile_kernels.hip).  Return hipError_t.
constexpr int kNumVariants = 9;  // tile-shape variants: RB = auto, 1, 2, 4; two thread sets of RB = 1; narrow RB = 1;
                                 // two thread sets of a few strips; kernel rows split, a few strips / narrow
int tile_variant_rb(int m, int variant);               // effective RB of a variant (0 = not compiled)
int tile_variant_sets(int m, int variant);             // thread sets of a variant (0 = not compiled)
int tile_variant_threads(int m, int variant);          // threads per workgroup of a variant (0 = not compiled)
int tile_dims(int m, int variant, int* ty, int* tx);   // tile height / width of a variant
int tile_grid_tiles(int m, int rows, int cols, int variant = 0);  // tiles of the valid region
hipError_t launch_tile(int mode, int m, int grid, const TileArgs& a, hipStream_t s, int variant = 0);
hipError_t launch_batched_eval(int m, int grid, const BatchedArgs& b, hipStream_t s, int variant = 0);

// Kernel-kernel block of the Hessian, H_KK[t1][t2] = sum_p h_p R_(p+t1) R_(p+t2) (hess_impl.h).
struct HessArgs {
    const float* R;
    long long ldR;
    const double* h;   // per-pixel curvature, valid region, row stride Wv
    int rows, cols;
    double* partial;   // [splits][n_pairblocks][32]
};
constexpr int kHessBlockElems = 64 * 64;  // doubles per (split, tap-region pair) block of the Hessian partials
int hess_pair_blocks(int m);
int hess_splits(int m, int rows, int cols);
hipError_t launch_hess(int m, const HessArgs& a, hipStream_t s);
int tile_max_blocks_per_cu(int m, int variant = 0, bool batched = false);

}  // namespace dia

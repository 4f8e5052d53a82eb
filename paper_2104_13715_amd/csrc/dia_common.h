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
    float s0sq;       // sigma0^2
    float inv_gain;   // 1 / G
    float excess;     // E
    float var_floor;  // lower bound on sigma^2
    float c;          // Huber / Cauchy scale
    float inv_c2;     // 1 / c^2
    const float* weights;
    const float* flat;
    const uint8_t* mask;
};

// What one launch of the tiled kernel does with the forward result.
enum TileMode { MODE_EVAL = 0, MODE_MODEL = 1, MODE_CLIP = 2 };

struct TileArgs {
    const float* R;
    long long ldR;
    const float* I;
    long long ldI;     // also the leading dimension of weights, flat, mask, w_out, mask_out
    int rows, cols;
    const float* theta;  // K (m*m, row-major) then B0
    ObjParams obj;
    double* partial;     // MODE_EVAL: [gridDim.x][m*m + 2]: dL/dK, dL/dB0, loss
    float* out;          // MODE_MODEL: valid model
    long long ld_out;
    float* w_out;        // MODE_CLIP: 1/v(M) on the target grid
    uint8_t* mask_out;   // MODE_CLIP: updated mask on the target grid
    float kappa;         // MODE_CLIP: clip |z| > kappa (0 = keep every pixel)
    int* clip_count;     // MODE_CLIP: pixels newly clipped (integer atomics)
    const int* done;     // if non-null and *done != 0 the launch does nothing
};

// Geometry of the tiled kernel for an m x m kernel (all compile-time).
//  - backward: thread (a, cs) owns kernel row a and column strip cs (S pixels wide),
//    so m * NS threads cover the m x m taps of one tile;
//  - forward: thread (rg, cs) owns RB output rows x S output columns.
//  - tile = TY x TX outputs; the reference tile (with its m-1 halo) and the g tile live in LDS.
template <int M>
struct Geo {
    static constexpr int S = 8;
    static constexpr int NS = (256 / M) < 32 ? (256 / M) : 32;
    static constexpr int NA = M * NS;                    // active threads
    static constexpr int NT = ((NA + 63) / 64) * 64;     // launched threads (whole waves)
    static constexpr int TX = NS * S;
    static constexpr int RW = TX + M - 1;                // reference tile width
    static constexpr int RS = RW + ((RW % 2 == 0) ? 1 : 0);  // odd LDS row stride
    static constexpr int lds_bytes(int rb) { return 4 * ((M * rb + M - 1) * RS + M * rb * TX); }
    static constexpr int RB = lds_bytes(4) <= 60 * 1024 ? 4 : (lds_bytes(2) <= 60 * 1024 ? 2 : 1);
    static constexpr int TY = M * RB;
    static constexpr int RH = TY + M - 1;                // reference tile height
};

// rho(z) and psi(z) = rho'(z) for the three loss shapes.
__device__ __forceinline__ void rho_psi(const ObjParams& o, float z, float& rho, float& psi) {
    if (o.rho == DIA_RHO_GAUSS) {
        rho = 0.5f * z * z;
        psi = z;
    } else if (o.rho == DIA_RHO_HUBER) {
        const float az = fabsf(z);
        if (az <= o.c) {
            rho = 0.5f * z * z;
            psi = z;
        } else {
            rho = o.c * (az - 0.5f * o.c);
            psi = copysignf(o.c, z);
        }
    } else {
        const float q = z * z * o.inv_c2;
        rho = 0.5f * o.c * o.c * log1pf(q);
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
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL) {
        slope = o.inv_gain / F;
        raw = o.s0sq / (F * F) + fmaxf(X, 0.0f) * slope;
    } else {
        slope = o.excess * o.inv_gain / F;
        raw = fmaxf(X, 0.0f) * slope;
    }
    const float v = fmaxf(raw, o.var_floor);
    const float inv_s = 1.0f / sqrtf(v);
    rho_psi(o, r * inv_s, rho, psi);
    if (!model) {
        l = rho;
        g = -psi * inv_s;
    } else {
        const float dv = (X > 0.0f && raw > o.var_floor) ? slope : 0.0f;
        const float inv_v = inv_s * inv_s;
        l = rho + 0.5f * logf(v);
        g = -psi * inv_s * (1.0f + 0.5f * r * dv * inv_v) + 0.5f * dv * inv_v;
    }
}

// Model variance v(M) (the CCD or EMCCD form of obj.var, evaluated on the model).
__device__ __forceinline__ float model_variance(const ObjParams& o, float M, float F) {
    if (o.var == DIA_VAR_CCD_DATA || o.var == DIA_VAR_CCD_MODEL)
        return fmaxf(o.s0sq / (F * F) + fmaxf(M, 0.0f) * o.inv_gain / F, o.var_floor);
    return fmaxf(o.excess * fmaxf(M, 0.0f) * o.inv_gain / F, o.var_floor);
}

// Launchers for the tiled kernel (tile_kernels.hip).  Return hipError_t.
int tile_grid_tiles(int m, int rows, int cols);       // number of tiles of the valid region
int tile_block_threads(int m);
hipError_t launch_tile(int mode, int m, int grid, const TileArgs& a, hipStream_t s);
int tile_max_blocks_per_cu(int m);

}  // namespace dia

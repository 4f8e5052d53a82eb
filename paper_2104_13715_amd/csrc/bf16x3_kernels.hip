// Batched split-precision (bf16 x 3) implicit-GEMM evaluation on gfx950 matrix cores.
//
// All epochs read the same reference window, so the forward pass of a block of 32 epochs is
// one GEMM  M[32 epochs x pixels] = K[32 x taps] . X[taps x pixels]  and the backward pass is
// dK[32 x taps] = G[32 x pixels] . X^T  with X = im2col(R) gathered from an LDS tile and never
// stored.  Both run on v_mfma_f32_32x32x16_bf16 with every operand split into bf16 hi + lo
// parts (products hi*hi + hi*lo + lo*hi: about 16 significant bits per operand, 2^-17 relative
// representation error).  MFMA accumulates one tile in FP32; tile results are added in FP64.
//
// Workgroup = 8 waves, one block of 32 epochs, a contiguous range of 8 x 64 pixel tiles.
//   * K of the block (hi / lo) is laid out in LDS in MFMA A-fragment order once per launch.
//   * Per tile the reference window (with its m-1 halo) is staged as packed (hi << 16 | lo)
//     words.  Forward: wave w forms row w of the tile (two blocks of 32 pixels, 32 words apart,
//     so a lane's paired read touches disjoint banks) for all 32 epochs; the B fragment of a
//     lane is 8 taps of one pixel, read with compile-time offsets.  The per-pixel objective
//     (FP32 with hardware reciprocal / log; the same formulas as the fused pass) gives g, split
//     into hi / lo bf16 in LDS.
//   * Backward: the flattened taps are cut into blocks of 32; wave w owns blocks w, w+8, ...; a
//     K step is 16 pixels of one tile row.  dL/dB0 = sum of g is added up in the objective phase.
// The lane layouts used (gfx950, 32x32x16): A lane l holds A[l % 32][8 (l / 32) + j],
// B lane l holds B[8 (l / 32) + j][l % 32], D lane l register r holds
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
#include <algorithm>
#include <type_traits>
#include <vector>

#include "api_util.h"
#include "bf16x3.h"

namespace dia {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kEB = kBf16x3Block;  // epochs per block
constexpr int kWaves = 8;
constexpr int kTR = kWaves;         // tile rows (one per wave in the forward pass)
constexpr int kTC = 64;             // tile columns (two MFMA blocks of 32)
constexpr int kThreads = 64 * kWaves;
static_assert(kTR * kTC == 8 * 64, "a wave covers the tile with eight 64-pixel groups (in pairs) in the objective phase");
constexpr int kTargetGroups = 256;  // workgroups per launch: one per CU on MI355X

template <int M>
struct BfGeo {
    static constexpr int T = M * M;
    static constexpr int TP = (T + 31) / 32 * 32;      // taps in blocks of 32 (padding taps: K = 0)
    static constexpr int NCH = TP / 16;                // forward K steps (16 taps)
    static constexpr int NTB = TP / 32;                // backward tap blocks
    static constexpr int TBW = (NTB + kWaves - 1) / kWaves;
    static constexpr int RH = kTR + M - 1;             // staged reference rows
    static constexpr int RW = kTC + M - 1 + 8;         // staged columns (+8: padded-tap reads stay inside)
    static constexpr int RS = RW | 1;                  // row stride (words)
    static_assert(kTC == 64, "the two forward column blocks are 32 words apart: disjoint LDS banks");
    static constexpr int PT = kTR * kTC;               // pixels per tile (= threads per workgroup)
    static constexpr int HALF = (M - 1) / 2;
    // forward gather with compile-time offsets: lanes of half 0 read tap t0 = 16 c + j, lanes of
    // half 1 tap t0 + 8; their addresses differ by 8 + delta * (RS - M) words (delta = 1 when the
    // two taps sit in different kernel rows), so each half keeps two base pointers and every
    // offset is an immediate.  Padding taps (t >= T) read an arbitrary staged word (their K is 0).
    __host__ __device__ __attribute__((always_inline)) static constexpr int off(int c, int j) {
        const int t0 = 16 * c + j;
        return t0 < T ? (t0 / M) * RS + t0 % M : 0;
    }
    __host__ __device__ __attribute__((always_inline)) static constexpr int delta(int c, int j) {
        const int t0 = 16 * c + j, t1 = t0 + 8;
        return (t0 < T && t1 < T) ? (t1 / M - t0 / M) : 0;
    }
};

__device__ __forceinline__ unsigned split_pack(float x) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    return ((unsigned)__builtin_bit_cast(unsigned short, h) << 16) | __builtin_bit_cast(unsigned short, l);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// two values split at once: hi = (hi(a) | hi(b) << 16), lo likewise (round to nearest even)
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
    const f32x2 v = {a, b};
    hi = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
    const f32x2 h = {__builtin_bit_cast(float, hi << 16), __builtin_bit_cast(float, hi & 0xFFFF0000u)};
    lo = __builtin_bit_cast(unsigned, __builtin_convertvector(v - h, bf16x2));
}

// 8 packed (hi << 16 | lo) words -> the hi and lo bf16 fragments, one byte permute per dword:
// hi dword k = upper halves of words 2k, 2k+1; lo dword k = their lower halves
__device__ __forceinline__ void unpack8(const unsigned (&w)[8], bf16x8& hi, bf16x8& lo) {
    u32x4 h, l;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        h[k] = __builtin_amdgcn_perm(w[2 * k + 1], w[2 * k], 0x07060302u);
        l[k] = __builtin_amdgcn_perm(w[2 * k + 1], w[2 * k], 0x05040100u);
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}

__device__ __forceinline__ f32x16 mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                                        f32x16 c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, c, 0, 0, 0);
    return c;
}

// The per-pixel objective of the split-precision path in FP32 with the hardware reciprocal,
// reciprocal square root and logarithm (about 1 ulp each: far below the 2^-17 split of g).
// Same formulas as the fused pass; Gaussian with fixed variance needs no square root at all.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718056f; }
__device__ __forceinline__ float fast_ln1p(float q) {
    // series where 1 + q would round away the information, hardware log2 elsewhere
    return q < 1e-3f ? q * (1.0f - q * (0.5f - q * (1.0f / 3.0f))) : fast_ln(1.0f + q);
}

template <int RHO>
__device__ __forceinline__ void rho_psi_fast(const ObjParams& o, float z, float& rho, float& psi) {
    if constexpr (RHO == DIA_RHO_GAUSS) {
        rho = 0.5f * z * z;
        psi = z;
    } else if constexpr (RHO == DIA_RHO_HUBER) {
        const float c = (float)o.c, az = fabsf(z);
        const bool in = az <= c;
        rho = in ? 0.5f * z * z : c * (az - 0.5f * c);
        psi = in ? z : copysignf(c, z);
    } else {
        const float c = (float)o.c;
        const float q = z * z * (float)o.inv_c2;
        rho = 0.5f * c * c * fast_ln1p(q);
        psi = z * fast_rcp(1.0f + q);
    }
}

// l and g = dl/dM of one pixel (r = I - M), the mode fixed at compile time; HAS_F = false
// means no flat field (F = 1), which drops a reciprocal and three products from the variance.
template <int RHO, int VAR, bool HAS_F>
__device__ __forceinline__ void pixel_objective_fast(const ObjParams& o, float Iv, float M, float w, float F, float& l,
                                                     float& g) {
    const float r = Iv - M;
    float rho, psi;
    if constexpr (VAR == DIA_VAR_WEIGHTS) {
        if constexpr (RHO == DIA_RHO_GAUSS) {
            const float t = r * w;
            l = 0.5f * r * t;
            g = -t;
        } else {
            const float sw = __builtin_amdgcn_sqrtf(w);
            rho_psi_fast<RHO>(o, r * sw, rho, psi);
            l = rho;
            g = -psi * sw;
        }
    } else {
        constexpr bool model = (VAR == DIA_VAR_CCD_MODEL || VAR == DIA_VAR_EMCCD_MODEL);
        constexpr bool ccd = (VAR == DIA_VAR_CCD_DATA || VAR == DIA_VAR_CCD_MODEL);
        const float X = model ? M : Iv;
        const float floor_v = (float)o.var_floor;
        float raw, slope;
        if constexpr (HAS_F) {
            const float iF = fast_rcp(F);
            slope = (float)(ccd ? o.inv_gain : o.excess * o.inv_gain) * iF;
            raw = ccd ? (float)o.s0sq * iF * iF + fmaxf(X, 0.0f) * slope : fmaxf(X, 0.0f) * slope;
        } else {
            slope = (float)(ccd ? o.inv_gain : o.excess * o.inv_gain);
            raw = ccd ? fmaf(fmaxf(X, 0.0f), slope, (float)o.s0sq) : fmaxf(X, 0.0f) * slope;
        }
        const float v = fmaxf(raw, floor_v);
        if constexpr (!model && RHO == DIA_RHO_GAUSS) {
            const float t = r * fast_rcp(v);
            l = 0.5f * r * t;
            g = -t;
        } else {
            const float inv_s = fast_rsq(v);
            rho_psi_fast<RHO>(o, r * inv_s, rho, psi);
            if constexpr (!model) {
                l = rho;
                g = -psi * inv_s;
            } else {
                const float dv = (X > 0.0f && raw > floor_v) ? slope : 0.0f;
                const float inv_v = inv_s * inv_s;
                l = rho + 0.5f * fast_ln(v);
                g = -psi * inv_s * (1.0f + 0.5f * r * dv * inv_v) + 0.5f * dv * inv_v;
            }
        }
    }
}

// calls f(integral_constant<RHO>, integral_constant<VAR>, integral_constant<HAS_F>) for the
// objective's run-time mode (the weights mode never reads a flat field)
template <int RHO, int VAR, class Fn>
__device__ __forceinline__ void with_flat(bool has_f, Fn&& f) {
    using R = std::integral_constant<int, RHO>;
    using V = std::integral_constant<int, VAR>;
    if (VAR != DIA_VAR_WEIGHTS && has_f)
        f(R{}, V{}, std::integral_constant<bool, VAR != DIA_VAR_WEIGHTS>{});
    else
        f(R{}, V{}, std::false_type{});
}
template <int RHO, class Fn>
__device__ __forceinline__ void with_var(int var, bool has_f, Fn&& f) {
    switch (var) {
        case DIA_VAR_WEIGHTS: with_flat<RHO, DIA_VAR_WEIGHTS>(has_f, f); break;
        case DIA_VAR_CCD_DATA: with_flat<RHO, DIA_VAR_CCD_DATA>(has_f, f); break;
        case DIA_VAR_CCD_MODEL: with_flat<RHO, DIA_VAR_CCD_MODEL>(has_f, f); break;
        case DIA_VAR_EMCCD_DATA: with_flat<RHO, DIA_VAR_EMCCD_DATA>(has_f, f); break;
        default: with_flat<RHO, DIA_VAR_EMCCD_MODEL>(has_f, f); break;
    }
}
template <class Fn>
__device__ __forceinline__ void with_mode(const ObjParams& o, bool has_f, Fn&& f) {
    switch (o.rho) {
        case DIA_RHO_GAUSS: with_var<DIA_RHO_GAUSS>(o.var, has_f, f); break;
        case DIA_RHO_HUBER: with_var<DIA_RHO_HUBER>(o.var, has_f, f); break;
        default: with_var<DIA_RHO_CAUCHY>(o.var, has_f, f); break;
    }
}

// A value that is the same in every lane, read from LDS, moved into scalar registers: the
// compiler then branches on it with the scalar unit and addresses memory as scalar base +
// per-lane offset instead of 64-bit vector arithmetic per epoch.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
// Raw buffer view of the bytes from a (wave-uniform) base on: a load is then the scalar
// descriptor + one 32-bit per-lane byte offset, with no 64-bit address arithmetic per lane.
// Callers keep their offsets inside the array they address.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_view(const char* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ float view_f32(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ unsigned view_u8(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
}
__device__ __forceinline__ float uniform_f(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(unsigned, x)));
}

// Sum of a double over the 64 lanes of a wave (the same value in every lane): DPP exchanges
// inside each row of 16 lanes (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror 4, row_ror 8)
// leave every lane with its row's sum; the four row sums are read out and added.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x124>(v);
    v += dpp_f64<0x128>(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

template <int M>
struct BfSmem {
    using G = BfGeo<M>;
    alignas(16) unsigned short Khi[G::NCH * 2 * kEB * 8];
    alignas(16) unsigned short Klo[G::NCH * 2 * kEB * 8];
    alignas(16) unsigned Rw[G::RH * G::RS];
    // forward results M[epoch][pixel] (float), then g as hi / lo bf16 planes in each epoch's slot
    alignas(16) unsigned short Gt[2 * kEB * G::PT];
    const float* Ip[kEB];
    const float* Wp[kEB];
    const float* Fp[kEB];
    const uint8_t* Mp[kEB];
    float B0[kEB];
    double lsum[kEB];          // FP64 loss of each epoch (added to by the wave that owns it)
    double gsum[kEB];          // FP64 dL/dB0 = sum of g of each epoch (likewise)
};

// g planes: epoch e owns the 4 * pt bytes that held its forward results: hi plane, then lo plane.
// 8-pixel groups are permuted by (e mod 16) so that the 16 lanes served together by a backward
// A-fragment read (one epoch each, the same 8 pixels, 16 bytes per lane) cover all 64 banks.
__device__ __forceinline__ int ghi(int e, int p, int pt) { return 2 * e * pt + (p ^ ((e & 15) << 3)); }
__device__ __forceinline__ int glo(int e, int p, int pt) { return 2 * e * pt + pt + (p ^ ((e & 15) << 3)); }

template <int M>
__global__ __launch_bounds__(kThreads) void bf16x3_eval_kernel(Bf16x3Args g) {
    using G = BfGeo<M>;
    __shared__ BfSmem<M> sm;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l32 = lane & 31, q = lane >> 5;
    const int wi = blockIdx.x;
    if (g.done != nullptr) {  // a fit: nothing to do once every epoch of the block has converged
        __shared__ int live;
        if (threadIdx.x == 0) live = 0;
        __syncthreads();
        const int eg = threadIdx.x < kEB ? g.ep[threadIdx.x] : -1;
        if (eg >= 0 &&
            *reinterpret_cast<const int*>(reinterpret_cast<const char*>(g.done) + eg * g.done_stride) == 0)
            live = 1;
        __syncthreads();
        if (live == 0) return;
    }
    const int Hv = g.rows - M + 1, Wv = g.cols - M + 1;
    const int ntx = (Wv + kTC - 1) / kTC, nty = (Hv + kTR - 1) / kTR, ntiles = ntx * nty;
    const int t_begin = (int)((long long)ntiles * wi / g.wpb), t_end = (int)((long long)ntiles * (wi + 1) / g.wpb);

    // K of this block in A-fragment order: (step c, half q, epoch e, j) <- tap 16 c + 8 q + j
    for (int idx = tid; idx < kEB * G::TP; idx += kThreads) {
        const int e = idx / G::TP, t = idx - e * G::TP;
        const int eg = g.ep[e];
        float v = 0.0f;
        if (eg >= 0 && t < G::T)
            v = reinterpret_cast<const float*>(reinterpret_cast<const char*>(g.theta0) + eg * g.theta_stride)[t];
        const unsigned p = split_pack(v);
        const int c = t >> 4, qq = (t >> 3) & 1, j = t & 7;
        const int at = ((c * 2 + qq) * kEB + e) * 8 + j;
        sm.Khi[at] = (unsigned short)(p >> 16);
        sm.Klo[at] = (unsigned short)(p & 0xFFFFu);
    }
    if (tid < kEB) {
        const int eg = g.ep[tid];
        const bool ok = eg >= 0;
        sm.B0[tid] = ok ? reinterpret_cast<const float*>(reinterpret_cast<const char*>(g.theta0) + eg * g.theta_stride)[G::T]
                        : 0.0f;
        sm.Ip[tid] = ok ? g.I[tid] : nullptr;
        sm.Wp[tid] = ok ? g.W[tid] : nullptr;
        sm.Fp[tid] = ok ? g.F[tid] : nullptr;
        sm.Mp[tid] = ok ? g.Mk[tid] : nullptr;
    }

    // backward B-fragment base of each owned tap block: tap n = 32 tb + l32 (clamped inside the tap range)
    const int nblk = (G::NTB - __builtin_amdgcn_readfirstlane(w) + kWaves - 1) / kWaves;  // TBW or TBW - 1
    int nb_off[G::TBW];
#pragma unroll
    for (int i = 0; i < G::TBW; ++i) {
        const int n = (w + kWaves * i) * 32 + l32;
        const int nc = n < G::T ? n : 0;
        nb_off[i] = (nc / M) * G::RS + nc % M + 8 * q;
    }

    double dk64[G::TBW][16];
#pragma unroll
    for (int i = 0; i < G::TBW; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) dk64[i][r] = 0.0;
    if (tid < kEB) sm.lsum[tid] = sm.gsum[tid] = 0.0;

    float* Ms = reinterpret_cast<float*>(sm.Gt);
    unsigned short* Ghi = sm.Gt;  // both planes, indexed by ghi() / glo()

    // The reference window of a tile (RH x RW words; this thread's are words tid + k * kThreads)
    // is fetched into registers one tile ahead, while the previous tile's backward pass runs, and
    // written to LDS at the top of the tile.  Words outside the reference read its last row /
    // column (always inside) and are replaced by zero.
    constexpr int SPT = (G::RH * G::RW + kThreads - 1) / kThreads;
    float rpre[SPT];
    auto fetch_R = [&](int t) {
        const int ty0 = (t / ntx) * kTR, tx0 = (t % ntx) * kTC;
        const char* Rb = uniform_ptr(reinterpret_cast<const char*>(g.R + (long long)ty0 * g.ldR + tx0));
        const int rmax = min(g.rows - 1 - ty0, G::RH - 1), cmax = min(g.cols - 1 - tx0, G::RW - 1);
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int idx = tid + k * kThreads;
            const int r = idx / G::RW, c = idx - r * G::RW;
            const float v = view_f32(raw_view(Rb), (unsigned)(min(r, rmax) * g.ldR + min(c, cmax)) * 4u);
            rpre[k] = (r <= rmax && c <= cmax) ? v : 0.0f;
        }
    };
    if (t_begin < t_end) fetch_R(t_begin);

    for (int t = t_begin; t < t_end; ++t) {
        const int ty0 = (t / ntx) * kTR, tx0 = (t % ntx) * kTC;
        // keep the per-epoch tables in LDS (not hoisted into registers across tiles)
        asm volatile("" ::: "memory");
        __syncthreads();  // previous tile's readers are done (and, first time, the tables are visible)
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int idx = tid + k * kThreads;
            const int r = idx / G::RW, c = idx - r * G::RW;
            if (idx < G::RH * G::RW) sm.Rw[r * G::RS + c] = split_pack(rpre[k]);
        }
        __syncthreads();

        // objective set-up, ahead of the forward pass so that the wave's first target loads are in
        // flight during it.  Lane l, group i is pixel (row i, column l) of the tile; its byte
        // offset from the tile's first pixel is the same in every epoch (lanes past a ragged edge
        // read the nearest pixel inside and contribute zero).  Target values (and B0) are fetched
        // one epoch ahead (epochs past the batch read epoch 0 and count nothing).
        constexpr int NG = G::PT / 64;
        unsigned ob[NG];
        unsigned vmask = 0u;
        {
            const int x = tx0 + lane, xc = min(x, Wv - 1) - tx0;
#pragma unroll
            for (int i = 0; i < NG; ++i) {
                const int y = ty0 + i, yc = min(y, Hv - 1) - ty0;
                vmask |= (y < Hv && x < Wv) ? (1u << i) : 0u;
                ob[i] = (unsigned)(yc * g.ldI + xc) * 4u;
            }
        }
        const long long tile0 = (long long)(ty0 + G::HALF) * g.ldI + (tx0 + G::HALF);
        float inext[NG], b0_next;
        bool live_next;
        auto fetch_I = [&](int k) {
            const int e = w + kWaves * k;
            const float* Ie = uniform_ptr(sm.Ip[e]);
            live_next = Ie != nullptr;
            b0_next = uniform_f(sm.B0[e]);
            const char* Ib = uniform_ptr(reinterpret_cast<const char*>((Ie ? Ie : uniform_ptr(sm.Ip[0])) + tile0));
#pragma unroll
            for (int i = 0; i < NG; ++i) inext[i] = view_f32(raw_view(Ib), ob[i]);
        };
        fetch_I(0);

        // forward: row w of the tile, pixels l32 and 32 + l32, all 32 epochs
        {
            f32x16 acc0, acc1;
#pragma unroll
            for (int r = 0; r < 16; ++r) acc0[r] = acc1[r] = 0.0f;
            const unsigned* p0 = sm.Rw + w * G::RS + l32 + (q ? 8 : 0);
            const unsigned* p1 = p0 + (q ? G::RS - M : 0);
#pragma unroll
            for (int c = 0; c < G::NCH; ++c) {
                const bf16x8 ah = *reinterpret_cast<const bf16x8*>(sm.Khi + ((c * 2 + q) * kEB + l32) * 8);
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(sm.Klo + ((c * 2 + q) * kEB + l32) * 8);
                unsigned wv0[8], wv1[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const unsigned* pj = (G::delta(c, j) ? p1 : p0) + G::off(c, j);
                    wv0[j] = pj[0];
                    wv1[j] = pj[32];
                }
                bf16x8 bh, bl;
                unpack8(wv0, bh, bl);
                acc0 = mfma3(ah, al, bh, bl, acc0);
                unpack8(wv1, bh, bl);
                acc1 = mfma3(ah, al, bh, bl, acc1);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int el = 8 * (r >> 2) + 4 * q + (r & 3);
                Ms[el * G::PT + w * kTC + l32] = acc0[r];
                Ms[el * G::PT + w * kTC + 32 + l32] = acc1[r];
            }
        }
        __syncthreads();

        // per-pixel objective (FP32).  Wave w owns epochs w, w + 8, w + 16, w + 24: it takes an
        // epoch's 512 forward results into registers, requests the epoch's weight / flat / mask
        // values (if any) before it uses any, and writes g as hi / lo bf16 planes into the slot the
        // forward results held (only this wave touches that slot, and its LDS reads precede its
        // writes).
        {
            with_mode(g.obj, g.has_f != 0, [&](auto rho_c, auto var_c, auto flat_c) {
                constexpr int RHO = decltype(rho_c)::value, VAR = decltype(var_c)::value;
                constexpr bool HAS_F = decltype(flat_c)::value;
#pragma unroll 1
                for (int k = 0; k < kEB / kWaves; ++k) {
                    const int e = w + kWaves * k;
                    const bool live = live_next;
                    const float B0 = b0_next;
                    float iv[NG], wv[NG], fv[NG], mv[NG];
                    bool ok[NG];
#pragma unroll
                    for (int i = 0; i < NG; ++i) ok[i] = live && ((vmask >> i) & 1u);
#pragma unroll
                    for (int i = 0; i < NG; ++i) iv[i] = inext[i];
                    if (k + 1 < kEB / kWaves) fetch_I(k + 1);
                    const float* We = (live && g.has_w) ? uniform_ptr(sm.Wp[e]) : nullptr;
                    if (We) {
                        const char* Wb = uniform_ptr(reinterpret_cast<const char*>(We + tile0));
#pragma unroll
                        for (int i = 0; i < NG; ++i) wv[i] = view_f32(raw_view(Wb), ob[i]);
                    } else {
#pragma unroll
                        for (int i = 0; i < NG; ++i) wv[i] = 1.0f;
                    }
                    const float* Fe = (HAS_F && live) ? uniform_ptr(sm.Fp[e]) : nullptr;
                    if (Fe) {
                        const char* Fb = uniform_ptr(reinterpret_cast<const char*>(Fe + tile0));
#pragma unroll
                        for (int i = 0; i < NG; ++i) fv[i] = view_f32(raw_view(Fb), ob[i]);
                    } else {
#pragma unroll
                        for (int i = 0; i < NG; ++i) fv[i] = 1.0f;
                    }
                    const uint8_t* Me = (live && g.has_m) ? uniform_ptr(sm.Mp[e]) : nullptr;
                    if (Me) {
                        const char* Mb = uniform_ptr(reinterpret_cast<const char*>(Me + tile0));
#pragma unroll
                        for (int i = 0; i < NG; ++i)
                            ok[i] = ok[i] & (view_u8(raw_view(Mb), ob[i] >> 2) != 0);  // offsets always inside
                    }
#pragma unroll
                    for (int i = 0; i < NG; ++i) mv[i] = Ms[e * G::PT + 64 * i + lane];
                    // ghi(e, 64 i + lane): the permutation flips bit 6 of the pixel index (the
                    // group's parity) when (e mod 16) >= 8, so even and odd groups get their own base
                    const int rot = (e & 15) << 3, flip = rot >> 6;
                    unsigned short* hb = Ghi + 2 * e * G::PT + (lane ^ (rot & 63));
                    unsigned short* hb_even = hb + 64 * flip;
                    unsigned short* hb_odd = hb - 64 * flip;
                    float lsum = 0.0f, gsum = 0.0f;
#pragma unroll
                    for (int i = 0; i < NG; i += 2) {
                        float l0, g0, l1, g1;
                        pixel_objective_fast<RHO, VAR, HAS_F>(g.obj, iv[i], mv[i] + B0, wv[i], fv[i], l0, g0);
                        pixel_objective_fast<RHO, VAR, HAS_F>(g.obj, iv[i + 1], mv[i + 1] + B0, wv[i + 1], fv[i + 1],
                                                              l1, g1);
                        lsum += ok[i] ? l0 : 0.0f;
                        lsum += ok[i + 1] ? l1 : 0.0f;
                        g0 = ok[i] ? g0 : 0.0f;
                        g1 = ok[i + 1] ? g1 : 0.0f;
                        gsum += g0 + g1;
                        unsigned hi, lo;
                        split2(g0, g1, hi, lo);
                        unsigned short* h0 = hb_even + 64 * i;
                        unsigned short* h1 = hb_odd + 64 * (i + 1);
                        h0[0] = (unsigned short)hi;
                        h0[G::PT] = (unsigned short)lo;
                        h1[0] = (unsigned short)(hi >> 16);
                        h1[G::PT] = (unsigned short)(lo >> 16);
                    }
                    const double dl = wave_sum_f64((double)lsum), dg = wave_sum_f64((double)gsum);
                    if (lane == 0) {
                        sm.lsum[e] += dl;
                        sm.gsum[e] += dg;
                    }
                }
            });
        }
        __syncthreads();

        if (t + 1 < t_end) fetch_R(t + 1);

        // backward: dK[32 epochs x 32 taps] per owned tap block, K steps of 16 pixels.  The number
        // of blocks a wave owns (TBW or TBW - 1) is wave-uniform and fixed at compile time in each
        // instance, so the step loop has no branches.  Padding taps (n >= T) read a valid word;
        // their columns are discarded.
        {
            auto backward = [&](auto nb_c) {
                constexpr int NB = decltype(nb_c)::value;
                f32x16 accb[NB];
#pragma unroll
                for (int i = 0; i < NB; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r) accb[i][r] = 0.0f;
#pragma unroll 2
                for (int s = 0; s < G::PT / 16; ++s) {
                    const int pofs = s * 16 + 8 * q;  // first pixel of this lane's 8 (tile row s / 4)
                    const bf16x8 ah = *reinterpret_cast<const bf16x8*>(Ghi + ghi(l32, pofs, G::PT));
                    const bf16x8 al = *reinterpret_cast<const bf16x8*>(Ghi + glo(l32, pofs, G::PT));
                    const int rofs = (s >> 2) * G::RS + (s & 3) * 16;
                    unsigned wv[NB][8];
#pragma unroll
                    for (int i = 0; i < NB; ++i)
#pragma unroll
                        for (int j = 0; j < 8; ++j) wv[i][j] = sm.Rw[nb_off[i] + rofs + j];
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        bf16x8 bh, bl;
                        unpack8(wv[i], bh, bl);
                        accb[i] = mfma3(ah, al, bh, bl, accb[i]);
                    }
                }
#pragma unroll
                for (int i = 0; i < NB; ++i)
#pragma unroll
                    for (int r = 0; r < 16; ++r) dk64[i][r] += (double)accb[i][r];
            };
            if (nblk == G::TBW) {
                backward(std::integral_constant<int, G::TBW>{});
            } else if constexpr (G::TBW > 1) {
                backward(std::integral_constant<int, G::TBW - 1>{});
            }
        }
    }

    // partial rows: [dK (m*m), dB0, loss] of (epoch, workgroup)
    const int npp = G::T + 2;
#pragma unroll
    for (int i = 0; i < G::TBW; ++i) {
        const int n = (w + kWaves * i) * 32 + l32;
        if (i < nblk && n < G::T) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int eg = g.ep[8 * (r >> 2) + 4 * q + (r & 3)];
                if (eg >= 0) g.partial[((long long)eg * g.wpb + wi) * npp + n] = dk64[i][r];
            }
        }
    }
    __syncthreads();
    if (tid < kEB) {
        const int eg = g.ep[tid];
        if (eg >= 0) {
            g.partial[((long long)eg * g.wpb + wi) * npp + G::T] = sm.gsum[tid];
            g.partial[((long long)eg * g.wpb + wi) * npp + G::T + 1] = sm.lsum[tid];
        }
    }
}

// workgroups per launch (one launch per block of 32 epochs): one per CU, or one per tile when
// there are fewer tiles
int wpb_for(int m, int rows, int cols) {
    const long long ntiles = (long long)((rows - m + 1 + kTR - 1) / kTR) * ((cols - m + 1 + kTC - 1) / kTC);
    return (int)std::max<long long>(std::min<long long>(kTargetGroups, ntiles), 1);
}

template <int M>
hipError_t launch_m(const std::vector<Bf16x3Args>& blocks, hipStream_t s) {
    for (const Bf16x3Args& g : blocks) {
        hipLaunchKernelGGL(bf16x3_eval_kernel<M>, dim3(g.wpb), dim3(kThreads), 0, s, g);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool bf16x3_supported(int m) { return m == 9 || m == 17 || m == 19 || m == 25; }

int bf16x3_partial_rows(int m, int rows, int cols, int n_ep) {
    if (!bf16x3_supported(m) || rows < m || cols < m || n_ep < 1) return n_ep > 0 ? n_ep : 1;
    return n_ep * wpb_for(m, rows, cols);
}

int bf16x3_check_epoch(const dia_epoch& first, const dia_epoch& x, int m) {
    if (!bf16x3_supported(m)) return DIA_E_ARG;
    // per-pixel byte offsets inside a tile (8 rows) are 32-bit
    if ((long long)x.ld * 4 * (kTR + 1) >= (1LL << 32)) return DIA_E_SIZE;
    if (x.rows != first.rows || x.cols != first.cols || x.ld != first.ld) return DIA_E_SIZE;
    if (x.ref_row0 != first.ref_row0 || x.ref_col0 != first.ref_col0) return DIA_E_SIZE;
    return DIA_OK;
}

int bf16x3_prepare(const dia_image& R, const dia_epoch* ep, int n, int m, const dia_objective& obj,
                   const float* theta0, long long theta_stride, double* partial, std::vector<Bf16x3Args>* out,
                   const int* done, long long done_stride, const std::vector<int>* live) {
    // byte offsets of a staged reference window (kTR + m - 1 rows) are 32-bit
    if ((long long)R.ld * 4 * (kTR + m) >= (1LL << 32)) return DIA_E_SIZE;
    Bf16x3Args g;
    std::memset(&g, 0, sizeof(g));
    g.R = R.data + (long long)ep[0].ref_row0 * R.ld + ep[0].ref_col0;
    g.ldR = R.ld;
    g.rows = ep[0].rows;
    g.cols = ep[0].cols;
    g.m = m;
    g.n_ep = n;
    for (int e = 0; e < n; ++e) {
        g.has_w |= ep[e].weights != nullptr;
        g.has_f |= ep[e].flat != nullptr;
        g.has_m |= ep[e].mask != nullptr;
    }
    g.ldI = ep[0].ld;
    g.theta0 = theta0;
    g.theta_stride = theta_stride;
    g.obj = to_params(obj);
    g.obj.weights = nullptr;
    g.obj.flat = nullptr;
    g.obj.mask = nullptr;
    g.partial = partial;
    g.wpb = wpb_for(m, g.rows, g.cols);
    g.done = done;
    g.done_stride = done_stride;
    out->clear();
    const int nl = live ? (int)live->size() : n;
    for (int b0 = 0; b0 < nl; b0 += kEB) {
        for (int k = 0; k < kEB; ++k) {
            const int e = b0 + k < nl ? (live ? (*live)[b0 + k] : b0 + k) : -1;
            if (e >= n) return DIA_E_ARG;
            const bool in = e >= 0;
            g.ep[k] = e;
            g.I[k] = in ? ep[e].I : nullptr;
            g.W[k] = in ? ep[e].weights : nullptr;
            g.F[k] = in ? ep[e].flat : nullptr;
            g.Mk[k] = in ? ep[e].mask : nullptr;
        }
        out->push_back(g);
    }
    return DIA_OK;
}

hipError_t bf16x3_launch_eval(const std::vector<Bf16x3Args>& blocks, hipStream_t s) {
    if (blocks.empty()) return hipErrorInvalidValue;
    switch (blocks[0].m) {
        case 9: return launch_m<9>(blocks, s);
        case 17: return launch_m<17>(blocks, s);
        case 19: return launch_m<19>(blocks, s);
        case 25: return launch_m<25>(blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dia

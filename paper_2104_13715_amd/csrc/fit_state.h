// Device-side optimiser state of one fit and the kernels that drive it.
#pragma once

#include "dia_common.h"

namespace dia {

constexpr int kMaxHistory = 32;
constexpr int kReduceThreads = 256;
constexpr int kReduceCols = 16;    // partial columns per reduce workgroup
constexpr int kReducePhases = 16;  // row phases per column
static_assert(kReduceCols * kReducePhases == kReduceThreads, "reduce workgroup shape");

enum FitPhase { PH_INIT = 0, PH_ADAM = 1, PH_LSEARCH = 2, PH_DONE = 3 };
enum StopReason { STOP_NONE = 0, STOP_CHANGE = 1, STOP_GRAD = 2, STOP_LINESEARCH = 3, STOP_CAP = 4, STOP_NEWTON = 5 };

struct FitOptsDev {
    double lr_K, lr_B0, beta1, beta2, eps;
    double tol_switch, tol_change, tol_grad;
    int history, max_adam, max_lbfgs, max_eval;
    int skip_adam;  // warm restart: go straight to L-BFGS with the kept curvature pairs
};

// Lives in the workspace; read back by the host after a fit.
struct FitState {
    int phase, done, status, stop;
    int n_eval, n_adam, n_lbfgs, ls_iter;
    int hist_n, hist_head, adam_t;
    int small_steps;  // consecutive accepted L-BFGS steps with relative change below tol_change
    int nk, n;        // kernel taps (m*m; the scalar background or b_00 sits at index nk) and parameters
    double L;        // loss at the current point (Adam) or the accepted point (L-BFGS)
    double alpha;    // line-search step
    double gtd;      // g . d at the accepted point
    double gmax0;    // max |grad| at the first evaluation
    double out_loss, out_P, out_B0;
    double ref_shift;  // s: mean of the reference
    double ref_scale;  // c: RMS of (reference - s)
    double pad[3];
};

// Pointers into the workspace for one fit (n = m*m + nb parameters: the kernel, then the background).
struct FitVecs {
    double *x, *g, *d, *xt, *m1, *v1, *xp, *gp;
    double *S, *Y, *rh, *al;  // L-BFGS history: S[kMaxHistory][ld], Y[kMaxHistory][ld]
    float* theta_eval;        // float copy of the point being evaluated (read by the tile kernel)
    double* theta_eval64;     // the same values widened to FP64 (the fused pass reads these)
    int ld;                   // padded vector length
};

constexpr int kStatBlocks = 64;

// Radix-select state for the two middle ranks of the median, and the per-block partial sums
// of the reference statistics (sum and sum of squares).
struct SelectState {
    unsigned prefix[2], mask[2];
    long long k[2];
    unsigned hist[2][256];
    double stat_part[2 * kStatBlocks];
    long long stat_n;
};

struct ReduceArgs {
    const double* partial;  // [nblk][npp]
    int nblk, npp;          // npp = n + 1 (gradient, then loss)
    double* gt;             // reduced gradient and loss (FP64)
    double* out_loss;       // loss-grad mode: device double[1]
    float* out_grad;        // loss-grad mode: device float[n]
    double* out_grad64;     // loss-grad mode: device double[n] (the FP64 entry point)
    FitState* st;           // fit mode when non-null
    FitVecs v;
    FitOptsDev o;
    int n, m;
    const int* done;
    int* n_done;            // incremented once when the fit finishes (batched polling)
    double reg;             // lambda N_data of the kernel-smoothness penalty (0 = none)
    const double* th64;     // the FP64 parameters the pass evaluated (read when reg > 0)
    int lds_hist;           // step kernel: its dynamic LDS holds a copy of the L-BFGS history (step_lds_bytes)
};

// Batched fits: epoch e's FitState, SelectState, vectors and theta_eval sit at byte offset
// e * stride from the epoch-0 pointers.
struct BatchReduceArgs {
    const double* partial;  // [n_chunks][npp]
    const int* cbeg;        // chunk rows of epoch e: [cbeg[e], cend[e]), or, when cbeg is null,
    const int* cend;        // [e * rows_per, (e + 1) * rows_per)
    int rows_per;
    int npp;
    double* gt;             // [n_epochs][npp]
    double* out_loss;       // loss-grad mode: [n_epochs]
    float* out_grad;        // loss-grad mode: [n_epochs][n]
    FitState* st;           // fit mode when non-null
    FitVecs v;
    long long stride;
    FitOptsDev o;
    int n, m;
    int* queue;             // work-queue head of the batched eval kernel, reset here
    int* n_done;
    int lds_hist;           // as in ReduceArgs
};

__host__ __device__ inline FitVecs offset_vecs(FitVecs v, long long bytes) {
    auto sh = [bytes](auto* p) { return reinterpret_cast<decltype(p)>(reinterpret_cast<char*>(p) + bytes); };
    FitVecs o = v;
    o.x = sh(v.x);
    o.g = sh(v.g);
    o.d = sh(v.d);
    o.xt = sh(v.xt);
    o.m1 = sh(v.m1);
    o.v1 = sh(v.v1);
    o.xp = sh(v.xp);
    o.gp = sh(v.gp);
    o.S = sh(v.S);
    o.Y = sh(v.Y);
    o.rh = sh(v.rh);
    o.al = sh(v.al);
    o.theta_eval = sh(v.theta_eval);
    o.theta_eval64 = sh(v.theta_eval64);
    return o;
}

hipError_t launch_reduce(const ReduceArgs& ra, hipStream_t s);
hipError_t launch_reduce_batched(const BatchReduceArgs& ra, int n_epochs, hipStream_t s);
hipError_t launch_median(const float* img, int rows, int cols, long long ld, SelectState* sel, hipStream_t s);
hipError_t launch_ref_stats(const float* R, int rows, int cols, long long ld, SelectState* sel, hipStream_t s);
// The init / restart / finalize launchers run one workgroup per epoch (n_epochs >= 1, epoch e at
// byte offset e * stride; theta_user / theta_out hold n_epochs consecutive parameter vectors).
hipError_t launch_init_fit(FitState* st, FitVecs v, int m, int nb, int init_kind, double phi, const float* theta_user,
                           const SelectState* sel, hipStream_t s, int n_epochs = 1, long long stride = 0);
hipError_t launch_restart_fit(FitState* st, FitVecs v, int n, hipStream_t s, int n_epochs = 1, long long stride = 0);
hipError_t launch_finalize(FitState* st, FitVecs v, int m, float* theta_out, hipStream_t s, int n_epochs = 1,
                           long long stride = 0);
hipError_t launch_fill_mask(uint8_t* dst, const uint8_t* src, int rows, int cols, long long ld, hipStream_t s);
hipError_t launch_count_masked(const uint8_t* mask, int rows, int cols, long long ld, int m, int* count,
                               hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
hipError_t launch_widen(const float* src, double* dst, long long n, hipStream_t s);

}  // namespace dia

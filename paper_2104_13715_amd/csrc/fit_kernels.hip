// Cross-workgroup reduction, the on-device optimiser (Adam then L-BFGS,
// Sections 2.3 and 2.9), median initialisation and fit finalisation.
//
// The reduce kernel adds the per-workgroup partial rows of the tiled kernel in
// FP64 in a fixed order (16 columns per workgroup, 16 row phases per column).  In fit mode a step
// kernel (one workgroup per fit) then runs one optimiser step with the full gradient, so one optimiser
// iteration is exactly three launches and the host never reads anything back between iterations.  The
// step has a kernel of its own rather than running in the last column workgroup to finish: handing the
// sums over inside one kernel takes a device-scope fence in every workgroup, and on a device whose L2
// is split over several XCDs each such fence writes back its XCD's L2 (measured at 36 us per
// iteration for a 32-epoch batch, against a few us for a kernel boundary).
#include <cstdlib>
#include <map>
#include <mutex>

#include "fit_state.h"

namespace dia {

// ---------------------------------------------------------------------------- block helpers
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

// Sum over the 256 threads of the workgroup, same value returned to all threads.
__device__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kReduceThreads / 64; ++w) s += sh[w];
    return s;
}

__device__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = sh[0];
    for (int w = 1; w < kReduceThreads / 64; ++w) s = fmax(s, sh[w]);
    return s;
}

__device__ double dot(const double* a, const double* b, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kReduceThreads) s += a[i] * b[i];
    return block_sum(s, sh);
}

__device__ double max_abs(const double* a, int n, double* sh) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kReduceThreads) s = fmax(s, fabs(a[i]));
    return block_max(s, sh);
}

// ---------------------------------------------------------------------------- L-BFGS pieces
// Store the curvature pair (s, y) when s.y > 0 (Nocedal & Wright, Chapter 7.2).
__device__ void push_pair(FitState* st, const FitVecs& v, const double* s, const double* y, int n, int H,
                          double* sh) {
    const double sy = dot(s, y, n, sh);
    const double ss = dot(s, s, n, sh);
    const double yy = dot(y, y, n, sh);
    if (!(sy > 1e-12 * sqrt(ss * yy)) || !(sy > 0.0)) return;
    const int slot = st->hist_head;
    double* Sd = v.S + (long long)slot * v.ld;
    double* Yd = v.Y + (long long)slot * v.ld;
    for (int i = threadIdx.x; i < n; i += kReduceThreads) {
        Sd[i] = s[i];
        Yd[i] = y[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v.rh[slot] = 1.0 / sy;
        st->hist_head = (slot + 1) % H;
        st->hist_n = st->hist_n < H ? st->hist_n + 1 : H;
    }
    __syncthreads();
}

// d = -H_k g by the two-loop recursion, H_0 = gamma I with gamma = s.y / y.y of the newest pair.
__device__ void lbfgs_direction(FitState* st, const FitVecs& v, const double* g, int n, int H, double* sh) {
    double* d = v.d;
    for (int i = threadIdx.x; i < n; i += kReduceThreads) d[i] = g[i];
    __syncthreads();
    const int cnt = st->hist_n, head = st->hist_head;
    for (int k = 0; k < cnt; ++k) {
        const int idx = (head - 1 - k + H) % H;
        const double a = v.rh[idx] * dot(v.S + (long long)idx * v.ld, d, n, sh);
        if (threadIdx.x == 0) v.al[idx] = a;
        const double* Yk = v.Y + (long long)idx * v.ld;
        for (int i = threadIdx.x; i < n; i += kReduceThreads) d[i] -= a * Yk[i];
        __syncthreads();
    }
    double gamma;
    if (cnt > 0) {
        const int nw = (head - 1 + H) % H;
        const double* Yn = v.Y + (long long)nw * v.ld;
        gamma = 1.0 / (v.rh[nw] * dot(Yn, Yn, n, sh));
    } else {
        double l1 = 0.0;
        for (int i = threadIdx.x; i < n; i += kReduceThreads) l1 += fabs(g[i]);
        l1 = block_sum(l1, sh);
        gamma = l1 > 0.0 ? fmin(1.0, 1.0 / l1) : 1.0;
    }
    for (int i = threadIdx.x; i < n; i += kReduceThreads) d[i] *= gamma;
    __syncthreads();
    for (int k = cnt - 1; k >= 0; --k) {
        const int idx = (head - 1 - k + H) % H;
        const double b = v.rh[idx] * dot(v.Y + (long long)idx * v.ld, d, n, sh);
        const double* Sk = v.S + (long long)idx * v.ld;
        const double coef = v.al[idx] - b;
        for (int i = threadIdx.x; i < n; i += kReduceThreads) d[i] += coef * Sk[i];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < n; i += kReduceThreads) d[i] = -d[i];
    __syncthreads();
}

__device__ void write_theta(const FitState* st, const double* u, float* theta, int n, double* sh,
                            double* theta64);

__device__ void set_trial(FitState* st, const FitVecs& v, int n, double* sh) {
    // xt = x + alpha d; theta_eval = theta(xt)
    const double al = st->alpha;
    for (int i = threadIdx.x; i < n; i += kReduceThreads) v.xt[i] = v.x[i] + al * v.d[i];
    __syncthreads();
    write_theta(st, v.xt, v.theta_eval, n, sh, v.theta_eval64);
}

__device__ void finish(FitState* st, int* n_done, int stop, int status) {
    __syncthreads();
    if (threadIdx.x == 0) {
        st->stop = stop;
        st->status = status;
        st->phase = PH_DONE;
        st->done = 1;
        if (n_done != nullptr) atomicAdd(n_done, 1);
    }
    __syncthreads();
}

// Start the L-BFGS phase (or a new search direction) from the accepted point x with gradient g.
// lds (or null): room for the history S, Y (H slots of ld each) and the direction d, in which the
// two-loop recursion then runs: its dot products depend on each other, and read from LDS each costs
// a fraction of a round trip to L2.  The arithmetic and its order are the same either way.
__device__ void new_direction(FitState* st, const FitVecs& v, const FitOptsDev& o, int n, double* sh,
                              double* lds) {
    const int H = o.history;
    FitVecs w = v;
    if (lds != nullptr) {
        const long long hl = (long long)H * v.ld;
        for (long long k = threadIdx.x; k < hl; k += kReduceThreads) {
            lds[k] = v.S[k];
            lds[hl + k] = v.Y[k];
        }
        __syncthreads();
        w.S = lds;
        w.Y = lds + hl;
        w.d = lds + 2 * hl;
    }
    lbfgs_direction(st, w, v.g, n, H, sh);
    double gtd = dot(v.g, w.d, n, sh);
    if (!(gtd < 0.0)) {  // not a descent direction: drop the history, use the scaled gradient
        if (threadIdx.x == 0) {
            st->hist_n = 0;
            st->hist_head = 0;
        }
        __syncthreads();
        lbfgs_direction(st, w, v.g, n, H, sh);
        gtd = dot(v.g, w.d, n, sh);
    }
    if (lds != nullptr) {
        for (int i = threadIdx.x; i < n; i += kReduceThreads) v.d[i] = w.d[i];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->gtd = gtd;
        st->alpha = 1.0;
        st->ls_iter = 0;
        st->phase = PH_LSEARCH;
    }
    __syncthreads();
    set_trial(st, v, n, sh);
}

__device__ void adam_update(FitState* st, const FitVecs& v, const FitOptsDev& o, int n, double* sh) {
    const int t = st->adam_t + 1;
    const int nk = st->nk;
    const double bc1 = 1.0 - pow(o.beta1, (double)t);
    const double bc2 = 1.0 - pow(o.beta2, (double)t);
    for (int i = threadIdx.x; i < n; i += kReduceThreads) {
        const double gi = v.g[i];
        const double m1 = o.beta1 * v.m1[i] + (1.0 - o.beta1) * gi;
        const double v1 = o.beta2 * v.v1[i] + (1.0 - o.beta2) * gi * gi;
        v.m1[i] = m1;
        v.v1[i] = v1;
        v.xp[i] = v.x[i];
        v.gp[i] = gi;
        // kernel steps of lr_K in K are steps of lr_K * c in u; every background coefficient takes lr_B0
        const double lr = (i >= nk) ? o.lr_B0 : o.lr_K * st->ref_scale;
        v.x[i] = v.x[i] - lr * (m1 / bc1) / (sqrt(v1 / bc2) + o.eps);
    }
    __syncthreads();
    write_theta(st, v.x, v.theta_eval, n, sh, v.theta_eval64);
    if (threadIdx.x == 0) {
        st->adam_t = t;
        st->n_adam += 1;
    }
    __syncthreads();
}

// The optimiser works in coordinates u = (c K, B0 + s sum K), s and c the mean and RMS spread
// of the reference.  M = sum K R + B0 = sum (u_K / c)(R - s) + u_B: the constant part of R no
// longer couples every kernel pixel to B0, and kernel pixels and background have comparable
// curvature.  The optimum is the same point (the reference-offset invariance of the model).  With a
// polynomial background B0 is its constant term b_00; the other coefficients are not coupled to
// the reference's offset and are used as they are.
__device__ void write_theta(const FitState* st, const double* u, float* theta, int n, double* sh,
                            double* theta64 = nullptr) {
    const double c = st->ref_scale, s = st->ref_shift;
    const int nk = st->nk;
    double ks = 0.0;
    for (int i = threadIdx.x; i < nk; i += kReduceThreads) {
        const double k = u[i] / c;
        const float kf = (float)k;
        theta[i] = kf;
        if (theta64) theta64[i] = (double)kf;
        ks += k;
    }
    for (int i = nk + 1 + threadIdx.x; i < n; i += kReduceThreads) {
        const float bf = (float)u[i];
        theta[i] = bf;
        if (theta64) theta64[i] = (double)bf;
    }
    ks = block_sum(ks, sh);
    if (threadIdx.x == 0) {
        const float bf = (float)(u[nk] - s * ks);
        theta[nk] = bf;
        if (theta64) theta64[nk] = (double)bf;
    }
    __syncthreads();
}

// Sums over the workgroup of NV per-thread values, each summed in the same order as block_sum
// (wave sums, then the four wave totals in order); sh holds 4 * NV doubles.
template <int NV>
__device__ void block_sums(double (&v)[NV], double* sh) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) s += sh[w * NV + k];
        v[k] = s;
    }
}

// One Adam iteration that does not switch to L-BFGS, in two passes over the vectors and one
// workgroup reduction: the same arithmetic, in the same order, as the general path (non-finite check,
// gradient in u, the curvature pair of the last step, the Adam update, the new theta), which would take
// about eight dependent passes.  Returns false, having changed nothing, when this evaluation ends the
// Adam phase.
__device__ bool adam_iteration(const ReduceArgs& ra, double* sh) {
    FitState* st = ra.st;
    const FitVecs& v = ra.v;
    const FitOptsDev& o = ra.o;
    const int n = ra.n;
    const double* gt = ra.gt;
    const double Lt = gt[n], Lprev = st->L;
    const double rel = fabs(Lprev - Lt) / fmax(fabs(Lprev), 1e-300);
    if (rel < o.tol_switch || st->n_adam >= o.max_adam) return false;
    const int nk = st->nk;
    const double gB = gt[nk], sft = st->ref_shift, c = st->ref_scale, inv_c = 1.0 / c;
    const int t = st->adam_t + 1;
    const double bc1 = 1.0 - pow(o.beta1, (double)t);
    const double bc2 = 1.0 - pow(o.beta2, (double)t);
    // element i of: the gradient in u, the last step's pair (s, y), and the Adam update
    auto grad_u = [&](int i) { return i < nk ? (gt[i] - sft * gB) * inv_c : gt[i]; };
    auto x_new = [&](int i, double gi, double& m1, double& v1) {
        m1 = o.beta1 * v.m1[i] + (1.0 - o.beta1) * gi;
        v1 = o.beta2 * v.v1[i] + (1.0 - o.beta2) * gi * gi;
        const double lr = (i >= nk) ? o.lr_B0 : o.lr_K * c;
        return v.x[i] - lr * (m1 / bc1) / (sqrt(v1 / bc2) + o.eps);
    };
    // pass 1: non-finite flag, s.y, s.s, y.y and the sum of the new kernel values
    // (one loop, so that every load of an element is in flight at once; each sum keeps its element order)
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    {
        int bad = (threadIdx.x == n % kReduceThreads) ? !isfinite(Lt) : 0;
        double sy = 0.0, ss = 0.0, yy = 0.0, ks = 0.0;
        for (int i = threadIdx.x; i < n; i += kReduceThreads) {
            bad |= !isfinite(gt[i]);
            const double gi = grad_u(i);
            const double si = v.x[i] - v.xp[i], yi = gi - v.gp[i];
            sy += si * yi;
            ss += si * si;
            yy += yi * yi;
            if (i < nk) {
                double m1, v1;
                ks += x_new(i, gi, m1, v1) / c;
            }
        }
        acc[0] = (double)bad;
        acc[1] = sy, acc[2] = ss, acc[3] = yy, acc[4] = ks;
    }
    block_sums(acc, sh);
    if (acc[0] > 0.0) {
        finish(st, ra.n_done, STOP_NONE, DIA_E_NONFINITE);
        return true;
    }
    const double sy = acc[1], ss = acc[2], yy = acc[3], ks = acc[4];
    const bool keep = (sy > 1e-12 * sqrt(ss * yy)) && (sy > 0.0);
    const int H = o.history, slot = st->hist_head;
    double* Sd = v.S + (long long)slot * v.ld;
    double* Yd = v.Y + (long long)slot * v.ld;
    __syncthreads();  // every thread has read the state it needs before any of it changes
    // pass 2: the pair into the history, the Adam moments and point, the new theta
    for (int i = threadIdx.x; i < n; i += kReduceThreads) {
        const double gi = grad_u(i);
        const double xi = v.x[i];
        if (keep) {
            Sd[i] = xi - v.xp[i];
            Yd[i] = gi - v.gp[i];
        }
        double m1, v1;
        const double xn = x_new(i, gi, m1, v1);
        v.m1[i] = m1;
        v.v1[i] = v1;
        v.xp[i] = xi;
        v.gp[i] = gi;
        v.g[i] = gi;
        v.x[i] = xn;
        if (i < nk) {
            const float kf = (float)(xn / c);
            v.theta_eval[i] = kf;
            v.theta_eval64[i] = (double)kf;
        } else if (i == nk) {
            const float bf = (float)(xn - sft * ks);
            v.theta_eval[i] = bf;
            v.theta_eval64[i] = (double)bf;
        } else {
            const float bf = (float)xn;
            v.theta_eval[i] = bf;
            v.theta_eval64[i] = (double)bf;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->n_eval += 1;
        if (keep) {
            v.rh[slot] = 1.0 / sy;
            st->hist_head = (slot + 1) % H;
            st->hist_n = st->hist_n < H ? st->hist_n + 1 : H;
        }
        st->L = Lt;
        st->adam_t = t;
        st->n_adam += 1;
    }
    __syncthreads();
    if (st->n_eval >= o.max_eval) finish(st, ra.n_done, STOP_CAP, DIA_W_NOT_CONVERGED);
    return true;
}

// One optimiser step, run by a single workgroup once the full gradient gt (and loss gt[n]) is known
// (lds: as in new_direction).
__device__ void optimiser_step(const ReduceArgs& ra, double* sh, double* lds) {
    if (ra.st->phase == PH_ADAM && adam_iteration(ra, sh)) return;
    FitState* st = ra.st;
    const FitVecs& v = ra.v;
    const FitOptsDev& o = ra.o;
    const int n = ra.n;
    double* gt = ra.gt;
    const double Lt = gt[n];

    // non-finite loss or gradient ends the fit
    int bad = 0;
    for (int i = threadIdx.x; i <= n; i += kReduceThreads) bad |= !isfinite(gt[i]);
    if (block_max((double)bad, sh) > 0.0) {
        finish(st, ra.n_done, STOP_NONE, DIA_E_NONFINITE);
        return;
    }
    // gradient in u: dL/du_K = (dL/dK - s dL/dB0) / c, dL/du_B = dL/dB0 (in place)
    {
        const int nk = st->nk;
        const double gB = gt[nk], sft = st->ref_shift, inv_c = 1.0 / st->ref_scale;
        __syncthreads();
        for (int i = threadIdx.x; i < nk; i += kReduceThreads) gt[i] = (gt[i] - sft * gB) * inv_c;
        __syncthreads();
    }
    if (threadIdx.x == 0) st->n_eval += 1;
    __syncthreads();
    const int phase = st->phase;

    if (phase == PH_INIT || phase == PH_ADAM) {
        const double Lprev = st->L;
        if (phase == PH_INIT) {
            const double gm = max_abs(gt, n, sh);
            if (threadIdx.x == 0) {
                st->gmax0 = gm;
                st->phase = PH_ADAM;
            }
        } else {
            // curvature pair from the last Adam step: s = x - xp, y = gt - gp (xd, d as scratch)
            for (int i = threadIdx.x; i < n; i += kReduceThreads) {
                v.xt[i] = v.x[i] - v.xp[i];
                v.d[i] = gt[i] - v.gp[i];
            }
            __syncthreads();
            push_pair(st, v, v.xt, v.d, n, o.history, sh);
        }
        for (int i = threadIdx.x; i < n; i += kReduceThreads) v.g[i] = gt[i];
        __syncthreads();
        if (threadIdx.x == 0) st->L = Lt;
        __syncthreads();
        const double rel = fabs(Lprev - Lt) / fmax(fabs(Lprev), 1e-300);
        const bool switch_now = (phase == PH_ADAM && (rel < o.tol_switch || st->n_adam >= o.max_adam)) ||
                                (phase == PH_INIT && o.skip_adam);
        if (!switch_now) {
            adam_update(st, v, o, n, sh);
        } else {
            const double gm = max_abs(v.g, n, sh);
            if (gm <= o.tol_grad * st->gmax0) {
                finish(st, ra.n_done, STOP_GRAD, DIA_OK);
                return;
            }
            if (o.max_lbfgs == 0) {
                // no quasi-Newton phase: the first-order part ends at the switch (the exact-Hessian Newton
                // polish, when enabled, continues from here)
                const bool capped = phase == PH_ADAM && !(rel < o.tol_switch);
                finish(st, ra.n_done, capped ? STOP_CAP : STOP_CHANGE, capped ? DIA_W_NOT_CONVERGED : DIA_OK);
                return;
            }
            new_direction(st, v, o, n, sh, lds);
        }
    } else if (phase == PH_LSEARCH) {
        const double L0 = st->L;
        const double alpha = st->alpha;
        // Change of the loss along the step.  Far from the optimum the FP64 sum of the FP32 pixel
        // terms is exact enough; once |dL| falls below 1e-5 |L| it is dominated by the rounding of
        // the FP32 model values, and the change is taken from the gradients instead:
        // L(x + s) - L(x) = (g(x) + g(x + s)) . s / 2, exact for a quadratic objective.
        double tr = 0.0;
        for (int i = threadIdx.x; i < n; i += kReduceThreads) tr += (v.g[i] + gt[i]) * (v.xt[i] - v.x[i]);
        const double dlg = 0.5 * block_sum(tr, sh);
        const double dll = Lt - L0;
        const double dL = (fabs(dll) > 1e-5 * fabs(L0)) ? dll : dlg;
        if (dL <= 1e-4 * alpha * st->gtd) {
            // accept: s = xt - x, y = gt - g
            for (int i = threadIdx.x; i < n; i += kReduceThreads) {
                v.d[i] = v.xt[i] - v.x[i];
                v.m1[i] = gt[i] - v.g[i];  // m1 is free in this phase
            }
            __syncthreads();
            push_pair(st, v, v.d, v.m1, n, o.history, sh);
            for (int i = threadIdx.x; i < n; i += kReduceThreads) {
                v.x[i] = v.xt[i];
                v.g[i] = gt[i];
            }
            __syncthreads();
            const double rel = fabs(dL) / fmax(fabs(L0), 1e-300);
            const int small = (rel < o.tol_change) ? st->small_steps + 1 : 0;
            __syncthreads();
            if (threadIdx.x == 0) {
                st->L = Lt;
                st->n_lbfgs += 1;
                st->small_steps = small;
            }
            __syncthreads();
            const double gm = max_abs(v.g, n, sh);
            if (gm <= o.tol_grad * st->gmax0) {
                finish(st, ra.n_done, STOP_GRAD, DIA_OK);
                return;
            }
            if (small >= 3) {
                finish(st, ra.n_done, STOP_CHANGE, DIA_OK);
                return;
            }
            if (st->n_lbfgs >= o.max_lbfgs) {
                finish(st, ra.n_done, STOP_CAP, DIA_W_NOT_CONVERGED);
                return;
            }
            new_direction(st, v, o, n, sh, lds);
        } else {
            // backtrack: minimiser of the quadratic through L0, slope gtd and L0 + dL, kept in [0.1, 0.5] alpha
            const int it = st->ls_iter + 1;
            if (it >= 40) {
                finish(st, ra.n_done, STOP_LINESEARCH, DIA_OK);
                return;
            }
            const double gtd = st->gtd;
            double an = -gtd * alpha * alpha / (2.0 * (dL - gtd * alpha));
            if (!(an >= 0.1 * alpha)) an = 0.1 * alpha;
            if (an > 0.5 * alpha) an = 0.5 * alpha;
            if (threadIdx.x == 0) {
                st->alpha = an;
                st->ls_iter = it;
            }
            __syncthreads();
            set_trial(st, v, n, sh);
        }
    }
    if (st->phase != PH_DONE && st->n_eval >= o.max_eval) finish(st, ra.n_done, STOP_CAP, DIA_W_NOT_CONVERGED);
}

// ---------------------------------------------------------------------------- reduce kernel
// Sum of rows r0, r0 + kReducePhases, ... < r1 of one partial column, four loads in flight
// (fixed order: the four running sums are combined the same way every time).
__device__ __forceinline__ double column_sum(const double* p, long long npp, int r0, int r1) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int r = r0;
    for (; r + 3 * kReducePhases < r1; r += 4 * kReducePhases) {
        s0 += p[(long long)r * npp];
        s1 += p[(long long)(r + kReducePhases) * npp];
        s2 += p[(long long)(r + 2 * kReducePhases) * npp];
        s3 += p[(long long)(r + 3 * kReducePhases) * npp];
    }
    for (; r < r1; r += kReducePhases) s0 += p[(long long)r * npp];
    return (s0 + s1) + (s2 + s3);
}

// Thread (phase, column): phases split the rows, then thread phase 0 adds the kReducePhases
// sums in order.
__device__ __forceinline__ double reduce_columns(const double* partial, int npp, int r0, int r1, int col,
                                                 double (*red)[kReduceCols]) {
    const int tid = threadIdx.x;
    const int ph = tid / kReduceCols, c = tid % kReduceCols;
    const double s = (col < npp) ? column_sum(partial + col, npp, r0 + ph, r1) : 0.0;
    red[ph][c] = s;
    __syncthreads();
    double tot = 0.0;
    if (ph == 0)
        for (int k = 0; k < kReducePhases; ++k) tot += red[k][c];
    return tot;
}

// (L t)_u for kernel pixel u = a m + b: Laplacian of the pixel graph whose edges join pixels
// sharing a side (Section 2.7, eq. laplacian): degree times t_u minus the neighbours' values.
__device__ __forceinline__ double lap_apply(const double* t, int u, int m) {
    const int a = u / m, b = u - a * m;
    double s = 0.0;
    int deg = 0;
    if (a > 0) s += t[u - m], ++deg;
    if (a + 1 < m) s += t[u + m], ++deg;
    if (b > 0) s += t[u - 1], ++deg;
    if (b + 1 < m) s += t[u + 1], ++deg;
    return deg * t[u] - s;
}

// (L L t)_u: the same stencil applied to (L t) at u and its neighbours (L is symmetric).
__device__ __forceinline__ double lap2_apply(const double* t, int u, int m) {
    const int a = u / m, b = u - a * m;
    double s = 0.0;
    int deg = 0;
    if (a > 0) s += lap_apply(t, u - m, m), ++deg;
    if (a + 1 < m) s += lap_apply(t, u + m, m), ++deg;
    if (b > 0) s += lap_apply(t, u - 1, m), ++deg;
    if (b + 1 < m) s += lap_apply(t, u + 1, m), ++deg;
    return deg * lap_apply(t, u, m) - s;
}

__global__ __launch_bounds__(kReduceThreads) void reduce_kernel(ReduceArgs ra) {
    __shared__ double red[kReducePhases][kReduceCols];
    __shared__ double sh[16];
    if (ra.done != nullptr && *ra.done != 0) return;
    const int tid = threadIdx.x;
    const int col = blockIdx.x * kReduceCols + (tid % kReduceCols);
    double tot = reduce_columns(ra.partial, ra.npp, 0, ra.nblk, col, red);
    if (ra.reg > 0.0) {
        // kernel-smoothness penalty reg t^T L^T L t (Section 2.7, eq. regularised_loss): its gradient
        // 2 reg (L L t) on the kernel columns, its value on the loss column (summed by the whole
        // workgroup that owns that column; the condition is uniform over the workgroup)
        const int nk = ra.m * ra.m;
        if (blockIdx.x == ra.n / kReduceCols) {
            double q = 0.0;
            for (int u = tid; u < nk; u += kReduceThreads) {
                const double l = lap_apply(ra.th64, u, ra.m);
                q += l * l;
            }
            q = block_sum(q, sh);
            if (col == ra.n) tot += ra.reg * q;
        }
        if (tid < kReduceCols && col < nk) tot += 2.0 * ra.reg * lap2_apply(ra.th64, col, ra.m);
    }
    if (tid < kReduceCols && col < ra.npp) {
        ra.gt[col] = tot;
        if (ra.out_grad != nullptr && col < ra.n) ra.out_grad[col] = (float)tot;
        if (ra.out_grad64 != nullptr && col < ra.n) ra.out_grad64[col] = tot;
        if (ra.out_loss != nullptr && col == ra.n) ra.out_loss[0] = tot;
    }
}

// One optimiser step of a single fit on the reduced gradient and loss gt (one workgroup).
__global__ __launch_bounds__(kReduceThreads) void step_kernel(ReduceArgs ra) {
    __shared__ double sh[32];
    extern __shared__ double step_lds[];
    if (ra.done != nullptr && *ra.done != 0) return;
    optimiser_step(ra, sh, ra.lds_hist ? step_lds : nullptr);
}

// Dynamic LDS of a step kernel: the L-BFGS history (S and Y, H slots of ld doubles each) and the
// direction, or 0 when that exceeds what one workgroup may hold (the recursion then reads L2).
constexpr size_t kStepLdsMax = 144 * 1024;
size_t step_lds_bytes(int history, int ld) {
    const size_t b = sizeof(double) * ((size_t)2 * history * ld + ld);
    return b <= kStepLdsMax ? b : 0;
}

__global__ void step_batched_kernel(BatchReduceArgs br);

// Raise the step kernels' dynamic-LDS limit once per device (beyond the default a launch may not ask
// for more); false: launch them without the LDS copy.  DIA_STEP_LDS=0 keeps every step on the L2 path
// (the two paths give bitwise the same results).
bool step_lds_ready() {
    const char* e = std::getenv("DIA_STEP_LDS");  // read at every launch (cheap), so a process can switch
    if (e != nullptr && e[0] == '0') return false;
    static std::mutex mu;
    static std::map<int, bool> ready;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(mu);
    auto it = ready.find(dev);
    if (it != ready.end()) return it->second;
    const bool ok =
        hipFuncSetAttribute(reinterpret_cast<const void*>(step_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kStepLdsMax) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(step_batched_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStepLdsMax) == hipSuccess;
    if (!ok) (void)hipGetLastError();  // a refused attribute is not the launch's error
    ready[dev] = ok;
    return ok;
}

hipError_t launch_reduce(const ReduceArgs& ra, hipStream_t s) {
    const int grid = (ra.npp + kReduceCols - 1) / kReduceCols;
    hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(kReduceThreads), 0, s, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ra.st == nullptr) return e;
    ReduceArgs r = ra;
    const size_t lds = step_lds_ready() ? step_lds_bytes(ra.o.history, ra.v.ld) : 0;
    r.lds_hist = lds > 0 ? 1 : 0;
    hipLaunchKernelGGL(step_kernel, dim3(1), dim3(kReduceThreads), lds, s, r);
    return hipGetLastError();
}

// Batched: grid (column blocks, epochs).  Epoch e adds its chunk rows [cbeg[e], cend[e]) in order;
// in fit mode a step kernel with one workgroup per epoch then runs each epoch's optimiser step.
__global__ __launch_bounds__(kReduceThreads) void reduce_batched_kernel(BatchReduceArgs br) {
    __shared__ double red[kReducePhases][kReduceCols];
    const int e = blockIdx.y;
    const int tid = threadIdx.x;
    if (br.queue != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *br.queue = 0;
    const long long off = (long long)e * br.stride;
    FitState* st = br.st ? reinterpret_cast<FitState*>(reinterpret_cast<char*>(br.st) + off) : nullptr;
    if (st != nullptr && st->done != 0) return;
    const int col = blockIdx.x * kReduceCols + (tid % kReduceCols);
    const int r0 = br.cbeg ? br.cbeg[e] : e * br.rows_per, r1 = br.cend ? br.cend[e] : (e + 1) * br.rows_per;
    const double tot = reduce_columns(br.partial, br.npp, r0, r1, col, red);
    double* gt = br.gt + (long long)e * br.npp;
    if (tid < kReduceCols && col < br.npp) {
        gt[col] = tot;
        if (br.out_grad != nullptr && col < br.n) br.out_grad[(long long)e * br.n + col] = (float)tot;
        if (br.out_loss != nullptr && col == br.n) br.out_loss[e] = tot;
    }
}

// The optimiser step of epoch blockIdx.x of a batched fit (one workgroup per epoch).
__global__ __launch_bounds__(kReduceThreads) void step_batched_kernel(BatchReduceArgs br) {
    __shared__ double sh[32];
    extern __shared__ double step_lds[];
    const int e = blockIdx.x;
    const long long off = (long long)e * br.stride;
    FitState* st = reinterpret_cast<FitState*>(reinterpret_cast<char*>(br.st) + off);
    if (st->done != 0) return;
    ReduceArgs ra;
    ra.partial = nullptr;
    ra.nblk = 0;
    ra.npp = br.npp;
    ra.gt = br.gt + (long long)e * br.npp;
    ra.out_loss = nullptr;
    ra.out_grad = nullptr;
    ra.out_grad64 = nullptr;
    ra.st = st;
    ra.v = offset_vecs(br.v, off);
    ra.o = br.o;
    ra.n = br.n;
    ra.m = br.m;
    ra.done = nullptr;
    ra.n_done = br.n_done;
    ra.reg = 0.0;
    ra.th64 = nullptr;
    ra.lds_hist = br.lds_hist;
    optimiser_step(ra, sh, br.lds_hist ? step_lds : nullptr);
}

hipError_t launch_reduce_batched(const BatchReduceArgs& ra, int n_epochs, hipStream_t s) {
    const int gx = (ra.npp + kReduceCols - 1) / kReduceCols;
    hipLaunchKernelGGL(reduce_batched_kernel, dim3(gx, n_epochs), dim3(kReduceThreads), 0, s, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ra.st == nullptr) return e;
    BatchReduceArgs r = ra;
    const size_t lds = step_lds_ready() ? step_lds_bytes(ra.o.history, ra.v.ld) : 0;
    r.lds_hist = lds > 0 ? 1 : 0;
    hipLaunchKernelGGL(step_batched_kernel, dim3(n_epochs), dim3(kReduceThreads), lds, s, r);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- median (radix select)
__device__ __forceinline__ unsigned f2key(float f) {
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key2f(unsigned k) {
    const unsigned u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}

__global__ __launch_bounds__(256) void select_init_kernel(SelectState* sel, long long npix) {
    const int t = threadIdx.x;
    if (t < 2) {
        sel->prefix[t] = 0u;
        sel->mask[t] = 0u;
        sel->k[t] = (t == 0) ? (npix - 1) / 2 : npix / 2;
    }
    sel->hist[0][t] = 0u;
    sel->hist[1][t] = 0u;
}

__global__ __launch_bounds__(256) void select_hist_kernel(const float* img, int rows, int cols, long long ld,
                                                          SelectState* sel, int shift) {
    __shared__ unsigned h[2][256];
    h[0][threadIdx.x] = 0u;
    h[1][threadIdx.x] = 0u;
    __syncthreads();
    const unsigned p0 = sel->prefix[0], m0 = sel->mask[0], p1 = sel->prefix[1], m1 = sel->mask[1];
    const long long npix = (long long)rows * cols;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npix;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long r = idx / cols, c = idx - r * cols;
        const unsigned key = f2key(img[r * ld + c]);
        const unsigned bin = (key >> shift) & 255u;
        if ((key & m0) == p0) atomicAdd(&h[0][bin], 1u);
        if ((key & m1) == p1) atomicAdd(&h[1][bin], 1u);
    }
    __syncthreads();
    if (h[0][threadIdx.x]) atomicAdd(&sel->hist[0][threadIdx.x], h[0][threadIdx.x]);
    if (h[1][threadIdx.x]) atomicAdd(&sel->hist[1][threadIdx.x], h[1][threadIdx.x]);
}

__global__ void select_pick_kernel(SelectState* sel, int shift) {
    const int w = threadIdx.x;  // 2 threads: one per rank
    if (w < 2) {
        long long cum = 0;
        const long long k = sel->k[w];
        int bin = 255;
        for (int b = 0; b < 256; ++b) {
            const long long c = sel->hist[w][b];
            if (cum + c > k) {
                bin = b;
                break;
            }
            cum += c;
        }
        sel->prefix[w] |= (unsigned)bin << shift;
        sel->mask[w] |= 255u << shift;
        sel->k[w] = k - cum;
        for (int b = 0; b < 256; ++b) sel->hist[w][b] = 0u;
    }
}

hipError_t launch_median(const float* img, int rows, int cols, long long ld, SelectState* sel, hipStream_t s) {
    const long long npix = (long long)rows * cols;
    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, sel, npix);
    long long blocks = (npix + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(select_hist_kernel, dim3((int)blocks), dim3(256), 0, s, img, rows, cols, ld, sel, shift);
        hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(64), 0, s, sel, shift);
    }
    return hipGetLastError();
}

// Sum and sum of squares of the reference, per block (fixed grid), reduced in order by the init kernel.
__global__ __launch_bounds__(256) void ref_stats_kernel(const float* R, int rows, int cols, long long ld,
                                                        SelectState* sel) {
    __shared__ double sh[2][4];
    const long long npix = (long long)rows * cols;
    double s1 = 0.0, s2 = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npix;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long r = idx / cols, c = idx - r * cols;
        const double x = (double)R[r * ld + c];
        s1 += x;
        s2 += x * x;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s1;
        sh[1][threadIdx.x >> 6] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sel->stat_part[2 * blockIdx.x] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        sel->stat_part[2 * blockIdx.x + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
        if (blockIdx.x == 0) sel->stat_n = npix;
    }
}

hipError_t launch_ref_stats(const float* R, int rows, int cols, long long ld, SelectState* sel, hipStream_t s) {
    hipLaunchKernelGGL(ref_stats_kernel, dim3(kStatBlocks), dim3(256), 0, s, R, rows, cols, ld, sel);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- fit init / finalize
__global__ __launch_bounds__(kReduceThreads) void init_fit_kernel(FitState* st0, FitVecs v0, int m, int nb,
                                                                  int init_kind, double phi,
                                                                  const float* theta_user0,
                                                                  const SelectState* sel0, long long stride) {
    __shared__ double sh[16];
    const int nk = m * m, n = nk + nb;
    const long long off = (long long)blockIdx.x * stride;
    FitState* st = reinterpret_cast<FitState*>(reinterpret_cast<char*>(st0) + off);
    const FitVecs v = offset_vecs(v0, off);
    const float* theta_user = theta_user0 ? theta_user0 + (long long)blockIdx.x * n : nullptr;
    const SelectState* sel = reinterpret_cast<const SelectState*>(reinterpret_cast<const char*>(sel0) + off);
    const int h = (m - 1) / 2;

    // reference statistics: s = mean, c = RMS of (R - s) (1 for a constant reference)
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < kStatBlocks; ++b) {
        s1 += sel->stat_part[2 * b];
        s2 += sel->stat_part[2 * b + 1];
    }
    const double np = (double)(sel->stat_n > 0 ? sel->stat_n : 1);
    const double sft = s1 / np;
    const double var = s2 / np - sft * sft;
    const double scl = var > 0.0 ? sqrt(var) : 1.0;

    double ksum = 1.0;
    if (init_kind == DIA_INIT_GAUSS) {
        double s = 0.0;
        for (int i = threadIdx.x; i < m * m; i += kReduceThreads) {
            const double da = (double)(i / m - h), db = (double)(i % m - h);
            s += exp(-0.5 * (da * da + db * db) / (phi * phi));
        }
        ksum = block_sum(s, sh);
    }
    double B0 = 0.0;
    if (init_kind != DIA_INIT_USER) {
        const double lo = (double)key2f(sel->prefix[0]);
        const double hi = (double)key2f(sel->prefix[1]);
        B0 = 0.5 * (lo + hi);
    }
    // theta_0 -> u: u_K = c K, u_B = B0 + s sum K
    double kt = 0.0;
    for (int i = threadIdx.x; i < v.ld; i += kReduceThreads) {
        double x = 0.0;
        if (i < n) {
            if (init_kind == DIA_INIT_USER) {
                x = (double)theta_user[i];
            } else if (i == nk) {
                x = B0;
            } else if (i > nk) {
                x = 0.0;  // higher background terms start flat
            } else if (init_kind == DIA_INIT_FLAT) {
                x = 1.0 / (double)(m * m);
            } else {
                const double da = (double)(i / m - h), db = (double)(i % m - h);
                x = exp(-0.5 * (da * da + db * db) / (phi * phi)) / ksum;
            }
            v.theta_eval[i] = (float)x;
            v.theta_eval64[i] = (double)(float)x;
            if (i < nk) kt += x;
        }
        const double u = (i < nk) ? scl * x : x;
        v.x[i] = u;
        v.xt[i] = u;
        v.g[i] = 0.0;
        v.d[i] = 0.0;
        v.m1[i] = 0.0;
        v.v1[i] = 0.0;
        v.xp[i] = u;
        v.gp[i] = 0.0;
    }
    kt = block_sum(kt, sh);
    if (threadIdx.x == 0) {
        v.x[nk] += sft * kt;
        v.xt[nk] = v.x[nk];
        v.xp[nk] = v.x[nk];
        FitState z = {};
        z.phase = PH_INIT;
        z.alpha = 1.0;
        z.ref_shift = sft;
        z.ref_scale = scl;
        z.nk = nk;
        z.n = n;
        *st = z;
    }
}

hipError_t launch_init_fit(FitState* st, FitVecs v, int m, int nb, int init_kind, double phi, const float* theta_user,
                           const SelectState* sel, hipStream_t s, int n_epochs, long long stride) {
    hipLaunchKernelGGL(init_fit_kernel, dim3(n_epochs), dim3(kReduceThreads), 0, s, st, v, m, nb, init_kind, phi,
                       theta_user, sel, stride);
    return hipGetLastError();
}

// Restart the optimiser from the current x (a warm start for the next outer fit); the L-BFGS
// curvature pairs are kept, the objective having changed only through the weights and mask.
__global__ __launch_bounds__(kReduceThreads) void restart_fit_kernel(FitState* st0, FitVecs v0, int n,
                                                                     long long stride) {
    __shared__ double sh[16];
    const long long off = (long long)blockIdx.x * stride;
    FitState* st = reinterpret_cast<FitState*>(reinterpret_cast<char*>(st0) + off);
    const FitVecs v = offset_vecs(v0, off);
    const int hist_n = st->hist_n, hist_head = st->hist_head, nk = st->nk, np = st->n;
    const double sft = st->ref_shift, scl = st->ref_scale;
    write_theta(st, v.x, v.theta_eval, n, sh, v.theta_eval64);
    for (int i = threadIdx.x; i < v.ld; i += kReduceThreads) {
        const double x = v.x[i];
        v.xt[i] = x;
        v.g[i] = 0.0;
        v.d[i] = 0.0;
        v.m1[i] = 0.0;
        v.v1[i] = 0.0;
        v.xp[i] = x;
        v.gp[i] = 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        FitState z = {};
        z.phase = PH_INIT;
        z.alpha = 1.0;
        z.hist_n = hist_n;
        z.hist_head = hist_head;
        z.ref_shift = sft;
        z.ref_scale = scl;
        z.nk = nk;
        z.n = np;
        *st = z;
    }
}

hipError_t launch_restart_fit(FitState* st, FitVecs v, int n, hipStream_t s, int n_epochs, long long stride) {
    hipLaunchKernelGGL(restart_fit_kernel, dim3(n_epochs), dim3(kReduceThreads), 0, s, st, v, n, stride);
    return hipGetLastError();
}

__global__ __launch_bounds__(kReduceThreads) void finalize_kernel(FitState* st0, FitVecs v0, int m, float* theta_out0,
                                                                  long long stride) {
    __shared__ double sh[16];
    const long long off = (long long)blockIdx.x * stride;
    FitState* st = reinterpret_cast<FitState*>(reinterpret_cast<char*>(st0) + off);
    const FitVecs v = offset_vecs(v0, off);
    const int n = st->n, nk = st->nk;
    float* theta_out = theta_out0 + (long long)blockIdx.x * n;
    write_theta(st, v.x, theta_out, n, sh, nullptr);
    // P and B0 of the FP64 iterate (the point whose loss is reported), not of its FP32 rounding:
    // when sum |K| is large against P (an unregularised kernel whose poorly constrained modes are
    // big), rounding every pixel to FP32 moves sum K by up to 2^-24 sum |K|
    double s = 0.0;
    for (int i = threadIdx.x; i < nk; i += kReduceThreads) s += v.x[i];
    const double P = block_sum(s, sh) / st->ref_scale;
    if (threadIdx.x == 0) {
        st->out_P = P;
        st->out_B0 = v.x[nk] - st->ref_shift * P;
        st->out_loss = st->L;
    }
}

hipError_t launch_finalize(FitState* st, FitVecs v, int m, float* theta_out, hipStream_t s, int n_epochs,
                           long long stride) {
    hipLaunchKernelGGL(finalize_kernel, dim3(n_epochs), dim3(kReduceThreads), 0, s, st, v, m, theta_out, stride);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- mask helpers
__global__ void fill_mask_kernel(uint8_t* dst, const uint8_t* src, int rows, int cols, long long ld) {
    const long long npix = (long long)rows * cols;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npix;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long r = idx / cols, c = idx - r * cols;
        dst[r * ld + c] = src ? (uint8_t)(src[r * ld + c] != 0) : (uint8_t)1;
    }
}

hipError_t launch_fill_mask(uint8_t* dst, const uint8_t* src, int rows, int cols, long long ld, hipStream_t s) {
    long long blocks = ((long long)rows * cols + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_mask_kernel, dim3((int)blocks), dim3(256), 0, s, dst, src, rows, cols, ld);
    return hipGetLastError();
}

__global__ void count_masked_kernel(const uint8_t* mask, int rows, int cols, long long ld, int m, int* count) {
    const int h = (m - 1) / 2;
    const int Hv = rows - m + 1, Wv = cols - m + 1;
    const long long npix = (long long)Hv * Wv;
    int c = 0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < npix;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long r = idx / Wv, cc = idx - r * Wv;
        c += (mask[(r + h) * ld + cc + h] == 0);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

hipError_t launch_count_masked(const uint8_t* mask, int rows, int cols, long long ld, int m, int* count,
                               hipStream_t s) {
    long long blocks = ((long long)rows * cols + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(count_masked_kernel, dim3((int)blocks), dim3(256), 0, s, mask, rows, cols, ld, m, count);
    return hipGetLastError();
}

__global__ void widen_kernel(const float* src, double* dst, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

hipError_t launch_widen(const float* src, double* dst, long long n, hipStream_t s) {
    long long blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(widen_kernel, dim3((int)blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

__global__ void zero_ints_kernel(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace dia

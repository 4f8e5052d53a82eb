// Host side of the exact-Hessian Newton polish and of the Hessian entry point.
#include "api_util.h"
#include "newton.h"

namespace dia {

NewtonLayout newton_layout(int m, int rows, int cols, bool own_partial, bool own_H) {
    NewtonLayout L;
    const int n = m * m + kMaxBgTerms;
    const long long hv_px = (long long)(rows - m + 1) * (cols - m + 1);
    L.npb = hess_pair_blocks(m);
    L.splits = hess_splits(m, rows, cols);
    L.has_part = own_partial;
    L.has_H = own_H;
    size_t off = 0;
    L.h = off;
    off = align_up(off + sizeof(double) * (size_t)hv_px);
    L.hpart = off;
    off = align_up(off + sizeof(double) * (size_t)L.splits * L.npb * kHessBlockElems);
    if (own_H) {
        L.H = off;
        off = align_up(off + sizeof(double) * (size_t)n * n);
    }
    L.hv = off;
    off = align_up(off + sizeof(double) * (size_t)kMaxBgTerms * (n + 1));
    L.d = off;
    off = align_up(off + sizeof(double) * (size_t)n);
    L.th = off;
    off = align_up(off + sizeof(double) * (size_t)n);
    L.info = off;
    off = align_up(off + sizeof(double) * 4);
    L.gt = off;
    off = align_up(off + sizeof(double) * (size_t)(n + 1));
    if (own_partial) {
        const int nt = max_tiles(m, rows, cols);
        L.part = off;
        off = align_up(off + sizeof(double) * (size_t)(nt < kMaxGrid ? nt : kMaxGrid) * (n + 1));
    }
    L.total = off;
    return L;
}

namespace {

// One fused pass at (theta, theta64) reduced into gt (gradient, then the loss at gt[n]).
bool eval_into(const dia_image& R, const dia_image& I, const ObjParams& obj, double reg, int m, int bg_deg, int grid,
               int variant, const float* theta, const double* theta64, double* partial, double* gt, hipStream_t s) {
    TileArgs a = base_args(R, I, theta);
    a.theta64 = theta64;
    a.obj = obj;
    a.partial = partial;
    set_background(a, bg_deg, m);
    if (launch_tile(MODE_EVAL, m, grid, a, s, variant) != hipSuccess) return false;
    const int n = m * m + a.nb;
    ReduceArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.partial = partial;
    ra.nblk = grid;
    ra.npp = n + 1;
    ra.gt = gt;
    ra.n = n;
    ra.m = m;
    ra.reg = reg;
    ra.th64 = theta64;
    return launch_reduce(ra, s) == hipSuccess;
}

bool read_back(void* dst, const void* src, size_t bytes, hipStream_t s) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) == hipSuccess &&
           hipStreamSynchronize(s) == hipSuccess;
}

}  // namespace

int hessian_into(const dia_image& R, const dia_image& I, const ObjParams& obj, double reg, int m, int bg_deg,
                 const float* theta, const double* theta64, int exact, double* partial, char* nbase,
                 const NewtonLayout& NL, double* H, hipStream_t s, double damp) {
    const int grid0 = eval_grid(m, tile_grid_tiles(m, R.rows, R.cols, 0), 0);
    TileArgs c = base_args(R, I, theta);
    c.theta64 = theta64;
    c.obj = obj;
    c.partial = partial;
    c.h_out = reinterpret_cast<double*>(nbase + NL.h);
    c.curv_exact = exact;
    set_background(c, bg_deg, m);
    const int nb = c.nb, n = m * m + nb;
    // one curvature pass per background term: term (a, b) weights the per-pixel curvature by
    // eta^a xi^b, so its partial row is that term's row of H (the first pass also writes h)
    for (int pa = 0; pa <= bg_deg; ++pa)
        for (int pb = 0; pb <= bg_deg - pa; ++pb) {
            c.curv_a = pa;
            c.curv_b = pb;
            if (launch_tile(MODE_CURV, m, grid0, c, s) != hipSuccess) return DIA_E_HIP;
            ReduceArgs ra;
            std::memset(&ra, 0, sizeof(ra));
            ra.partial = partial;
            ra.nblk = grid0;
            ra.npp = n + 1;
            ra.gt = reinterpret_cast<double*>(nbase + NL.hv) + (size_t)bg_index(pa, pb, bg_deg) * (n + 1);
            ra.n = n;
            ra.m = m;
            if (launch_reduce(ra, s) != hipSuccess) return DIA_E_HIP;
        }
    HessArgs ha;
    std::memset(&ha, 0, sizeof(ha));
    ha.R = R.data;
    ha.ldR = R.ld;
    ha.h = reinterpret_cast<const double*>(nbase + NL.h);
    ha.rows = R.rows;
    ha.cols = R.cols;
    ha.partial = reinterpret_cast<double*>(nbase + NL.hpart);
    if (launch_hess(m, ha, s) != hipSuccess) return DIA_E_HIP;
    if (launch_hess_assemble(ha.partial, NL.splits, NL.npb, m, nb, reinterpret_cast<const double*>(nbase + NL.hv), H,
                             reg, damp, s) != hipSuccess)
        return DIA_E_HIP;
    return DIA_OK;
}

int newton_polish(const dia_image& R, const dia_image& I, const ObjParams& obj, double reg, int m, int bg_deg,
                  int grid, int variant,
                  FitState* st, const FitVecs& v, double* partial, char* nbase, const NewtonLayout& NL,
                  int max_steps, bool quadratic, hipStream_t s, NewtonOutcome* out) {
    const int n = m * m + bg_terms(bg_deg);
    double* th = reinterpret_cast<double*>(nbase + NL.th);
    double* d = reinterpret_cast<double*>(nbase + NL.d);
    double* H = reinterpret_cast<double*>(nbase + NL.H);
    double* info = reinterpret_cast<double*>(nbase + NL.info);
    double* gt = reinterpret_cast<double*>(nbase + NL.gt);
    *out = NewtonOutcome();
    if (!NL.has_H) return DIA_E_ARG;
    if (launch_theta_from_x(st, v, n, s) != hipSuccess) return DIA_E_HIP;
    if (hipMemcpyAsync(th, v.theta_eval64, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return DIA_E_HIP;
    if (!eval_into(R, I, obj, reg, m, bg_deg, grid, variant, v.theta_eval, v.theta_eval64, partial, gt, s)) return DIA_E_HIP;
    ++out->evals;
    double L = 0.0;
    if (!read_back(&L, gt + n, sizeof(double), s)) return DIA_E_HIP;
    if (!std::isfinite(L)) return DIA_E_NONFINITE;
    int form0 = quadratic ? 1 : 0;  // the first Hessian form to try; later steps start at the last that factored
    // Chord steps: a quadratic loss keeps its first factor throughout (its Hessian is constant).  For
    // the others, after a full step (alpha = 1) the next step reuses the factor of the point before;
    // a reused factor is kept while its full steps shrink the decrement at least fourfold each, and
    // is replaced by a fresh one as soon as a step falls short of that.
    bool reuse_next = false;
    double dec_prev = 0.0;
    for (int it = 0; it < max_steps; ++it) {
        const bool factor = (it == 0) || (!quadratic && !reuse_next);
        double hinfo[4];
        // The exact Hessian (quadratic convergence; a Huber or model-variance loss makes the
        // Gauss-Newton form only linearly convergent); where it is not positive definite, the
        // positive Gauss-Newton / IRLS form (a quadratic loss has one form: exact == Gauss-Newton);
        // where even that fails in FP64 (a reference PSF so wide that the kernel's high-frequency
        // modes have curvature below the rounding of the rest), that form with its diagonal scaled
        // by 1 + 1e-12, 1e-9, 1e-6 (Levenberg-Marquardt).  The FP64 line search keeps every accepted
        // step a decrease of the true loss.
        static const double kDamp[] = {0.0, 1e-12, 1e-9, 1e-6};
        for (int form = form0; form < 5; ++form) {
            if (factor) {
                const int rc = hessian_into(R, I, obj, reg, m, bg_deg, v.theta_eval, v.theta_eval64, form == 0 ? 1 : 0,
                                            partial, nbase, NL, H, s, form == 0 ? 0.0 : kDamp[form - 1]);
                if (rc != DIA_OK) return rc;
                ++out->evals;
                ++out->hessians;
            }
            if (launch_chol_solve(H, n, factor ? 1 : 0, gt, th, d, info, s) != hipSuccess) return DIA_E_HIP;
            if (!read_back(hinfo, info, sizeof(hinfo), s)) return DIA_E_HIP;
            if (hinfo[0] == 0.0 || !factor) {
                form0 = form;
                break;
            }
        }
        if (hinfo[0] != 0.0) break;  // not positive definite: keep the current point
        const double dec = hinfo[1];
        const bool fast = factor || dec <= 0.25 * dec_prev;  // (a chord step's progress)
        dec_prev = dec;
        // a negligible predicted decrease ends the polish at once
        if (!(dec > 2e-12 * (std::fabs(L) + 1.0))) {
            out->converged = 1;
            break;
        }
        // a step that moves every parameter by at most two FP32 spacings (the fit is stored in FP32:
        // nothing finer can be represented), or by at most 3e-8 of the largest parameter, is still
        // taken through the line search below; the polish ends after it
        const bool last = hinfo[2] <= 3e-8 || hinfo[3] <= 2.0;
        bool accepted = false;
        double alpha = 1.0;
        for (int ls = 0; ls < 8; ++ls, alpha *= 0.5) {
            if (launch_newton_trial(th, d, alpha, v.theta_eval, v.theta_eval64, n, s) != hipSuccess) return DIA_E_HIP;
            if (!eval_into(R, I, obj, reg, m, bg_deg, grid, variant, v.theta_eval, v.theta_eval64, partial, gt, s))
                return DIA_E_HIP;
            ++out->evals;
            double Lt = 0.0;
            if (!read_back(&Lt, gt + n, sizeof(double), s)) return DIA_E_HIP;
            if (std::isfinite(Lt) && Lt <= L - 1e-4 * alpha * dec) {
                if (hipMemcpyAsync(th, v.theta_eval64, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
                    return DIA_E_HIP;
                // a decrease at the rounding level of the FP64 loss sum (millions of terms):
                // the gradient is at its noise floor, and further steps only chase that noise
                if (L - Lt <= 1e-13 * (std::fabs(L) + 1.0)) out->converged = 1;
                L = Lt;
                accepted = true;
                break;
            }
        }
        if (!accepted) {
            if (!factor && !quadratic) {
                // a reused factor whose step no trial accepts: a fresh one from the same point (this
                // try does not count as a step); the trials overwrote gt, so the gradient there is
                // evaluated again
                if (launch_newton_trial(th, d, 0.0, v.theta_eval, v.theta_eval64, n, s) != hipSuccess)
                    return DIA_E_HIP;
                if (!eval_into(R, I, obj, reg, m, bg_deg, grid, variant, v.theta_eval, v.theta_eval64, partial, gt, s))
                    return DIA_E_HIP;
                ++out->evals;
                reuse_next = false;
                --it;
                continue;
            }
            // no trial point lowers the loss: at the resolution of FP32 parameters when the predicted
            // decrease is already tiny against the loss
            if (last || dec <= 1e-10 * (std::fabs(L) + 1.0)) out->converged = 1;
            if (launch_newton_trial(th, d, 0.0, v.theta_eval, v.theta_eval64, n, s) != hipSuccess) return DIA_E_HIP;
            break;
        }
        reuse_next = alpha == 1.0 && fast;
        ++out->steps;
        if (last) out->converged = 1;
        if (out->converged) break;
    }
    if (launch_set_x(st, v, th, n, L, s) != hipSuccess) return DIA_E_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? DIA_OK : DIA_E_HIP;
}

}  // namespace dia

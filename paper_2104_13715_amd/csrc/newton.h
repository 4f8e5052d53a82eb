// Exact-Hessian Newton polish of a fit and the observed Fisher information (Section 2.5).
#pragma once

#include "fit_state.h"

namespace dia {

constexpr int kMaxTheta = DIA_MAX_M * DIA_MAX_M + kMaxBgTerms;  // parameters: the taps and the largest background

// reg = lambda N_data adds the smoothness penalty's Hessian 2 reg L L (Section 2.7) to the kernel block;
// damp scales the diagonal by 1 + damp (Levenberg-Marquardt damping of a numerically singular H).
hipError_t launch_hess_assemble(const double* partial, int splits, int npb, int m, int nb, const double* hv,
                                double* H, double reg, double damp, hipStream_t s);
hipError_t launch_chol_solve(double* A, int n, int factor, const double* g, const double* th, double* d, double* info,
                             hipStream_t s);
// Sigma = F^-1 with the validity flag (Section 2.5); A holds F on entry (factored in place),
// W (n x n) is scratch; S (n x n), sigma (n), sigma_P (1, over the first nk parameters), info (3)
// are the outputs.
hipError_t launch_covariance(double* A, int n, int nk, double* W, double* S, double* sigma, double* sigma_P,
                             double* info, hipStream_t s);
hipError_t launch_newton_trial(const double* th, const double* d, double alpha, float* theta, double* theta64, int n,
                               hipStream_t s);
hipError_t launch_set_x(FitState* st, FitVecs v, const double* th, int n, double L, hipStream_t s);
hipError_t launch_theta_from_x(const FitState* st, FitVecs v, int n, hipStream_t s);

// Workspace of one Newton polish or one Hessian (byte offsets from its start), sized for the largest
// background (n = m*m + kMaxBgTerms).  part: partial rows of the fused pass for this image (only
// when the caller has none of its own); H: the n x n matrix (only when the caller does not supply
// it); hv: one curvature-weighted row per background term.
struct NewtonLayout {
    size_t h = 0, hpart = 0, H = 0, hv = 0, d = 0, th = 0, info = 0, gt = 0, part = 0, total = 0;
    int splits = 0, npb = 0;
    bool has_part = false, has_H = false;
};
NewtonLayout newton_layout(int m, int rows, int cols, bool own_partial, bool own_H);

// Hessian of the loss at (theta, theta64) into H (n x n row-major, FP64).  exact = 1: d2L itself;
// exact = 0: the positive Gauss-Newton / IRLS form used for Newton steps.  partial: partial rows
// with room for the default tile shape's grid.  reg = lambda N_data of the smoothness penalty; damp
// scales the diagonal by 1 + damp (0 for the Hessian itself).
// bg_deg: degree of the background (0 = the scalar B0; H is then (m*m + bg_terms) square).
int hessian_into(const dia_image& R, const dia_image& I, const ObjParams& obj, double reg, int m, int bg_deg,
                 const float* theta, const double* theta64, int exact, double* partial, char* nbase,
                 const NewtonLayout& NL, double* H, hipStream_t s, double damp = 0.0);

struct NewtonOutcome {
    int steps = 0;      // accepted Newton steps
    int evals = 0;      // fused passes spent (loss evaluations and Hessians)
    int hessians = 0;   // Hessians formed
    int converged = 0;  // decrement or step below the resolution of the FP32 parameters
};

// Newton steps from the optimiser point x of a finished fit (st, v) until the Newton decrement is
// negligible (at most max_steps).  Leaves x and st->L at the result.  quadratic: the Hessian does
// not depend on theta (Gaussian objective, variance fixed), so it is factored once.
int newton_polish(const dia_image& R, const dia_image& I, const ObjParams& obj, double reg, int m, int bg_deg,
                  int grid, int variant,
                  FitState* st, const FitVecs& v, double* partial, char* nbase, const NewtonLayout& NL,
                  int max_steps, bool quadratic, hipStream_t s, NewtonOutcome* out);

}  // namespace dia

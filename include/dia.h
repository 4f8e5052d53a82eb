/*
 * dia.h — C ABI of the MI355X (gfx950) DIA kernel-fit library, libdia.so.
 *
 * The library fits the model image of Hitchcock et al. (PyTorchDIA),
 * Section 2.1, eq. (model_image_delta_basis):
 *
 *     M_ij = sum_{a,b} K_ab R_{(i+a)(j+b)} + B0,      a, b = 0 .. m-1,
 *
 * to a target image I on the same pixel grid, by minimising a scalar
 * objective (Section 2.3 eq. loss, Section 2.4 eq. huber_nll, or a Cauchy
 * drop-in) with Adam followed by L-BFGS (Section 2.3, Section 2.9, the
 * algorithm of Section 2.10).  Every step runs in hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are row-major float32: element (r, c) is data[r * ld + c], ld >= cols.
 * - R and I have the same rows and cols.  Only "valid" target pixels enter
 *   the fit (Section 2.1: pixels closer than half a kernel to an edge are
 *   excluded): valid output (i, j), 0 <= i <= rows-m, 0 <= j <= cols-m, is
 *   target pixel (i + h, j + h) with h = (m - 1) / 2.
 * - theta is m*m + 1 floats: K row-major (K[a*m + b], a = row offset,
 *   b = column offset, the kernel centre at a = b = h), then B0.  With a
 *   polynomial background of degree d >= 1 (dia_objective.bg_degree) it is
 *   m*m + (d+1)(d+2)/2 values: K, then the background coefficients, b_00
 *   where B0 was; "n" below is that length and gradients, Hessians and fits
 *   follow the same layout.
 * - m is odd, 1 <= m <= DIA_MAX_M.
 * - Array arguments are DEVICE pointers owned by the caller, except where a
 *   comment says "host".  Option and result structs are host memory.
 * - stream is a hipStream_t (NULL = the default stream).
 * - The library allocates no device memory: callers pass a workspace of at
 *   least dia_workspace_size() bytes, 256-byte aligned.  Its contents need no
 *   initialisation and are scratch after the call.  Two calls that overlap in
 *   time must not share a workspace.
 * - Return value: 0 success, > 0 warning, < 0 error.  Arguments are checked
 *   before anything is enqueued, so an argument error has no side effects.
 *   No C++ exception crosses this interface.
 * - Reductions run in a fixed order (no float atomics): identical calls give
 *   bitwise-identical results.
 */
#ifndef DIA_H
#define DIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DIA_MAX_M 49
#define DIA_MAX_BG_DEGREE 4     /* highest degree of the polynomial background (Section 2.6)         */

/* status codes */
#define DIA_OK 0
#define DIA_W_NOT_CONVERGED 1   /* iteration cap hit; theta holds the last accepted iterate      */
#define DIA_E_ARG (-1)          /* NULL pointer, unknown enum, option out of range                */
#define DIA_E_SIZE (-2)         /* m even, < 1 or > DIA_MAX_M; image smaller than m; ld < cols    */
#define DIA_E_WORKSPACE (-3)    /* workspace NULL, misaligned or smaller than dia_workspace_size  */
#define DIA_E_HIP (-4)          /* a HIP runtime call failed                                      */
#define DIA_E_NONFINITE (-5)    /* the loss or gradient became NaN or infinite                    */
#define DIA_E_SCRATCH (-6)      /* dia_loss_grad_noalloc: the call needs more workspace than the
                                   library's static scratch, DIA_NOALLOC_SCRATCH_BYTES          */

/* An image in device memory. */
typedef struct {
    const float* data;
    int32_t rows, cols;
    int64_t ld; /* elements between row starts, >= cols */
} dia_image;

/* Loss shape rho(z), z = (I - M) / sigma:
 *   GAUSS  : z^2 / 2                            (eq. chi_squared, eq. loss)
 *   HUBER  : z^2/2 if |z| <= c else c(|z| - c/2) (eq. huber_loss, eq. huber_nll)
 *   CAUCHY : (c^2/2) ln(1 + z^2/c^2)             (a wide-tailed drop-in, Section 2.4) */
enum { DIA_RHO_GAUSS = 0, DIA_RHO_HUBER = 1, DIA_RHO_CAUCHY = 2 };

/* Source of the pixel variance sigma^2 (F = flat field, 1 if none):
 *   WEIGHTS     : sigma^2 = 1 / weights                                    fixed
 *   CCD_DATA    : max(sigma0^2/F^2 + max(I,0)/(G F), var_floor)            fixed  (eq. CCDNM on I)
 *   CCD_MODEL   : max(sigma0^2/F^2 + max(M,0)/(G F), var_floor)            (eq. CCDNM)
 *   EMCCD_DATA  : max(E max(I,0)/(G F), var_floor)                         fixed  (eq. EMCCDNM on I)
 *   EMCCD_MODEL : max(E max(M,0)/(G F), var_floor)                         (eq. EMCCDNM)
 * When sigma depends on the model, each pixel adds ln sigma (eq. loss,
 * eq. huber_nll); for fixed sigma that term is a constant and is left out. */
enum { DIA_VAR_WEIGHTS = 0, DIA_VAR_CCD_DATA = 1, DIA_VAR_CCD_MODEL = 2,
       DIA_VAR_EMCCD_DATA = 3, DIA_VAR_EMCCD_MODEL = 4 };

typedef struct {
    int32_t rho;       /* DIA_RHO_*                                             */
    int32_t var;       /* DIA_VAR_*                                             */
    double sigma0;     /* read noise, ADU (CCD)                                 */
    double gain;       /* G, e-/ADU (CCD) or G_Total (EMCCD), > 0               */
    double excess;     /* E, the EMCCD excess noise factor                       */
    double var_floor;  /* lower bound on sigma^2, ADU^2, >= 0                    */
    double c;          /* Huber or Cauchy scale, > 0                             */
    /* Optional arrays laid out like the target (same rows, cols and ld).       */
    const float* weights;  /* 1/sigma^2; required for DIA_VAR_WEIGHTS, else NULL */
    const float* flat;     /* master flat F; NULL means F = 1                    */
    const uint8_t* mask;   /* nonzero = pixel used; NULL means every valid pixel */
    /* Kernel-smoothness penalty of Section 2.7 (eq. regularised_loss): the loss
     * gains lambda N_data theta^T L^T L theta, L the Laplacian of eq. laplacian
     * over the kernel pixels (pixels sharing a side are adjacent; B0 is not
     * penalised) and N_data the number of valid-region pixels.  lambda >= 0;
     * 0 is the maximum-likelihood fit.  The single-pair entry points
     * (dia_loss_grad, dia_hessian, dia_fit) include it in the loss, gradient and
     * Hessian; the batched ones require lambda = 0 (DIA_E_ARG otherwise). */
    double lambda;
    /* Differential background of Section 2.6 (eq. polybackground): 0 = the
     * scalar B0; d = 1 .. DIA_MAX_BG_DEGREE = the polynomial
     *     B(x, y) = sum over a + b <= d of b_ab eta^a xi^b,
     * eta = (x - x_c) / N_x, xi = (y - y_c) / N_y (eq. normcoords), x the
     * target column, y the target row, (x_c, y_c) = ((cols - 1)/2, (rows - 1)/2)
     * and N_x = cols, N_y = rows.  theta then holds the m*m kernel taps and the
     * (d+1)(d+2)/2 coefficients in the equation's summation order (a = 0..d
     * outer, b = 0..d-a inner), b_00 in B0's place; the smoothness penalty
     * leaves every coefficient free.  Single-pair entry points only (the
     * batched ones require 0); dia_fit requires max_outer = 1 with d >= 1. */
    int32_t bg_degree;
} dia_objective;

/* Operations for dia_workspace_size. */
enum { DIA_OP_MODEL = 0, DIA_OP_LOSS_GRAD = 1, DIA_OP_FIT = 2, DIA_OP_FIT_CLIPPED = 3, DIA_OP_HESSIAN = 4,
       DIA_OP_COVARIANCE = 5 };

/* Workspace bytes that dia_loss_grad (DIA_OP_LOSS_GRAD) or dia_fit
 * (DIA_OP_FIT; DIA_OP_FIT_CLIPPED when opts->max_outer > 1) need for an image
 * of rows x cols with leading dimension ld and an m x m kernel
 * (DIA_OP_COVARIANCE: n = m*m + 1 parameters; rows, cols and ld are not used).
 * Returns DIA_E_ARG / DIA_E_SIZE on bad input. */
int dia_workspace_size(int32_t op, int32_t rows, int32_t cols, int64_t ld, int32_t m, size_t* bytes /*host*/);

/* Model image, eq. (model_image_delta_basis), on the valid region:
 * M[i * ldM + j], i < rows-m+1, j < cols-m+1, ldM >= cols-m+1.
 * Asynchronous on stream; needs no workspace. */
int dia_model(dia_image R, const float* theta, int32_t m, float* M, int64_t ldM, void* stream);

/* dia_model with the polynomial background of Section 2.6 (eq. model_image
 * with eq. polybackground): theta holds m*m + (d+1)(d+2)/2 values for
 * bg_degree = d (see dia_objective.bg_degree; the coordinates are those of
 * R's grid, rows x cols).  bg_degree = 0 is dia_model. */
int dia_model_bg(dia_image R, const float* theta, int32_t m, int32_t bg_degree, float* M, int64_t ldM,
                 void* stream);

/* One fused forward + objective + backward pass (the residual is never
 * written to memory).  The tile shape is the one the fits use for this kernel
 * size and image-size class: the first call for a new (m, size class) in a
 * process times the compiled shapes on this data, synchronising the stream
 * once (DIA_TILE_VARIANT=k pins shape k, DIA_AUTOTUNE=0 keeps the default;
 * shapes: 0 the default rows per thread, 1 / 2 / 3 one / two / four rows per
 * thread where the LDS budget allows, 4 two sets of threads with one row each
 * (eight waves per workgroup), 5 a narrow tile for small images; 1-5 are
 * compiled for m = 9, 17, 19, 25):
 *   *loss   = L(theta)  summed over valid, unmasked pixels, FP64      (device double[1])
 *   grad[k] = dL/dK_k = sum_p g_p R_(p + k),  grad[m*m] = dL/dB0 = sum_p g_p,
 *             g_p = d l_p / d M_p                                      (device float[n])
 *   with a polynomial background grad[m*m + j] = sum_p g_p eta_p^a xi_p^b for
 *   the j-th coefficient b_ab.  A polynomial background always uses the
 *   default tile shape.
 * Asynchronous on stream. */
int dia_loss_grad(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m,
                  double* loss, float* grad, void* ws, size_t ws_bytes, void* stream);

/* dia_loss_grad with FP64 parameters and gradient: theta is device double[m*m+1]
 * (same layout), grad receives the FP64 reduction, device double[m*m+1].  The
 * fused pass computes in FP64 from FP64 parameters in either form; this one
 * skips the FP32 rounding of theta and of the gradient, for callers that
 * iterate in FP64 (an FP64 autograd parameter, a line search at points closer
 * than the FP32 spacing).  Same workspace (DIA_OP_LOSS_GRAD) and tile-shape
 * choice as dia_loss_grad.  Asynchronous on stream. */
int dia_loss_grad64(dia_image R, dia_image I, const dia_objective* obj, const double* theta, int32_t m,
                    double* loss, double* grad, void* ws, size_t ws_bytes, void* stream);

/* dia_loss_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and kernels as dia_loss_grad, without the workspace:
 * the partial rows and the reduced gradient live in a static device array of
 * the library, DIA_NOALLOC_SCRATCH_BYTES on every GPU the library's kernels
 * are loaded on, held until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree, stream or event): the tile shape is one already chosen by an
 * earlier call for this kernel size and image-size class, else the default
 * shape; nothing is timed.  The first call on a GPU looks the array up there
 * (hipGetSymbolAddress) under a lock.  Returns DIA_E_SCRATCH, before anything
 * is enqueued, when dia_workspace_size(DIA_OP_LOSS_GRAD, ...) exceeds
 * DIA_NOALLOC_SCRATCH_BYTES (every image fits for m <= 31).  Every call on
 * one GPU uses that GPU's one array: calls that overlap in time on one GPU
 * (two streams, two host threads) race and must be ordered by the caller; a
 * call leaves the array holding its own partial sums, and each call writes
 * every word it later reads, so nothing needs clearing.  Asynchronous on
 * stream. */
#define DIA_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int dia_loss_grad_noalloc(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m,
                          double* loss, float* grad, void* stream);

/* The tile shape a single-pair call uses for an m x m kernel on a rows x cols
 * image (host): the autotuner's choice for that kernel size and image-size
 * class if it has been made in this process (or pinned by DIA_TILE_VARIANT),
 * else the default shape (variant 0).  variant is the shape's index (see
 * dia_loss_grad), tile_rows x tile_cols the valid outputs per workgroup. */
int dia_tile_shape(int32_t m, int32_t rows, int32_t cols, int32_t* variant, int32_t* tile_rows, int32_t* tile_cols);

/* Observed Fisher information (Section 2.5): the Hessian of L at theta,
 *   H[i * n + j] = d2L / dtheta_i dtheta_j,   n = m*m + 1 (m*m + (d+1)(d+2)/2
 * with a polynomial background of degree d),
 * FP64, row-major, parameters in theta's order (kernel taps row by row, then
 * B0 or the background coefficients); device double[n * n].  Since M is
 * affine in theta,
 *   H = sum_p (d2 l_p / dM_p^2) x_p x_p^T,  x_p = (R_(p + k) for every tap k, 1)
 *   (with a polynomial background the 1 becomes eta_p^a xi_p^b for each term),
 * computed exactly (including the derivative of the variance when it
 * depends on the model).  When L is a negative log-likelihood, H^-1 is the
 * asymptotic covariance of the fitted parameters and sqrt(H^-1[m*m][m*m])
 * the standard error of B0.  Workspace: DIA_OP_HESSIAN.  Asynchronous on
 * stream. */
int dia_hessian(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m, double* H,
                void* ws, size_t ws_bytes, void* stream);

/* Kernel initialisation (Section 2.9): FLAT = 1/m^2 everywhere; GAUSS = a
 * symmetric Gaussian of standard deviation init_phi, normalised to sum 1;
 * USER = theta as passed in.  FLAT and GAUSS set B0 = median of I. */
enum { DIA_INIT_FLAT = 0, DIA_INIT_GAUSS = 1, DIA_INIT_USER = 2 };

typedef struct {
    int32_t init;          /* DIA_INIT_*                                                   */
    double init_phi;       /* Gaussian init standard deviation, pixels                     */
    double lr_K, lr_B0;    /* Adam learning rates (paper: 1e-3 and 1, 10 or 100)           */
    double beta1, beta2, eps;  /* Adam moments (Kingma & Ba defaults)                      */
    double tol_switch;     /* hand over to L-BFGS when |dL|/|L| < tol_switch (paper 1e-6)   */
    double tol_change;     /* stop when |dL|/|L| < tol_change over an accepted L-BFGS step  */
    double tol_grad;       /* stop when max|grad| <= tol_grad * max|grad at start|          */
    int32_t history;       /* L-BFGS memory, 1..32                                         */
    int32_t max_adam;      /* Adam steps before the switch is forced                       */
    int32_t max_lbfgs;     /* accepted L-BFGS steps (then DIA_W_NOT_CONVERGED unless the
                              Newton polish below converges); 0 = no L-BFGS phase: the
                              first-order part ends at the Adam switch and the Newton
                              polish (max_newton > 0) takes the fit from there              */
    int32_t max_eval;      /* total objective evaluations before DIA_W_NOT_CONVERGED       */
    int32_t max_outer;     /* fits in the reweight/clip loop (1 = a single fit)            */
    double clip_kappa;     /* clip |z| > clip_kappa between fits; 0 = no clipping          */
    int32_t poll_every;    /* graph replays between host checks of the done flag          */
    int32_t max_newton;    /* exact-Hessian Newton steps after each fit (0 = none)         */
} dia_fit_opts;

/* Covariance of the fitted parameters from the observed Fisher information
 * (Section 2.5, eq. covmatrix): for F = dia_hessian's H at the fit (device
 * double[n*n], n = m*m + 1, symmetric; not modified; see dia_covariance_bg
 * for a polynomial background),
 *   cov     = F^-1                           (device double[n*n], row-major)
 *   sigma   = sqrt(diag cov), the Cramer-Rao error of each parameter (eq. deltatheta)
 *                                            (device double[n])
 *   sigma_P = sqrt(sum over kernel taps i, j of cov[i][j]), the error of the
 *             photometric scale factor P = sum K   (device double[1])
 *   info    = [valid, ln det cov, smallest Cholesky pivot of F]   (device double[3])
 * valid = 1 when F is positive definite (its Cholesky factorisation exists),
 * which is the paper's validity test of cov: then every eigenvalue of cov and
 * its determinant are positive.  valid = 0 means cov is not a covariance
 * matrix; the other outputs are then NaN.  Computed in FP64: F = L L^T in one
 * workgroup, W = L^-1, cov = W^T W.  Workspace: DIA_OP_COVARIANCE (two n x n
 * FP64 matrices).  Asynchronous on stream. */
int dia_covariance(const double* F, int32_t m, double* cov, double* sigma, double* sigma_P, double* info, void* ws,
                   size_t ws_bytes, void* stream);

/* dia_covariance for a fit with the polynomial background of Section 2.6:
 * F is n x n with n = m*m + (d+1)(d+2)/2 for bg_degree = d (dia_hessian's H
 * with dia_objective.bg_degree = d); sigma_P still sums over the m*m kernel
 * taps.  Same workspace (DIA_OP_COVARIANCE covers every degree). */
int dia_covariance_bg(const double* F, int32_t m, int32_t bg_degree, double* cov, double* sigma, double* sigma_P,
                      double* info, void* ws, size_t ws_bytes, void* stream);

/* Fill opts with the paper's settings (Section 2.9): flat init, lr_K 1e-3,
 * lr_B0 10, tol_switch 1e-6, L-BFGS lr 1 with history 10, tol_change 1e-8,
 * tol_grad 1e-9, at most 5000 Adam and 500 L-BFGS steps, one outer fit; then
 * up to 8 Newton steps.
 *
 * The Newton polish is an addition to the paper's optimiser: at m ~ 19 the
 * normal matrix of the problem has a condition number near 1e10, so the
 * first-order optimisers stop on the paper's rule well before the kernel's
 * weak directions have converged.  Each Newton step solves H d = -g with the
 * FP64 Hessian H = sum_p h_p x_p x_p^T (x_p the pixel's design row, h_p the
 * exact per-pixel curvature; where that H is not positive definite, the
 * Gauss-Newton / IRLS weight) by Cholesky, with a backtracking
 * line search on the loss (trial points evaluated at their unrounded FP64
 * values).  A quadratic loss factors H once; for the others a step taken in
 * full lets the next reuse the factor of the point before, for as long as
 * each such step shrinks -g.d fourfold (n_hessian counts the factors
 * formed).  The polish stops when the Newton decrement -g.d is below
 * the FP64 resolution of the loss, the step below the FP32 resolution of
 * theta, or an accepted step lowers the loss by no more than 1e-13 |L| (the
 * rounding level of the loss summed over millions of pixels: the gradient
 * is then at its noise floor). */
void dia_fit_opts_default(dia_fit_opts* opts /*host*/);

typedef struct {
    /* loss, P and B0 belong to the optimiser's final FP64 iterate; the returned
     * theta is that iterate rounded to FP32 (sum K of the rounded kernel can
     * differ from P by up to 2^-24 sum |K|) */
    double loss;      /* final L, FP64 reduction                        */
    double P;         /* photometric scale factor sum K, FP64 (eq. photometric_scale_factor) */
    double B0;
    int32_t n_eval;   /* objective evaluations, all outer fits          */
    int32_t n_adam;   /* Adam steps                                     */
    int32_t n_lbfgs;  /* accepted L-BFGS steps                          */
    int32_t n_outer;  /* fits run by the reweight/clip loop             */
    int64_t n_masked; /* valid pixels excluded by mask and clipping     */
    int32_t stop;     /* why the last fit stopped: 1 rel. change, 2 gradient, 3 line search at
                         precision limit, 4 iteration cap, 5 Newton decrement negligible            */
    int32_t status;   /* same as the return value                       */
    int32_t n_newton; /* accepted Newton steps, all outer fits          */
    int32_t n_hessian; /* Hessians formed by the Newton polish          */
    int32_t first_order_stop; /* why the last fit's Adam -> L-BFGS phase stopped (codes of stop
                                 1 .. 4), before any Newton polish: 4 means that phase hit its
                                 iteration cap even when the polish then converged          */
    int32_t reserved;
} dia_fit_result;

/* Full fit from the chosen initialisation to the stopping rule; theta
 * (device float[m*m+1]) is the start when opts->init == DIA_INIT_USER and
 * receives the fit.  With opts->max_outer > 1 the B08-style loop of
 * Sections 2.1 and 2.4 runs: the first fit uses obj as given (its var must
 * be CCD_* or EMCCD_*), later fits use sigma^2 = v(M_prev) held fixed and,
 * if clip_kappa > 0, drop pixels with |I - M_prev| / sigma > clip_kappa
 * (masks accumulate); the loop ends early when the mask stops changing.
 * Optimiser state lives in the workspace; each optimiser step is a captured
 * hipGraph replay with no host synchronisation (the L-BFGS recursion runs on
 * an LDS copy of its history where it fits; DIA_STEP_LDS=0 keeps it in global
 * memory, with bitwise the same results).  Returns after the work on
 * stream has completed.  res (host) may be NULL. */
int dia_fit(dia_image R, dia_image I, const dia_objective* obj, int32_t m, const dia_fit_opts* opts,
            float* theta, dia_fit_result* res, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Batched fits: many epochs of uneven size against one shared reference.
 * Every epoch is its own independent fit (its own theta, loss and optimiser
 * state, same objective scalars and options); all epochs advance together,
 * one persistent launch per optimiser iteration, and an epoch that has
 * converged drops out of the work queue.  The tile shape is chosen per
 * kernel size and image-size class by a timing autotuner (process-wide
 * cache; DIA_TILE_VARIANT=k pins variant k, DIA_AUTOTUNE_CACHE=<file> keeps
 * the choices across processes) — the analogue of the convolution-algorithm
 * benchmark cache mentioned in the paper's Section 5.3.
 * ------------------------------------------------------------------------ */

/* One epoch: a target and the position of its pixel (0, 0) in the shared reference. */
typedef struct {
    const float* I;            /* target, device                                         */
    int32_t rows, cols;
    int64_t ld;
    int32_t ref_row0, ref_col0; /* target pixel (r, c) sits on reference pixel (r + ref_row0, c + ref_col0) */
    const float* weights;      /* optional arrays laid out like this target (see dia_objective) */
    const float* flat;
    const uint8_t* mask;
} dia_epoch;

/* Arithmetic of the batched contraction.
 *   FP32   : the plain form: direct correlation on the vector ALUs, FP32 images and
 *            parameters widened exactly to FP64, FP64 products and sums (an FP64 FMA
 *            issues at the rate of an unpacked FP32 FMA on gfx950).
 *   BF16X3 : forward and dL/dK as implicit GEMMs over the epochs on BF16 matrix
 *            cores, each FP32 operand split x = hi + lo (both bf16) and the
 *            product taken as hi*hi + hi*lo + lo*hi with FP32 accumulation;
 *            needs every epoch to have the same size and reference offset. */
enum { DIA_PREC_FP32 = 0, DIA_PREC_BF16X3 = 1 };

/* Workspace bytes for dia_loss_grad_batched (fit = 0) or dia_fit_batched (fit = 1). */
int dia_batched_workspace_size(dia_image R, const dia_epoch* epochs /*host[n]*/, int32_t n, int32_t m,
                               int32_t precision, int32_t fit, size_t* bytes /*host*/);

/* Per-epoch loss and gradient at theta[e] (device float[n][m*m+1]):
 * loss[e] (device double[n]), grad[e*(m*m+1) + k] (device float[n][m*m+1]).
 * Asynchronous on stream.  BF16X3 only launches kernels (one per block of 32
 * epochs, the epochs' array pointers passed as kernel arguments) and never
 * waits on the host; FP32 uploads its tile plan and synchronizes stream first.
 * Calls that share ws must be ordered on one stream. */
int dia_loss_grad_batched(dia_image R, const dia_epoch* epochs /*host[n]*/, int32_t n, int32_t m,
                          const dia_objective* obj, int32_t precision, const float* theta, double* loss,
                          float* grad, void* ws, size_t ws_bytes, void* stream);

/* Fit every epoch (see dia_fit; opts->max_outer must be 1).  theta is device
 * float[n][m*m+1] (start values when opts->init == DIA_INIT_USER, fits on
 * return); res is host dia_fit_result[n] or NULL.  Returns the most severe
 * status over the epochs; res[e].status holds each epoch's own.  Returns after
 * the fits have finished; the Newton polishes run up to four epochs at a time,
 * each on a host thread with a stream of its own (on the caller's device) and
 * its own part of ws. */
int dia_fit_batched(dia_image R, const dia_epoch* epochs /*host[n]*/, int32_t n, int32_t m,
                    const dia_objective* obj, const dia_fit_opts* opts, int32_t precision, float* theta,
                    dia_fit_result* res, void* ws, size_t ws_bytes, void* stream);

/* Name of a status code (static string). */
const char* dia_status_string(int status);

/* Library version, major * 10000 + minor * 100 + patch. */
int dia_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DIA_H */

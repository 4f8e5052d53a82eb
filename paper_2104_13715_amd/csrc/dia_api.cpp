// C ABI of libdia, single pair: argument checks, workspace layout and the host
// side of the fit (graph capture and replay).  Everything numeric runs in the
// HIP kernels.
#include "api_util.h"
#include "newton.h"

namespace dia {
namespace {

struct Layout {
    int n = 0, npp = 0, nld = 0, nblk_max = 0;
    size_t partial = 0, gt = 0, th64 = 0, state = 0, sel = 0, vecs = 0, clip_w = 0, clip_mask = 0, ints = 0;
    size_t newton = 0;
    NewtonLayout NL;
    size_t total = 0;
};

Layout make_layout(int op, int rows, int cols, long long ld, int m) {
    Layout L;
    L.n = m * m + kMaxBgTerms;  // room for the largest background; a call uses m*m + bg_terms(bg_degree)
    L.npp = L.n + 1;
    L.nld = (L.n + 63) / 64 * 64;
    const int nt = max_tiles(m, rows, cols);
    L.nblk_max = nt < kMaxGrid ? nt : kMaxGrid;
    size_t off = 0;
    L.partial = off;
    off = align_up(off + sizeof(double) * (size_t)L.nblk_max * L.npp);
    L.gt = off;
    off = align_up(off + sizeof(double) * (size_t)L.npp);
    L.th64 = off;
    off = align_up(off + sizeof(double) * (size_t)L.n);
    if (op == DIA_OP_FIT || op == DIA_OP_FIT_CLIPPED) {
        L.state = off;
        off = align_up(off + sizeof(FitState));
        L.sel = off;
        off = align_up(off + sizeof(SelectState));
        L.vecs = off;
        off = align_up(off + vec_bytes(L.nld));
        L.ints = off;
        off = align_up(off + sizeof(int) * 16);
    }
    if (op == DIA_OP_FIT_CLIPPED) {
        L.clip_w = off;
        off = align_up(off + sizeof(float) * (size_t)rows * ld);
        L.clip_mask = off;
        off = align_up(off + (size_t)rows * ld);
    }
    if (op == DIA_OP_FIT || op == DIA_OP_FIT_CLIPPED || op == DIA_OP_HESSIAN) {
        L.NL = newton_layout(m, rows, cols, /*own_partial=*/false, /*own_H=*/op != DIA_OP_HESSIAN);
        L.newton = off;
        off = align_up(off + L.NL.total);
    }
    L.total = off;
    return L;
}

// Tile-shape variant for a single-pair evaluation, timed on the caller's data once per
// (kernel size, size class); the timing passes write only the workspace's partial rows.
// s must be a stream this library owns (the timing waits on it).
// Each timing covers kTuneBurst passes back to back: a small image's pass (tens of us) is then not
// lost in the launch and event overheads of one.
constexpr int kTuneBurst = 4;

int choose_variant(const TileArgs& a, int m, hipStream_t s) {
    const int sc = size_class((double)(a.rows - m + 1) * (a.cols - m + 1));
    return autotuner().pick(m, sc, /*kind=*/0, [&](int v) -> float {
        const int grid = eval_grid(m, tile_grid_tiles(m, a.rows, a.cols, v), v);
        return time_launches(s, [&]() {
            for (int k = 0; k < kTuneBurst; ++k)
                if (launch_tile(MODE_EVAL, m, grid, a, s, v) != hipSuccess) return false;
            return true;
        });
    });
}

// The same for a call on the caller's stream: the timing runs on a private stream that first waits
// for the work already queued on the caller's stream (it writes the workspace); nothing is timed
// while the caller's stream is being captured into a graph (then a cached choice or the default).
// may_time = false: never time (no stream or event is created), a cached choice or the default.
int choose_variant_for_caller(const TileArgs& a, int m, hipStream_t user, bool may_time = true) {
    const int sc = size_class((double)(a.rows - m + 1) * (a.cols - m + 1));
    if (!may_time || stream_capturing(user)) return autotuner().pick(m, sc, /*kind=*/0, nullptr, kNumVariants, false);
    // a settled choice needs no private stream (and no wait on the caller's work)
    int settled = 0;
    if (autotuner().settled(m, sc, /*kind=*/0, kNumVariants, &settled)) return settled;
    hipStream_t ps = nullptr;
    hipEvent_t ev = nullptr;
    int v = 0;
    if (hipStreamCreateWithFlags(&ps, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess && hipEventRecord(ev, user) == hipSuccess &&
        hipStreamWaitEvent(ps, ev, 0) == hipSuccess) {
        v = choose_variant(a, m, ps);
        (void)hipStreamSynchronize(ps);
    } else {
        v = autotuner().pick(m, sc, /*kind=*/0, nullptr, kNumVariants, false);
    }
    if (ev) (void)hipEventDestroy(ev);
    if (ps) (void)hipStreamDestroy(ps);
    return v;
}

// One fit (init already done on cs): capture poll_every iterations in a graph, replay until done.
int run_fit_graph(const TileArgs& ta, int m, int grid, int variant, const ReduceArgs& ra, int poll_every,
                  int max_eval, hipStream_t cs, FitState* st_dev, FitState* st_host) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = DIA_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return DIA_E_HIP;
    for (int k = 0; k < poll_every; ++k) {
        if (launch_tile(MODE_EVAL, m, grid, ta, cs, variant) != hipSuccess) rc = DIA_E_HIP;
        if (launch_reduce(ra, cs) != hipSuccess) rc = DIA_E_HIP;
    }
    if (hipStreamEndCapture(cs, &graph) != hipSuccess) return DIA_E_HIP;
    if (rc != DIA_OK) {
        (void)hipGraphDestroy(graph);
        return rc;
    }
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return DIA_E_HIP;
    }
    const int max_reps = max_eval / poll_every + 2;
    int done = 0;
    for (int rep = 0; rep < max_reps && !done && rc == DIA_OK; ++rep) {
        if (hipGraphLaunch(exec, cs) != hipSuccess) rc = DIA_E_HIP;
        if (rc == DIA_OK && hipMemcpyAsync(&done, &st_dev->done, sizeof(int), hipMemcpyDeviceToHost, cs) != hipSuccess)
            rc = DIA_E_HIP;
        if (rc == DIA_OK && hipStreamSynchronize(cs) != hipSuccess) rc = DIA_E_HIP;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (rc != DIA_OK) return rc;
    if (hipMemcpyAsync(st_host, st_dev, sizeof(FitState), hipMemcpyDeviceToHost, cs) != hipSuccess) return DIA_E_HIP;
    if (hipStreamSynchronize(cs) != hipSuccess) return DIA_E_HIP;
    if (!done) st_host->status = DIA_W_NOT_CONVERGED, st_host->stop = STOP_CAP;
    return DIA_OK;
}

int fit_impl(const dia_image& R, const dia_image& I, const dia_objective& obj, int m, const dia_fit_opts& o,
             float* theta, dia_fit_result* res, void* ws, hipStream_t user_stream) {
    const int op = o.max_outer > 1 ? DIA_OP_FIT_CLIPPED : DIA_OP_FIT;
    const Layout L = make_layout(op, R.rows, R.cols, I.ld, m);
    char* base = static_cast<char*>(ws);
    FitState* st = reinterpret_cast<FitState*>(base + L.state);
    SelectState* sel = reinterpret_cast<SelectState*>(base + L.sel);
    int* ints = reinterpret_cast<int*>(base + L.ints);
    const FitVecs v = make_vecs(base, L.vecs, L.nld);

    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DIA_E_HIP;
    int rc = DIA_OK;
#define TRY(expr)               \
    if ((expr) != hipSuccess) { \
        rc = DIA_E_HIP;         \
        break;                  \
    }
    do {
        TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        TRY(hipEventRecord(ev, user_stream));
        TRY(hipStreamWaitEvent(cs, ev, 0));
        if (o.init != DIA_INIT_USER) TRY(launch_median(I.data, I.rows, I.cols, I.ld, sel, cs));
        TRY(launch_ref_stats(R.data, R.rows, R.cols, R.ld, sel, cs));
        TRY(launch_init_fit(st, v, m, bg_terms(obj.bg_degree), o.init, o.init_phi, theta, sel, cs));
        TRY(launch_zero_ints(ints, 16, cs));

        FitOptsDev od = opts_dev(o);
        dia_objective cur = obj;
        uint8_t* wmask = nullptr;
        float* wts = nullptr;
        if (op == DIA_OP_FIT_CLIPPED) {
            wmask = reinterpret_cast<uint8_t*>(base + L.clip_mask);
            wts = reinterpret_cast<float*>(base + L.clip_w);
            TRY(launch_fill_mask(wmask, obj.mask, I.rows, I.cols, I.ld, cs));
            cur.mask = wmask;
        }

        // tile shape: timed on this pair at the start point (the default shape with a polynomial background)
        TileArgs tune = base_args(R, I, v.theta_eval);
        tune.theta64 = v.theta_eval64;
        tune.obj = to_params(cur);
        tune.partial = reinterpret_cast<double*>(base + L.partial);
        const int variant = obj.bg_degree > 0 ? 0 : choose_variant(tune, m, cs);
        const int n = n_params(m, obj);
        const int grid = eval_grid(m, tile_grid_tiles(m, R.rows, R.cols, variant), variant);

        int n_eval = 0, n_adam = 0, n_lbfgs = 0, n_outer = 0, n_newton = 0, n_hess = 0, first_stop = 0;
        FitState fs;
        std::memset(&fs, 0, sizeof(fs));
        for (int outer = 0; outer < o.max_outer; ++outer) {
            if (outer > 0) {
                // reweight with sigma^2 = v(M_prev) and clip |z| > kappa (B08 iteration)
                TRY(launch_finalize(st, v, m, theta, cs));
                TileArgs ca = base_args(R, I, theta);
                ca.obj = to_params(obj);
                ca.obj.mask = wmask;
                ca.w_out = wts;
                ca.mask_out = wmask;
                ca.kappa = (float)o.clip_kappa;
                ca.clip_count = ints + outer;
                TRY(launch_tile(MODE_CLIP, m, eval_grid(m, tile_grid_tiles(m, R.rows, R.cols)), ca, cs));
                cur = obj;
                cur.var = DIA_VAR_WEIGHTS;
                cur.weights = wts;
                cur.flat = nullptr;
                cur.mask = wmask;
                TRY(launch_restart_fit(st, v, n, cs));
            }
            TileArgs ta = base_args(R, I, v.theta_eval);
            ta.theta64 = v.theta_eval64;
            ta.obj = to_params(cur);
            ta.partial = reinterpret_cast<double*>(base + L.partial);
            ta.done = &st->done;
            set_background(ta, obj.bg_degree, m);
            ReduceArgs ra;
            std::memset(&ra, 0, sizeof(ra));
            ra.partial = ta.partial;
            ra.nblk = grid;
            ra.npp = n + 1;
            ra.gt = reinterpret_cast<double*>(base + L.gt);
            ra.st = st;
            ra.v = v;
            ra.o = od;
            ra.o.skip_adam = outer > 0 ? 1 : 0;
            ra.n = n;
            ra.m = m;
            ra.done = &st->done;
            ra.reg = penalty_weight(obj, I, m);
            ra.th64 = v.theta_eval64;
            const int r = run_fit_graph(ta, m, grid, variant, ra, o.poll_every, o.max_eval, cs, st, &fs);
            if (r != DIA_OK) {
                rc = r;
                break;
            }
            n_eval += fs.n_eval;
            n_adam += fs.n_adam;
            n_lbfgs += fs.n_lbfgs;
            n_outer = outer + 1;
            first_stop = fs.stop;
            if (fs.status < 0) break;
            if (o.max_newton > 0) {
                const bool quad = cur.rho == DIA_RHO_GAUSS && cur.var != DIA_VAR_CCD_MODEL &&
                                  cur.var != DIA_VAR_EMCCD_MODEL;
                NewtonOutcome no;
                const int pr = newton_polish(R, I, to_params(cur), penalty_weight(obj, I, m), m, obj.bg_degree, grid,
                                             variant, st, v,
                                             ta.partial, base + L.newton, L.NL, o.max_newton, quad, cs, &no);
                if (pr != DIA_OK) {
                    rc = pr;
                    break;
                }
                n_eval += no.evals;
                n_newton += no.steps;
                n_hess += no.hessians;
                if (no.converged) {
                    fs.status = DIA_OK;
                    fs.stop = STOP_NEWTON;
                }
            }
            if (outer > 0) {
                int changed = 0;
                TRY(hipMemcpyAsync(&changed, ints + outer, sizeof(int), hipMemcpyDeviceToHost, cs));
                TRY(hipStreamSynchronize(cs));
                if (changed == 0) break;
            }
        }
        if (rc != DIA_OK) break;
        TRY(launch_finalize(st, v, m, theta, cs));
        const uint8_t* final_mask = (op == DIA_OP_FIT_CLIPPED) ? wmask : obj.mask;
        int n_masked = 0;
        if (final_mask != nullptr) TRY(launch_count_masked(final_mask, I.rows, I.cols, I.ld, m, ints + 15, cs));
        FitState fin;
        TRY(hipMemcpyAsync(&fin, st, sizeof(FitState), hipMemcpyDeviceToHost, cs));
        if (final_mask != nullptr) TRY(hipMemcpyAsync(&n_masked, ints + 15, sizeof(int), hipMemcpyDeviceToHost, cs));
        TRY(hipStreamSynchronize(cs));
        rc = fs.status;
        if (res != nullptr) {
            res->loss = fin.out_loss;
            res->P = fin.out_P;
            res->B0 = fin.out_B0;
            res->n_eval = n_eval;
            res->n_adam = n_adam;
            res->n_lbfgs = n_lbfgs;
            res->n_outer = n_outer;
            res->n_masked = n_masked;
            res->stop = fs.stop;
            res->status = rc;
            res->n_newton = n_newton;
            res->n_hessian = n_hess;
            res->first_order_stop = first_stop;
            res->reserved = 0;
        }
    } while (false);
#undef TRY
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    if (res != nullptr && rc < 0) res->status = rc;
    return rc;
}

}  // namespace

// One fused pass and its reduction on the caller's stream.  Exactly one of theta32 / theta64 is given:
// FP32 parameters are widened into the workspace first, FP64 ones are read where they are.
// may_time = false keeps the tile-shape choice to a cached one or the default (nothing is timed,
// no stream or event is created).
int loss_grad_impl(const dia_image& R, const dia_image& I, const dia_objective* obj, const float* theta32,
                   const double* theta64, int m, double* loss, float* grad32, double* grad64, void* ws,
                   size_t ws_bytes, void* stream, bool may_time) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if ((theta32 == nullptr && theta64 == nullptr) || loss == nullptr || (grad32 == nullptr && grad64 == nullptr))
        return DIA_E_ARG;
    const Layout L = make_layout(DIA_OP_LOSS_GRAD, R.rows, R.cols, I.ld, m);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    char* base = static_cast<char*>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = n_params(m, *obj);
    TileArgs a = base_args(R, I, theta32);
    const double* th64 = theta64;
    if (th64 == nullptr) {
        double* w = reinterpret_cast<double*>(base + L.th64);
        if (launch_widen(theta32, w, n, s) != hipSuccess) return DIA_E_HIP;
        th64 = w;
    }
    a.theta64 = th64;
    a.obj = to_params(*obj);
    a.partial = reinterpret_cast<double*>(base + L.partial);
    set_background(a, obj->bg_degree, m);
    // the tile shape the fits use for this kernel and image size (timed once per process on the first
    // call for a size class, on a private stream; the timing passes write only the workspace's partial rows)
    const int variant = obj->bg_degree > 0 ? 0 : choose_variant_for_caller(a, m, s, may_time);
    const int grid = eval_grid(m, tile_grid_tiles(m, R.rows, R.cols, variant), variant);
    if (launch_tile(MODE_EVAL, m, grid, a, s, variant) != hipSuccess) return DIA_E_HIP;
    ReduceArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.partial = a.partial;
    ra.nblk = grid;
    ra.npp = n + 1;
    ra.gt = reinterpret_cast<double*>(base + L.gt);
    ra.out_loss = loss;
    ra.out_grad = grad32;
    ra.out_grad64 = grad64;
    ra.n = n;
    ra.m = m;
    ra.reg = penalty_weight(*obj, I, m);
    ra.th64 = th64;
    return launch_reduce(ra, s) == hipSuccess ? DIA_OK : DIA_E_HIP;
}

}  // namespace dia

using namespace dia;

extern "C" {

int dia_version(void) { return 1 * 10000 + 1 * 100 + 0; }

const char* dia_status_string(int status) {
    switch (status) {
        case DIA_OK: return "DIA_OK";
        case DIA_W_NOT_CONVERGED: return "DIA_W_NOT_CONVERGED: iteration cap reached";
        case DIA_E_ARG: return "DIA_E_ARG: invalid argument";
        case DIA_E_SIZE: return "DIA_E_SIZE: invalid size (m even/out of range, image smaller than m, ld < cols)";
        case DIA_E_WORKSPACE: return "DIA_E_WORKSPACE: workspace missing, misaligned or too small";
        case DIA_E_HIP: return "DIA_E_HIP: HIP runtime error";
        case DIA_E_NONFINITE: return "DIA_E_NONFINITE: loss or gradient not finite";
        case DIA_E_SCRATCH:
            return "DIA_E_SCRATCH: the call needs more than the library's static scratch (DIA_NOALLOC_SCRATCH_BYTES)";
        default: return "unknown status";
    }
}

// the covariance region: F factored in place, then W = L^-1
static size_t covariance_bytes(int m) {
    const size_t n = (size_t)m * m + kMaxBgTerms;
    return 2 * align_up(sizeof(double) * n * n);
}

int dia_workspace_size(int32_t op, int32_t rows, int32_t cols, int64_t ld, int32_t m, size_t* bytes) {
    if (bytes == nullptr) return DIA_E_ARG;
    if (op == DIA_OP_COVARIANCE) {
        if (m < 1 || m > DIA_MAX_M || m % 2 == 0) return DIA_E_SIZE;
        *bytes = covariance_bytes(m);
        return DIA_OK;
    }
    if (op < DIA_OP_MODEL || op > DIA_OP_HESSIAN) return DIA_E_ARG;
    if (rows < 1 || cols < 1 || ld < cols) return DIA_E_SIZE;
    const int c = check_m(m, rows, cols);
    if (c != DIA_OK) return c;
    if (op == DIA_OP_MODEL) {
        *bytes = 0;
        return DIA_OK;
    }
    *bytes = make_layout(op, rows, cols, ld, m).total;
    return DIA_OK;
}

int dia_model_bg(dia_image R, const float* theta, int32_t m, int32_t bg_degree, float* M, int64_t ldM, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if (theta == nullptr || M == nullptr) return DIA_E_ARG;
    if (bg_degree < 0 || bg_degree > DIA_MAX_BG_DEGREE) return DIA_E_ARG;
    if (ldM < R.cols - m + 1) return DIA_E_SIZE;
    TileArgs a = base_args(R, R, theta);
    a.out = M;
    a.ld_out = ldM;
    set_background(a, bg_degree, m);
    const int grid = eval_grid(m, tile_grid_tiles(m, R.rows, R.cols));
    return launch_tile(MODE_MODEL, m, grid, a, static_cast<hipStream_t>(stream)) == hipSuccess ? DIA_OK : DIA_E_HIP;
}

int dia_model(dia_image R, const float* theta, int32_t m, float* M, int64_t ldM, void* stream) {
    return dia_model_bg(R, theta, m, 0, M, ldM, stream);
}

int dia_loss_grad(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m, double* loss,
                  float* grad, void* ws, size_t ws_bytes, void* stream) {
    return loss_grad_impl(R, I, obj, theta, nullptr, m, loss, grad, nullptr, ws, ws_bytes, stream, true);
}

int dia_loss_grad64(dia_image R, dia_image I, const dia_objective* obj, const double* theta, int32_t m, double* loss,
                    double* grad, void* ws, size_t ws_bytes, void* stream) {
    return loss_grad_impl(R, I, obj, nullptr, theta, m, loss, nullptr, grad, ws, ws_bytes, stream, true);
}

int dia_hessian(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m, double* H,
                void* ws, size_t ws_bytes, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if (theta == nullptr || H == nullptr) return DIA_E_ARG;
    const Layout L = make_layout(DIA_OP_HESSIAN, R.rows, R.cols, I.ld, m);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    char* base = static_cast<char*>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* th64 = reinterpret_cast<double*>(base + L.th64);
    if (launch_widen(theta, th64, n_params(m, *obj), s) != hipSuccess) return DIA_E_HIP;
    try {
        return hessian_into(R, I, to_params(*obj), penalty_weight(*obj, I, m), m, obj->bg_degree, theta, th64,
                            /*exact=*/1,
                            reinterpret_cast<double*>(base + L.partial), base + L.newton, L.NL, H, s);
    } catch (...) {
        return DIA_E_HIP;
    }
}

int dia_covariance_bg(const double* F, int32_t m, int32_t bg_degree, double* cov, double* sigma, double* sigma_P,
                      double* info, void* ws, size_t ws_bytes, void* stream) {
    if (m < 1 || m > DIA_MAX_M || m % 2 == 0) return DIA_E_SIZE;
    if (bg_degree < 0 || bg_degree > DIA_MAX_BG_DEGREE) return DIA_E_ARG;
    if (F == nullptr || cov == nullptr || sigma == nullptr || sigma_P == nullptr || info == nullptr) return DIA_E_ARG;
    const int c = check_ws(ws, ws_bytes, covariance_bytes(m));
    if (c != DIA_OK) return c;
    const int n = m * m + bg_terms(bg_degree);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* A = static_cast<double*>(ws);
    double* W = reinterpret_cast<double*>(static_cast<char*>(ws) + align_up(sizeof(double) * (size_t)n * n));
    if (hipMemcpyAsync(A, F, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return DIA_E_HIP;
    return launch_covariance(A, n, m * m, W, cov, sigma, sigma_P, info, s) == hipSuccess ? DIA_OK : DIA_E_HIP;
}

int dia_covariance(const double* F, int32_t m, double* cov, double* sigma, double* sigma_P, double* info, void* ws,
                   size_t ws_bytes, void* stream) {
    return dia_covariance_bg(F, m, 0, cov, sigma, sigma_P, info, ws, ws_bytes, stream);
}

int dia_tile_shape(int32_t m, int32_t rows, int32_t cols, int32_t* variant, int32_t* tile_rows, int32_t* tile_cols) {
    if (variant == nullptr || tile_rows == nullptr || tile_cols == nullptr) return DIA_E_ARG;
    if (rows < 1 || cols < 1) return DIA_E_SIZE;
    const int c = check_m(m, rows, cols);
    if (c != DIA_OK) return c;
    const int sc = size_class((double)(rows - m + 1) * (cols - m + 1));
    int v = 0;
    if (!autotuner().settled(m, sc, /*kind=*/0, kNumVariants, &v)) v = 0;
    int ty = 0, tx = 0;
    if (tile_dims(m, v, &ty, &tx) != 0) return DIA_E_ARG;
    *variant = v;
    *tile_rows = ty;
    *tile_cols = tx;
    return DIA_OK;
}

void dia_fit_opts_default(dia_fit_opts* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof(*o));
    o->init = DIA_INIT_FLAT;
    o->init_phi = 1.0;
    o->lr_K = 1e-3;
    o->lr_B0 = 10.0;
    o->beta1 = 0.9;
    o->beta2 = 0.999;
    o->eps = 1e-8;
    o->tol_switch = 1e-6;
    o->tol_change = 1e-8;
    o->tol_grad = 1e-9;
    o->history = 10;
    o->max_adam = 5000;
    o->max_lbfgs = 500;
    o->max_eval = 20000;
    o->max_outer = 1;
    o->clip_kappa = 0.0;
    o->poll_every = 16;
    o->max_newton = 8;
}

int dia_fit(dia_image R, dia_image I, const dia_objective* obj, int32_t m, const dia_fit_opts* opts, float* theta,
            dia_fit_result* res, void* ws, size_t ws_bytes, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if ((c = check_opts(opts)) != DIA_OK) return c;
    if (theta == nullptr) return DIA_E_ARG;
    if (opts->max_outer > 1 && obj->var == DIA_VAR_WEIGHTS) return DIA_E_ARG;
    if (opts->max_outer > 1 && obj->bg_degree > 0) return DIA_E_ARG;  // the clip pass has the scalar background
    const int op = opts->max_outer > 1 ? DIA_OP_FIT_CLIPPED : DIA_OP_FIT;
    const Layout L = make_layout(op, R.rows, R.cols, I.ld, m);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    try {
        return fit_impl(R, I, *obj, m, *opts, theta, res, ws, static_cast<hipStream_t>(stream));
    } catch (...) {
        return DIA_E_HIP;
    }
}

}  // extern "C"

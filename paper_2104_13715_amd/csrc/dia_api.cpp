// C ABI of libdia: argument checks, workspace layout and the host side of the
// fit (graph capture and replay).  Everything numeric runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "dia_common.h"
#include "fit_state.h"

namespace dia {
namespace {

constexpr int kMaxGrid = 2048;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int n = 0, npp = 0, nld = 0, ntiles = 0, nblk_max = 0;
    size_t partial = 0, gt = 0, state = 0, sel = 0, vecs = 0, clip_w = 0, clip_mask = 0, ints = 0, total = 0;
};

Layout make_layout(int op, int rows, int cols, long long ld, int m) {
    Layout L;
    L.n = m * m + 1;
    L.npp = L.n + 1;
    L.nld = (L.n + 63) / 64 * 64;
    L.ntiles = tile_grid_tiles(m, rows, cols);
    L.nblk_max = L.ntiles < kMaxGrid ? L.ntiles : kMaxGrid;
    size_t off = 0;
    L.partial = off;
    off = align_up(off + sizeof(double) * (size_t)L.nblk_max * L.npp);
    L.gt = off;
    off = align_up(off + sizeof(double) * (size_t)L.npp);
    if (op == DIA_OP_FIT || op == DIA_OP_FIT_CLIPPED) {
        L.state = off;
        off = align_up(off + sizeof(FitState));
        L.sel = off;
        off = align_up(off + sizeof(SelectState));
        L.vecs = off;
        off = align_up(off + sizeof(double) * ((size_t)(8 + 2 * kMaxHistory) * L.nld + 2 * kMaxHistory) +
                       sizeof(float) * L.nld);
        L.ints = off;
        off = align_up(off + sizeof(int) * 16);
    }
    if (op == DIA_OP_FIT_CLIPPED) {
        L.clip_w = off;
        off = align_up(off + sizeof(float) * (size_t)rows * ld);
        L.clip_mask = off;
        off = align_up(off + (size_t)rows * ld);
    }
    L.total = off;
    return L;
}

FitVecs make_vecs(char* base, const Layout& L) {
    FitVecs v;
    double* p = reinterpret_cast<double*>(base + L.vecs);
    const size_t ld = L.nld;
    v.x = p;
    v.g = p + ld;
    v.d = p + 2 * ld;
    v.xt = p + 3 * ld;
    v.m1 = p + 4 * ld;
    v.v1 = p + 5 * ld;
    v.xp = p + 6 * ld;
    v.gp = p + 7 * ld;
    v.S = p + 8 * ld;
    v.Y = v.S + kMaxHistory * ld;
    v.rh = v.Y + kMaxHistory * ld;
    v.al = v.rh + kMaxHistory;
    v.theta_eval = reinterpret_cast<float*>(v.al + kMaxHistory);
    v.ld = (int)ld;
    return v;
}

bool is_fin(double x) { return std::isfinite(x); }

int check_image(const dia_image& im) {
    if (im.data == nullptr) return DIA_E_ARG;
    if (im.rows < 1 || im.cols < 1 || im.ld < im.cols) return DIA_E_SIZE;
    return DIA_OK;
}

int check_m(int m, int rows, int cols) {
    if (m < 1 || m > DIA_MAX_M || (m % 2) == 0) return DIA_E_SIZE;
    if (rows < m || cols < m) return DIA_E_SIZE;
    return DIA_OK;
}

int check_obj(const dia_objective* o) {
    if (o == nullptr) return DIA_E_ARG;
    if (o->rho < DIA_RHO_GAUSS || o->rho > DIA_RHO_CAUCHY) return DIA_E_ARG;
    if (o->var < DIA_VAR_WEIGHTS || o->var > DIA_VAR_EMCCD_MODEL) return DIA_E_ARG;
    if (o->rho != DIA_RHO_GAUSS && !(o->c > 0.0 && is_fin(o->c))) return DIA_E_ARG;
    if (o->var == DIA_VAR_WEIGHTS) {
        if (o->weights == nullptr) return DIA_E_ARG;
    } else {
        if (!(o->gain > 0.0) || !is_fin(o->gain)) return DIA_E_ARG;
        if (!(o->var_floor >= 0.0) || !is_fin(o->var_floor)) return DIA_E_ARG;
        if (!is_fin(o->sigma0)) return DIA_E_ARG;
        if ((o->var == DIA_VAR_EMCCD_DATA || o->var == DIA_VAR_EMCCD_MODEL) && !(o->excess > 0.0 && is_fin(o->excess)))
            return DIA_E_ARG;
        if ((o->var == DIA_VAR_EMCCD_DATA || o->var == DIA_VAR_EMCCD_MODEL) && !(o->var_floor > 0.0))
            return DIA_E_ARG;  // the EMCCD variance is zero where the signal is zero
        if ((o->var == DIA_VAR_CCD_DATA || o->var == DIA_VAR_CCD_MODEL) && !(o->sigma0 != 0.0 || o->var_floor > 0.0))
            return DIA_E_ARG;
    }
    return DIA_OK;
}

int check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return DIA_OK;
    if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < need) return DIA_E_WORKSPACE;
    return DIA_OK;
}

ObjParams to_params(const dia_objective& o) {
    ObjParams p;
    p.rho = o.rho;
    p.var = o.var;
    p.s0sq = (float)(o.sigma0 * o.sigma0);
    p.inv_gain = o.gain > 0.0 ? (float)(1.0 / o.gain) : 0.0f;
    p.excess = (float)o.excess;
    p.var_floor = (float)o.var_floor;
    p.c = (float)o.c;
    p.inv_c2 = o.c > 0.0 ? (float)(1.0 / (o.c * o.c)) : 0.0f;
    p.weights = o.weights;
    p.flat = o.flat;
    p.mask = o.mask;
    return p;
}

// Persistent grid: as many workgroups as fit on the device at once, balanced so
// that every workgroup walks the same number of tiles.
int eval_grid(int m, int ntiles) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, int> cap_cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    int cap;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cap_cache.find({dev, m});
        if (it == cap_cache.end()) {
            int ncu = 0;
            if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
                ncu = 1;
            int c = ncu * tile_max_blocks_per_cu(m);
            if (c > kMaxGrid) c = kMaxGrid;
            if (c < 1) c = 1;
            it = cap_cache.emplace(std::make_pair(dev, m), c).first;
        }
        cap = it->second;
    }
    if (ntiles <= cap) return ntiles;
    const int waves = (ntiles + cap - 1) / cap;
    return (ntiles + waves - 1) / waves;
}

TileArgs base_args(const dia_image& R, const dia_image& I, const float* theta) {
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.R = R.data;
    a.ldR = R.ld;
    a.I = I.data;
    a.ldI = I.ld;
    a.rows = R.rows;
    a.cols = R.cols;
    a.theta = theta;
    return a;
}

#define HIP_TRY(expr)                         \
    do {                                      \
        if ((expr) != hipSuccess) return DIA_E_HIP; \
    } while (0)

struct FitRun {
    int n_eval = 0, n_adam = 0, n_lbfgs = 0, stop = 0, status = DIA_OK;
    FitState last;
};

// One fit (init already done on cs): capture poll_every iterations in a graph, replay until done.
int run_fit_graph(const TileArgs& ta, int m, int grid, const ReduceArgs& ra, int poll_every, int max_eval,
                  hipStream_t cs, FitState* st_dev, FitState* st_host) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = DIA_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return DIA_E_HIP;
    for (int k = 0; k < poll_every; ++k) {
        if (launch_tile(MODE_EVAL, m, grid, ta, cs) != hipSuccess) rc = DIA_E_HIP;
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
    const FitVecs v = make_vecs(base, L);
    const int grid = eval_grid(m, L.ntiles);

    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int rc = DIA_OK;
    auto fail = [&](int code) {
        rc = code;
        return code;
    };
    do {
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { fail(DIA_E_HIP); break; }
        if (hipEventRecord(ev, user_stream) != hipSuccess) { fail(DIA_E_HIP); break; }
        if (hipStreamWaitEvent(cs, ev, 0) != hipSuccess) { fail(DIA_E_HIP); break; }

        if (o.init != DIA_INIT_USER && launch_median(I.data, I.rows, I.cols, I.ld, sel, cs) != hipSuccess) {
            fail(DIA_E_HIP);
            break;
        }
        if (launch_init_fit(st, v, m, o.init, o.init_phi, theta, sel, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
        if (launch_zero_ints(ints, 16, cs) != hipSuccess) { fail(DIA_E_HIP); break; }

        FitOptsDev od;
        od.lr_K = o.lr_K;
        od.lr_B0 = o.lr_B0;
        od.beta1 = o.beta1;
        od.beta2 = o.beta2;
        od.eps = o.eps;
        od.tol_switch = o.tol_switch;
        od.tol_change = o.tol_change;
        od.tol_grad = o.tol_grad;
        od.history = o.history;
        od.max_adam = o.max_adam;
        od.max_lbfgs = o.max_lbfgs;
        od.max_eval = o.max_eval;
        od.skip_adam = 0;

        dia_objective cur = obj;
        uint8_t* wmask = nullptr;
        float* wts = nullptr;
        if (op == DIA_OP_FIT_CLIPPED) {
            wmask = reinterpret_cast<uint8_t*>(base + L.clip_mask);
            wts = reinterpret_cast<float*>(base + L.clip_w);
            if (launch_fill_mask(wmask, obj.mask, I.rows, I.cols, I.ld, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
            cur.mask = wmask;
        }

        int n_eval = 0, n_adam = 0, n_lbfgs = 0, n_outer = 0;
        FitState fs;
        std::memset(&fs, 0, sizeof(fs));
        for (int outer = 0; outer < o.max_outer; ++outer) {
            if (outer > 0) {
                // reweight with sigma^2 = v(M_prev) and clip |z| > kappa (B08 iteration)
                TileArgs ca = base_args(R, I, v.theta_eval);
                dia_objective vobj = obj;
                ca.obj = to_params(vobj);
                ca.obj.mask = wmask;
                ca.w_out = wts;
                ca.mask_out = wmask;
                ca.kappa = (float)o.clip_kappa;
                ca.clip_count = ints + outer;
                if (launch_finalize(st, v, m, theta, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
                ca.theta = theta;
                if (launch_tile(MODE_CLIP, m, grid, ca, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
                cur = obj;
                cur.var = DIA_VAR_WEIGHTS;
                cur.weights = wts;
                cur.flat = nullptr;
                cur.mask = wmask;
                if (launch_restart_fit(st, v, L.n, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
            }
            TileArgs ta = base_args(R, I, v.theta_eval);
            ta.obj = to_params(cur);
            ta.partial = reinterpret_cast<double*>(base + L.partial);
            ta.done = &st->done;
            ReduceArgs ra;
            std::memset(&ra, 0, sizeof(ra));
            ra.partial = ta.partial;
            ra.nblk = grid;
            ra.npp = L.npp;
            ra.gt = reinterpret_cast<double*>(base + L.gt);
            ra.st = st;
            ra.v = v;
            ra.o = od;
            ra.o.skip_adam = outer > 0 ? 1 : 0;
            ra.n = L.n;
            ra.m = m;
            ra.done = &st->done;
            const int r = run_fit_graph(ta, m, grid, ra, o.poll_every, o.max_eval, cs, st, &fs);
            if (r != DIA_OK) { fail(r); break; }
            n_eval += fs.n_eval;
            n_adam += fs.n_adam;
            n_lbfgs += fs.n_lbfgs;
            n_outer = outer + 1;
            if (fs.status < 0) break;
            if (outer > 0) {
                int changed = 0;
                if (hipMemcpyAsync(&changed, ints + outer, sizeof(int), hipMemcpyDeviceToHost, cs) != hipSuccess ||
                    hipStreamSynchronize(cs) != hipSuccess) {
                    fail(DIA_E_HIP);
                    break;
                }
                if (changed == 0) break;
            }
        }
        if (rc != DIA_OK) break;
        if (launch_finalize(st, v, m, theta, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
        const uint8_t* final_mask = (op == DIA_OP_FIT_CLIPPED) ? wmask : obj.mask;
        int n_masked = 0;
        if (final_mask != nullptr) {
            if (launch_count_masked(final_mask, I.rows, I.cols, I.ld, m, ints + 15, cs) != hipSuccess) {
                fail(DIA_E_HIP);
                break;
            }
        }
        FitState fin;
        if (hipMemcpyAsync(&fin, st, sizeof(FitState), hipMemcpyDeviceToHost, cs) != hipSuccess) { fail(DIA_E_HIP); break; }
        if (final_mask != nullptr &&
            hipMemcpyAsync(&n_masked, ints + 15, sizeof(int), hipMemcpyDeviceToHost, cs) != hipSuccess) {
            fail(DIA_E_HIP);
            break;
        }
        if (hipStreamSynchronize(cs) != hipSuccess) { fail(DIA_E_HIP); break; }
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
        }
    } while (false);
    if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    if (res != nullptr && rc < 0) res->status = rc;
    return rc;
}

}  // namespace
}  // namespace dia

using namespace dia;

extern "C" {

int dia_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char* dia_status_string(int status) {
    switch (status) {
        case DIA_OK: return "DIA_OK";
        case DIA_W_NOT_CONVERGED: return "DIA_W_NOT_CONVERGED: iteration cap reached";
        case DIA_E_ARG: return "DIA_E_ARG: invalid argument";
        case DIA_E_SIZE: return "DIA_E_SIZE: invalid size (m even/out of range, image smaller than m, ld < cols)";
        case DIA_E_WORKSPACE: return "DIA_E_WORKSPACE: workspace missing, misaligned or too small";
        case DIA_E_HIP: return "DIA_E_HIP: HIP runtime error";
        case DIA_E_NONFINITE: return "DIA_E_NONFINITE: loss or gradient not finite";
        default: return "unknown status";
    }
}

int dia_workspace_size(int32_t op, int32_t rows, int32_t cols, int64_t ld, int32_t m, size_t* bytes) {
    if (bytes == nullptr) return DIA_E_ARG;
    if (op < DIA_OP_MODEL || op > DIA_OP_FIT_CLIPPED) return DIA_E_ARG;
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

int dia_model(dia_image R, const float* theta, int32_t m, float* M, int64_t ldM, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if (theta == nullptr || M == nullptr) return DIA_E_ARG;
    if (ldM < R.cols - m + 1) return DIA_E_SIZE;
    TileArgs a = base_args(R, R, theta);
    a.out = M;
    a.ld_out = ldM;
    const int grid = eval_grid(m, tile_grid_tiles(m, R.rows, R.cols));
    return launch_tile(MODE_MODEL, m, grid, a, static_cast<hipStream_t>(stream)) == hipSuccess ? DIA_OK : DIA_E_HIP;
}

int dia_loss_grad(dia_image R, dia_image I, const dia_objective* obj, const float* theta, int32_t m, double* loss,
                  float* grad, void* ws, size_t ws_bytes, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if (theta == nullptr || loss == nullptr || grad == nullptr) return DIA_E_ARG;
    const Layout L = make_layout(DIA_OP_LOSS_GRAD, R.rows, R.cols, I.ld, m);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    char* base = static_cast<char*>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int grid = eval_grid(m, L.ntiles);
    TileArgs a = base_args(R, I, theta);
    a.obj = to_params(*obj);
    a.partial = reinterpret_cast<double*>(base + L.partial);
    if (launch_tile(MODE_EVAL, m, grid, a, s) != hipSuccess) return DIA_E_HIP;
    ReduceArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.partial = a.partial;
    ra.nblk = grid;
    ra.npp = L.npp;
    ra.gt = reinterpret_cast<double*>(base + L.gt);
    ra.out_loss = loss;
    ra.out_grad = grad;
    ra.n = L.n;
    ra.m = m;
    return launch_reduce(ra, s) == hipSuccess ? DIA_OK : DIA_E_HIP;
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
    o->tol_change = 1e-10;
    o->tol_grad = 1e-9;
    o->history = 10;
    o->max_adam = 5000;
    o->max_lbfgs = 2000;
    o->max_eval = 20000;
    o->max_outer = 1;
    o->clip_kappa = 0.0;
    o->poll_every = 16;
}

int dia_fit(dia_image R, dia_image I, const dia_objective* obj, int32_t m, const dia_fit_opts* opts, float* theta,
            dia_fit_result* res, void* ws, size_t ws_bytes, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if (opts == nullptr || theta == nullptr) return DIA_E_ARG;
    const dia_fit_opts& o = *opts;
    if (o.init < DIA_INIT_FLAT || o.init > DIA_INIT_USER) return DIA_E_ARG;
    if (o.init == DIA_INIT_GAUSS && !(o.init_phi > 0.0 && is_fin(o.init_phi))) return DIA_E_ARG;
    if (!(o.lr_K > 0.0) || !(o.lr_B0 > 0.0) || !is_fin(o.lr_K) || !is_fin(o.lr_B0)) return DIA_E_ARG;
    if (!(o.beta1 >= 0.0 && o.beta1 < 1.0) || !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps >= 0.0)) return DIA_E_ARG;
    if (!(o.tol_switch >= 0.0) || !(o.tol_change >= 0.0) || !(o.tol_grad >= 0.0)) return DIA_E_ARG;
    if (o.history < 1 || o.history > kMaxHistory) return DIA_E_ARG;
    if (o.max_adam < 1 || o.max_lbfgs < 1 || o.max_eval < 1 || o.max_outer < 1 || o.poll_every < 1) return DIA_E_ARG;
    if (o.poll_every > 1024) return DIA_E_ARG;
    if (!(o.clip_kappa >= 0.0) || !is_fin(o.clip_kappa)) return DIA_E_ARG;
    if (o.max_outer > 1 && obj->var == DIA_VAR_WEIGHTS) return DIA_E_ARG;
    const int op = o.max_outer > 1 ? DIA_OP_FIT_CLIPPED : DIA_OP_FIT;
    const Layout L = make_layout(op, R.rows, R.cols, I.ld, m);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    try {
        return fit_impl(R, I, *obj, m, o, theta, res, ws, static_cast<hipStream_t>(stream));
    } catch (...) {
        return DIA_E_HIP;
    }
}

}  // extern "C"

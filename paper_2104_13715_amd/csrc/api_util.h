// Host-side helpers shared by the single-pair and batched C-ABI entry points:
// argument checks, objective conversion, grid sizing and the tile-shape autotuner.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dia_common.h"
#include "fit_state.h"

namespace dia {

constexpr int kMaxGrid = 2048;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline bool is_fin(double x) { return std::isfinite(x); }

inline int check_image(const dia_image& im) {
    if (im.data == nullptr) return DIA_E_ARG;
    if (im.rows < 1 || im.cols < 1 || im.ld < im.cols) return DIA_E_SIZE;
    return DIA_OK;
}

inline int check_m(int m, int rows, int cols) {
    if (m < 1 || m > DIA_MAX_M || (m % 2) == 0) return DIA_E_SIZE;
    if (rows < m || cols < m) return DIA_E_SIZE;
    return DIA_OK;
}

inline int check_obj(const dia_objective* o, bool need_weights_ptr = true) {
    if (o == nullptr) return DIA_E_ARG;
    if (o->rho < DIA_RHO_GAUSS || o->rho > DIA_RHO_CAUCHY) return DIA_E_ARG;
    if (o->var < DIA_VAR_WEIGHTS || o->var > DIA_VAR_EMCCD_MODEL) return DIA_E_ARG;
    if (o->rho != DIA_RHO_GAUSS && !(o->c > 0.0 && is_fin(o->c))) return DIA_E_ARG;
    if (!(o->lambda >= 0.0) || !is_fin(o->lambda)) return DIA_E_ARG;
    if (o->bg_degree < 0 || o->bg_degree > DIA_MAX_BG_DEGREE) return DIA_E_ARG;
    if (o->var == DIA_VAR_WEIGHTS) {
        if (need_weights_ptr && o->weights == nullptr) return DIA_E_ARG;
    } else {
        if (!(o->gain > 0.0) || !is_fin(o->gain)) return DIA_E_ARG;
        if (!(o->var_floor >= 0.0) || !is_fin(o->var_floor)) return DIA_E_ARG;
        if (!is_fin(o->sigma0)) return DIA_E_ARG;
        const bool em = (o->var == DIA_VAR_EMCCD_DATA || o->var == DIA_VAR_EMCCD_MODEL);
        if (em && !(o->excess > 0.0 && is_fin(o->excess))) return DIA_E_ARG;
        if (em && !(o->var_floor > 0.0)) return DIA_E_ARG;  // the EMCCD variance is zero where the signal is
        if (!em && !(o->sigma0 != 0.0 || o->var_floor > 0.0)) return DIA_E_ARG;
    }
    return DIA_OK;
}

// lambda N_data of the kernel-smoothness penalty (Section 2.7, eq. regularised_loss), N_data the
// number of valid-region pixels of the target.
inline double penalty_weight(const dia_objective& o, const dia_image& I, int m) {
    return o.lambda * (double)(I.rows - m + 1) * (double)(I.cols - m + 1);
}

inline int check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (need == 0) return DIA_OK;
    if (ws == nullptr || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < need) return DIA_E_WORKSPACE;
    return DIA_OK;
}

inline int check_opts(const dia_fit_opts* opts) {
    if (opts == nullptr) return DIA_E_ARG;
    const dia_fit_opts& o = *opts;
    if (o.init < DIA_INIT_FLAT || o.init > DIA_INIT_USER) return DIA_E_ARG;
    if (o.init == DIA_INIT_GAUSS && !(o.init_phi > 0.0 && is_fin(o.init_phi))) return DIA_E_ARG;
    if (!(o.lr_K > 0.0) || !(o.lr_B0 > 0.0) || !is_fin(o.lr_K) || !is_fin(o.lr_B0)) return DIA_E_ARG;
    if (!(o.beta1 >= 0.0 && o.beta1 < 1.0) || !(o.beta2 >= 0.0 && o.beta2 < 1.0) || !(o.eps >= 0.0)) return DIA_E_ARG;
    if (!(o.tol_switch >= 0.0) || !(o.tol_change >= 0.0) || !(o.tol_grad >= 0.0)) return DIA_E_ARG;
    if (o.history < 1 || o.history > kMaxHistory) return DIA_E_ARG;
    if (o.max_adam < 1 || o.max_lbfgs < 0 || o.max_eval < 1 || o.max_outer < 1 || o.poll_every < 1) return DIA_E_ARG;
    if (o.poll_every > 1024) return DIA_E_ARG;
    if (o.max_newton < 0 || o.max_newton > 1000) return DIA_E_ARG;
    if (!(o.clip_kappa >= 0.0) || !is_fin(o.clip_kappa)) return DIA_E_ARG;
    return DIA_OK;
}

inline FitOptsDev opts_dev(const dia_fit_opts& o) {
    FitOptsDev od;
    std::memset(&od, 0, sizeof(od));
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
    return od;
}

inline ObjParams to_params(const dia_objective& o) {
    ObjParams p;
    p.rho = o.rho;
    p.var = o.var;
    p.s0sq = o.sigma0 * o.sigma0;
    p.inv_gain = o.gain > 0.0 ? 1.0 / o.gain : 0.0;
    p.excess = o.excess;
    p.var_floor = o.var_floor;
    p.c = o.c;
    p.inv_c2 = o.c > 0.0 ? 1.0 / (o.c * o.c) : 0.0;
    p.weights = o.weights;
    p.flat = o.flat;
    p.mask = o.mask;
    return p;
}

inline TileArgs base_args(const dia_image& R, const dia_image& I, const float* theta) {
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.R = R.data;
    a.ldR = R.ld;
    a.I = I.data;
    a.ldI = I.ld;
    a.rows = R.rows;
    a.cols = R.cols;
    a.theta = theta;
    a.nb = 1;
    return a;
}

// The background of a call: degree d (0 = the scalar B0) and, for d >= 1, the normalised coordinates
// of eq. normcoords at the valid pixels: eta = (x - x_c) / N_x with x = ox + h the target column,
// x_c = (N_x - 1) / 2 the centre and N_x = cols the target's width; xi the same along the rows.
inline void set_background(TileArgs& a, int d, int m) {
    const int h = (m - 1) / 2;
    a.bg_deg = d;
    a.nb = bg_terms(d);
    a.deta = 1.0 / (double)a.cols;
    a.eta0 = ((double)h - 0.5 * (double)(a.cols - 1)) / (double)a.cols;
    a.dxi = 1.0 / (double)a.rows;
    a.xi0 = ((double)h - 0.5 * (double)(a.rows - 1)) / (double)a.rows;
}

// Parameters of a single-pair call: m*m kernel taps and the background coefficients.
inline int n_params(int m, const dia_objective& o) { return m * m + bg_terms(o.bg_degree); }

// Optimiser vectors of one fit: 8 vectors, the L-BFGS history (S, Y, rho, alpha) and theta_eval.
inline size_t vec_bytes(int nld) {
    return sizeof(double) * ((size_t)(9 + 2 * kMaxHistory) * nld + 2 * kMaxHistory) + sizeof(float) * nld;
}

inline FitVecs make_vecs(char* base, size_t at, int nld) {
    FitVecs v;
    double* p = reinterpret_cast<double*>(base + at);
    const size_t ld = nld;
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
    v.theta_eval64 = v.al + kMaxHistory;
    v.theta_eval = reinterpret_cast<float*>(v.theta_eval64 + ld);
    v.ld = (int)ld;
    return v;
}

// Largest tile count over the compiled tile-shape variants (sizes the partial rows).
inline int max_tiles(int m, int rows, int cols) {
    int mx = 0;
    for (int v = 0; v < kNumVariants; ++v) {
        if (tile_variant_rb(m, v) == 0) continue;
        const int t = tile_grid_tiles(m, rows, cols, v);
        if (t > mx) mx = t;
    }
    return mx;
}

inline int device_id() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return dev;
}

// Workgroups that fit on the device at once for a variant (cached per device).
inline int resident_blocks(int m, int variant, bool batched) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int>, int> cache;
    const int dev = device_id();
    std::lock_guard<std::mutex> lk(mu);
    auto key = std::make_tuple(dev, m, variant, batched ? 1 : 0);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
    int c = ncu * tile_max_blocks_per_cu(m, variant, batched);
    if (c > kMaxGrid) c = kMaxGrid;
    if (c < 1) c = 1;
    cache[key] = c;
    return c;
}

// Persistent grid for a single pair: as many workgroups as are resident.  One-set shapes are
// balanced so every workgroup walks the same number of tiles; two-set shapes keep every resident
// workgroup, since the kernel splits the tiles of a short last round into half tiles (so that no CU
// holds more than its share of the work, whichever workgroups it runs).
inline int eval_grid(int m, int ntiles, int variant = 0) {
    const int cap = resident_blocks(m, variant, false);
    if (ntiles <= cap) return ntiles;
    if (tile_variant_sets(m, variant) == 2) return cap;
    const int waves = (ntiles + cap - 1) / cap;
    return (ntiles + waves - 1) / waves;
}

// ---------------------------------------------------------------------------- autotuner
// Times each compiled tile-shape variant once on the caller's data and keeps the
// fastest per (device, kernel size, image-size class, kind).  DIA_TILE_VARIANT pins a
// variant; DIA_AUTOTUNE=0 keeps the default; DIA_AUTOTUNE_CACHE names a text file that
// stores the choices ("device m size_class kind variant" per line).
inline int size_class(double pixels_per_item) {
    int c = 0;
    while (pixels_per_item >= 2.0 && c < 40) {
        pixels_per_item *= 0.5;
        ++c;
    }
    return c;
}

struct Autotuner {
    std::mutex mu;
    std::map<std::tuple<std::string, int, int, int>, int> cache;
    bool loaded = false;

    // the architecture name of the current device (looked up once per device)
    static std::string device_name() {
        static std::mutex nmu;
        static std::map<int, std::string> names;
        const int dev = device_id();
        std::lock_guard<std::mutex> lk(nmu);
        auto it = names.find(dev);
        if (it != names.end()) return it->second;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
        std::string s = p.gcnArchName;
        for (auto& ch : s)
            if (ch == ' ') ch = '_';
        names[dev] = s;
        return s;
    }

    void load_locked() {
        if (loaded) return;
        loaded = true;
        const char* path = std::getenv("DIA_AUTOTUNE_CACHE");
        if (!path) return;
        FILE* f = std::fopen(path, "r");
        if (!f) return;
        char name[128];
        int m, sc, kind, v;
        while (std::fscanf(f, "%127s %d %d %d %d", name, &m, &sc, &kind, &v) == 5) cache[{name, m, sc, kind}] = v;
        std::fclose(f);
    }

    void store_locked(const std::string& name, int m, int sc, int kind, int v) {
        const char* path = std::getenv("DIA_AUTOTUNE_CACHE");
        if (!path) return;
        FILE* f = std::fopen(path, "a");
        if (!f) return;
        std::fprintf(f, "%s %d %d %d %d\n", name.c_str(), m, sc, kind, v);
        std::fclose(f);
    }

    // time_fn(variant) returns the measured milliseconds (< 0 on failure).
    // The choice that needs no timing, if there is one: a pinned variant, the default when tuning is
    // off, or a cached choice.
    bool settled(int m, int sc, int kind, int n_variants, int* v) {
        if (const char* pin = std::getenv("DIA_TILE_VARIANT")) {
            const int p = std::atoi(pin);
            if (p >= 0 && p < n_variants && tile_variant_rb(m, p) != 0) return *v = p, true;
        }
        if (const char* at = std::getenv("DIA_AUTOTUNE"))
            if (std::atoi(at) == 0) return *v = 0, true;
        const std::string name = device_name();
        std::lock_guard<std::mutex> lk(mu);
        load_locked();
        auto it = cache.find({name, m, sc, kind});
        if (it != cache.end() && it->second < n_variants && tile_variant_rb(m, it->second) != 0)
            return *v = it->second, true;
        return false;
    }

    // Variants 0 .. n_variants - 1 are candidates (the batched kinds leave out the narrow shape).
    // may_time = false (a call being captured into a graph): a cached choice or the default, nothing
    // timed and nothing cached.  A choice is cached only when every candidate was timed.
    int pick(int m, int sc, int kind, const std::function<float(int)>& time_fn, int n_variants = kNumVariants,
             bool may_time = true) {
        if (const char* pin = std::getenv("DIA_TILE_VARIANT")) {
            const int v = std::atoi(pin);
            if (v >= 0 && v < n_variants && tile_variant_rb(m, v) != 0) return v;
        }
        if (const char* at = std::getenv("DIA_AUTOTUNE"))
            if (std::atoi(at) == 0) return 0;
        const std::string name = device_name();
        {
            std::lock_guard<std::mutex> lk(mu);
            load_locked();
            auto it = cache.find({name, m, sc, kind});
            if (it != cache.end() && it->second < n_variants && tile_variant_rb(m, it->second) != 0) return it->second;
        }
        if (!may_time) return 0;
        // distinct effective shapes only: the same tile (height, width) with the same forward rows per
        // thread and threads per workgroup is the same kernel (a variant whose requested rows do not fit
        // the LDS budget falls back to the default's); the two-thread-set shape has the default's tile
        // with other rows per thread, the split-kernel-row shapes twice the threads of a one-row tile
        std::vector<int> cand;
        std::vector<std::tuple<int, int, int, int>> seen;
        for (int v = 0; v < n_variants; ++v) {
            int ty = 0, tx = 0;
            if (tile_dims(m, v, &ty, &tx) != 0) continue;
            const auto key = std::make_tuple(ty, tx, tile_variant_rb(m, v), tile_variant_threads(m, v));
            bool dup = false;
            for (const auto& d : seen) dup |= (d == key);
            if (dup) continue;
            seen.push_back(key);
            cand.push_back(v);
        }
        // kRounds rounds over the candidates, each candidate's fastest time kept: the clock drifts while
        // the candidates run one after another, and interleaving them keeps that drift from picking one
        constexpr int kRounds = 3;
        int best = 0;
        float best_ms = 1e30f;
        bool all_timed = true;
        if (cand.size() > 1) {
            std::vector<float> fastest(cand.size(), 1e30f);
            for (int r = 0; r < kRounds; ++r)
                for (size_t i = 0; i < cand.size(); ++i) {
                    const float ms = time_fn(cand[i]);
                    all_timed = all_timed && ms >= 0.0f;
                    if (ms >= 0.0f && ms < fastest[i]) fastest[i] = ms;
                }
            for (size_t i = 0; i < cand.size(); ++i)
                if (fastest[i] < best_ms) {
                    best_ms = fastest[i];
                    best = cand[i];
                }
        }
        if (!all_timed) return best;
        std::lock_guard<std::mutex> lk(mu);
        cache[{name, m, sc, kind}] = best;
        store_locked(name, m, sc, kind, best);
        return best;
    }
};

inline Autotuner& autotuner() {
    static Autotuner t;
    return t;
}

// Whether s is being captured into a graph (then nothing may be timed or waited for on it).
inline bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
    return st != hipStreamCaptureStatusNone;
}

// Fastest of a few timed runs of fn on stream s, in milliseconds (-1 on error).
inline float time_launches(hipStream_t s, const std::function<bool()>& fn, int reps = 3) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.0f;
    float best = 1e30f;
    bool ok = fn();  // warm-up
    for (int r = 0; r < reps && ok; ++r) {
        ok = hipEventRecord(a, s) == hipSuccess;
        ok = ok && fn();
        ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ok ? best : -1.0f;
}

// One fused pass and its reduction on the caller's stream (dia_api.cpp); see dia_loss_grad.
int loss_grad_impl(const dia_image& R, const dia_image& I, const dia_objective* obj, const float* theta32,
                   const double* theta64, int m, double* loss, float* grad32, double* grad64, void* ws,
                   size_t ws_bytes, void* stream, bool may_time);

}  // namespace dia

// C ABI of libdia, batched epochs: every epoch is an independent fit against a crop
// of one shared reference; all epochs advance together, one persistent launch per
// optimiser iteration.
#include <atomic>
#include <thread>

#include "api_util.h"
#include "bf16x3.h"
#include "newton.h"

namespace dia {
namespace {

constexpr int kTargetChunks = 4096;  // work items per launch (load balance of the work queue)

struct Plan {
    std::vector<ChunkDev> chunks;
    std::vector<int> cbeg, cend, ntx;
};

Plan make_plan(int m, const dia_epoch* ep, int n, int variant) {
    Plan p;
    int ty = 0, tx = 0;
    tile_dims(m, variant, &ty, &tx);
    std::vector<int> tiles(n);
    long long total = 0;
    p.ntx.resize(n);
    for (int e = 0; e < n; ++e) {
        const int Hv = ep[e].rows - m + 1, Wv = ep[e].cols - m + 1;
        p.ntx[e] = (Wv + tx - 1) / tx;
        tiles[e] = ((Hv + ty - 1) / ty) * p.ntx[e];
        total += tiles[e];
    }
    const int per = (int)std::max<long long>(1, (total + kTargetChunks - 1) / kTargetChunks);
    p.cbeg.resize(n);
    p.cend.resize(n);
    for (int e = 0; e < n; ++e) {
        p.cbeg[e] = (int)p.chunks.size();
        for (int t = 0; t < tiles[e]; t += per) p.chunks.push_back(ChunkDev{e, t, std::min(tiles[e], t + per), 0});
        p.cend[e] = (int)p.chunks.size();
    }
    return p;
}

// The batched forms use the wide tile shapes only: every epoch descriptor carries the tiles across
// for the default tile width, which the narrow shape (variant 5) does not share; many epochs fill
// the chip without it.
constexpr int kBatchedVariants = 5;

int max_chunks(int m, const dia_epoch* ep, int n) {
    int mx = 0;
    for (int v = 0; v < kBatchedVariants; ++v) {
        if (tile_variant_rb(m, v) == 0) continue;
        mx = std::max(mx, (int)make_plan(m, ep, n, v).chunks.size());
    }
    return mx;
}

// Concurrent Newton polishes of a batched fit (each on its own stream and workspace region): the
// per-epoch Hessian fills the chip for large epochs, but the factorisation, the substitutions and
// the host round trips of one epoch leave it mostly idle for small ones.
constexpr int kNewtonLanes = 4;

struct BLayout {
    int n = 0, npp = 0, nld = 0, nchunks = 0;
    size_t partial = 0, gt = 0, th64 = 0, epochs = 0, chunks = 0, cbeg = 0, cend = 0, ints = 0;
    size_t blocks = 0, stride = 0, b_state = 0, b_sel = 0, b_vecs = 0;
    size_t newton = 0;
    size_t newton_each = 0;  // one Newton region per concurrent polish
    size_t total = 0;
};

BLayout make_blayout(const dia_epoch* ep, int n_ep, int m, int precision, bool fit) {
    BLayout L;
    L.n = m * m + 1;
    L.npp = L.n + 1;
    L.nld = (L.n + 63) / 64 * 64;
    L.nchunks = precision == DIA_PREC_FP32 ? max_chunks(m, ep, n_ep) : bf16x3_partial_rows(m, ep[0].rows, ep[0].cols, n_ep);
    size_t off = 0;
    L.partial = off;
    off = align_up(off + sizeof(double) * (size_t)L.nchunks * L.npp);
    L.gt = off;
    off = align_up(off + sizeof(double) * (size_t)n_ep * L.npp);
    L.th64 = off;
    off = align_up(off + sizeof(double) * (size_t)n_ep * L.n);
    L.epochs = off;
    off = align_up(off + sizeof(EpochDev) * (size_t)n_ep);
    L.chunks = off;
    off = align_up(off + sizeof(ChunkDev) * (size_t)std::max(L.nchunks, 1));
    L.cbeg = off;
    off = align_up(off + sizeof(int) * (size_t)n_ep);
    L.cend = off;
    off = align_up(off + sizeof(int) * (size_t)n_ep);
    L.ints = off;
    off = align_up(off + sizeof(int) * 16);
    if (fit) {
        L.b_state = 0;
        L.b_sel = align_up(sizeof(FitState));
        L.b_vecs = L.b_sel + align_up(sizeof(SelectState));
        L.stride = L.b_vecs + align_up(vec_bytes(L.nld));
        L.blocks = off;
        off = align_up(off + L.stride * (size_t)n_ep);
        // Newton polish: kNewtonLanes epochs at a time on their own streams, each lane with its own
        // region (laid out per epoch as that epoch's size needs)
        size_t need = 0;
        for (int e = 0; e < n_ep; ++e)
            need = std::max(need, newton_layout(m, ep[e].rows, ep[e].cols, /*own_partial=*/true, /*own_H=*/true).total);
        L.newton_each = align_up(need);
        L.newton = off;
        off = align_up(off + L.newton_each * (size_t)std::min(kNewtonLanes, std::max(n_ep, 1)));
    }
    L.total = off;
    return L;
}

int check_epochs(const dia_image& R, const dia_epoch* ep, int n, int m, const dia_objective* obj, int precision) {
    if (ep == nullptr || n < 1) return DIA_E_ARG;
    if (precision != DIA_PREC_FP32 && precision != DIA_PREC_BF16X3) return DIA_E_ARG;
    for (int e = 0; e < n; ++e) {
        const dia_epoch& x = ep[e];
        if (x.I == nullptr) return DIA_E_ARG;
        if (x.rows < 1 || x.cols < 1 || x.ld < x.cols) return DIA_E_SIZE;
        const int c = check_m(m, x.rows, x.cols);
        if (c != DIA_OK) return c;
        if (x.ref_row0 < 0 || x.ref_col0 < 0 || (long long)x.ref_row0 + x.rows > R.rows ||
            (long long)x.ref_col0 + x.cols > R.cols)
            return DIA_E_SIZE;
        if (obj != nullptr && obj->var == DIA_VAR_WEIGHTS && x.weights == nullptr) return DIA_E_ARG;
        if (precision == DIA_PREC_BF16X3) {
            const int c2 = bf16x3_check_epoch(ep[0], x, m);
            if (c2 != DIA_OK) return c2;
        }
    }
    return DIA_OK;
}

// Epoch descriptors; the tile width (and so the tiles across) is the same for every variant.
std::vector<EpochDev> epoch_descs(const dia_image& R, const dia_epoch* ep, int n, int m, const float* theta0,
                                  long long theta_stride_bytes, const double* theta64_0, long long theta64_stride_bytes,
                                  const int* done0, long long done_stride_bytes) {
    int ty = 0, tx = 0;
    tile_dims(m, 0, &ty, &tx);
    std::vector<EpochDev> d(n);
    for (int e = 0; e < n; ++e) {
        EpochDev& x = d[e];
        std::memset(&x, 0, sizeof(x));
        x.R = R.data + (long long)ep[e].ref_row0 * R.ld + ep[e].ref_col0;
        x.I = ep[e].I;
        x.ldI = ep[e].ld;
        x.rows = ep[e].rows;
        x.cols = ep[e].cols;
        x.theta = reinterpret_cast<const float*>(reinterpret_cast<const char*>(theta0) + e * theta_stride_bytes);
        x.theta64 =
            reinterpret_cast<const double*>(reinterpret_cast<const char*>(theta64_0) + e * theta64_stride_bytes);
        x.weights = ep[e].weights;
        x.flat = ep[e].flat;
        x.mask = ep[e].mask;
        x.done = reinterpret_cast<const int*>(reinterpret_cast<const char*>(done0) + e * done_stride_bytes);
        x.ntx = (ep[e].cols - m + 1 + tx - 1) / tx;
    }
    return d;
}

// Upload host arrays into the workspace on stream s; the host buffers may go away on return.
bool upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return true;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
}

bool upload_plan(char* base, const BLayout& L, const Plan& p, hipStream_t s) {
    return upload(base + L.chunks, p.chunks.data(), sizeof(ChunkDev) * p.chunks.size(), s) &&
           upload(base + L.cbeg, p.cbeg.data(), sizeof(int) * p.cbeg.size(), s) &&
           upload(base + L.cend, p.cend.data(), sizeof(int) * p.cend.size(), s);
}

int batched_grid(int m, int variant, int n_chunks) {
    const int cap = resident_blocks(m, variant, true);
    return n_chunks < cap ? std::max(n_chunks, 1) : cap;
}

BatchedArgs batched_args(char* base, const BLayout& L, const dia_image& R, const dia_objective& obj, int n_chunks) {
    BatchedArgs b;
    std::memset(&b, 0, sizeof(b));
    b.ep = reinterpret_cast<const EpochDev*>(base + L.epochs);
    b.chunks = reinterpret_cast<const ChunkDev*>(base + L.chunks);
    b.n_chunks = n_chunks;
    b.ldR = R.ld;
    b.obj = to_params(obj);
    b.obj.weights = nullptr;
    b.obj.flat = nullptr;
    b.obj.mask = nullptr;
    b.partial = reinterpret_cast<double*>(base + L.partial);
    b.queue = reinterpret_cast<int*>(base + L.ints);
    return b;
}

// Choose the FP32 tile shape by timing one batched pass per variant (descriptors already uploaded).
int choose_batched_variant(char* base, const BLayout& L, const dia_image& R, const dia_epoch* ep, int n, int m,
                           const dia_objective& obj, hipStream_t s) {
    double px = 0.0;
    for (int e = 0; e < n; ++e) px += (double)(ep[e].rows - m + 1) * (ep[e].cols - m + 1);
    const int sc = size_class(px / n);
    return autotuner().pick(m, sc, /*kind=*/1, [&](int v) -> float {
        const Plan p = make_plan(m, ep, n, v);
        if (!upload_plan(base, L, p, s)) return -1.0f;
        const BatchedArgs b = batched_args(base, L, R, obj, (int)p.chunks.size());
        const int grid = batched_grid(m, v, (int)p.chunks.size());
        return time_launches(s, [&]() {
            return launch_zero_ints(b.queue, 1, s) == hipSuccess && launch_batched_eval(m, grid, b, s, v) == hipSuccess;
        });
    }, kBatchedVariants);
}

}  // namespace
}  // namespace dia

using namespace dia;

extern "C" {

int dia_batched_workspace_size(dia_image R, const dia_epoch* epochs, int32_t n, int32_t m, int32_t precision,
                               int32_t fit, size_t* bytes) {
    if (bytes == nullptr) return DIA_E_ARG;
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_epochs(R, epochs, n, m, nullptr, precision)) != DIA_OK) return c;
    *bytes = make_blayout(epochs, n, m, precision, fit != 0).total;
    return DIA_OK;
}

int dia_loss_grad_batched(dia_image R, const dia_epoch* epochs, int32_t n, int32_t m, const dia_objective* obj,
                          int32_t precision, const float* theta, double* loss, float* grad, void* ws, size_t ws_bytes,
                          void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_obj(obj, false)) != DIA_OK) return c;
    if (obj->lambda != 0.0 || obj->bg_degree != 0) return DIA_E_ARG;  // penalty and polynomial background: single pair
    if ((c = check_epochs(R, epochs, n, m, obj, precision)) != DIA_OK) return c;
    if (theta == nullptr || loss == nullptr || grad == nullptr) return DIA_E_ARG;
    const BLayout L = make_blayout(epochs, n, m, precision, false);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    try {
        int* ints = reinterpret_cast<int*>(base + L.ints);
        int rows_per = 0;
        if (precision == DIA_PREC_BF16X3) {
            // nothing is uploaded: the per-epoch pointers travel in the kernel arguments, and the
            // reduction derives each epoch's partial rows from rows_per
            std::vector<Bf16x3Args> g;
            const int pc = bf16x3_prepare(R, epochs, n, m, *obj, theta, (long long)L.n * sizeof(float),
                                          reinterpret_cast<double*>(base + L.partial), &g);
            if (pc != DIA_OK) return pc;
            if (bf16x3_launch_eval(g, s) != hipSuccess) return DIA_E_HIP;
            rows_per = bf16x3_partial_rows(m, epochs[0].rows, epochs[0].cols, n) / n;
        } else {
            if (hipStreamSynchronize(s) != hipSuccess) return DIA_E_HIP;  // the workspace is free to overwrite
            double* th64 = reinterpret_cast<double*>(base + L.th64);
            if (launch_widen(theta, th64, (long long)n * L.n, s) != hipSuccess) return DIA_E_HIP;
            const std::vector<EpochDev> d = epoch_descs(R, epochs, n, m, theta, (long long)L.n * sizeof(float), th64,
                                                        (long long)L.n * sizeof(double), ints + 2, 0);
            if (!upload(base + L.epochs, d.data(), sizeof(EpochDev) * n, s)) return DIA_E_HIP;
            if (launch_zero_ints(ints, 4, s) != hipSuccess) return DIA_E_HIP;
            const int variant = choose_batched_variant(base, L, R, epochs, n, m, *obj, s);
            const Plan p = make_plan(m, epochs, n, variant);
            if (!upload_plan(base, L, p, s)) return DIA_E_HIP;
            const BatchedArgs b = batched_args(base, L, R, *obj, (int)p.chunks.size());
            if (launch_zero_ints(ints, 4, s) != hipSuccess) return DIA_E_HIP;
            if (launch_batched_eval(m, batched_grid(m, variant, (int)p.chunks.size()), b, s, variant) != hipSuccess)
                return DIA_E_HIP;
        }
        BatchReduceArgs br;
        std::memset(&br, 0, sizeof(br));
        br.partial = reinterpret_cast<const double*>(base + L.partial);
        br.cbeg = rows_per > 0 ? nullptr : reinterpret_cast<const int*>(base + L.cbeg);
        br.cend = rows_per > 0 ? nullptr : reinterpret_cast<const int*>(base + L.cend);
        br.rows_per = rows_per;
        br.npp = L.npp;
        br.gt = reinterpret_cast<double*>(base + L.gt);
        br.out_loss = loss;
        br.out_grad = grad;
        br.n = L.n;
        br.m = m;
        br.queue = ints;
        return launch_reduce_batched(br, n, s) == hipSuccess ? DIA_OK : DIA_E_HIP;
    } catch (...) {
        return DIA_E_HIP;
    }
}

int dia_fit_batched(dia_image R, const dia_epoch* epochs, int32_t n, int32_t m, const dia_objective* obj,
                    const dia_fit_opts* opts, int32_t precision, float* theta, dia_fit_result* res, void* ws,
                    size_t ws_bytes, void* stream) {
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_obj(obj, false)) != DIA_OK) return c;
    if (obj->lambda != 0.0 || obj->bg_degree != 0) return DIA_E_ARG;  // penalty and polynomial background: single pair
    if ((c = check_epochs(R, epochs, n, m, obj, precision)) != DIA_OK) return c;
    if ((c = check_opts(opts)) != DIA_OK) return c;
    if (opts->max_outer != 1 || theta == nullptr) return DIA_E_ARG;
    const BLayout L = make_blayout(epochs, n, m, precision, true);
    if ((c = check_ws(ws, ws_bytes, L.total)) != DIA_OK) return c;
    const dia_fit_opts& o = *opts;
    char* base = static_cast<char*>(ws);
    FitState* st0 = reinterpret_cast<FitState*>(base + L.blocks + L.b_state);
    SelectState* sel0 = reinterpret_cast<SelectState*>(base + L.blocks + L.b_sel);
    const FitVecs v0 = make_vecs(base, L.blocks + L.b_vecs, L.nld);
    int* ints = reinterpret_cast<int*>(base + L.ints);
    hipStream_t us = static_cast<hipStream_t>(stream);

    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return DIA_E_HIP;
    int rc = DIA_OK;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
#define TRY(expr)               \
    if (!(expr)) {              \
        rc = DIA_E_HIP;         \
        break;                  \
    }
    try {
        do {
            TRY(hipStreamSynchronize(us) == hipSuccess);
            // init every epoch: median of its target (radix select) then theta and the optimiser state
            for (int e = 0; e < n; ++e) {
                SelectState* sel = reinterpret_cast<SelectState*>(reinterpret_cast<char*>(sel0) + e * L.stride);
                if (o.init != DIA_INIT_USER)
                    TRY(launch_median(epochs[e].I, epochs[e].rows, epochs[e].cols, epochs[e].ld, sel, cs) == hipSuccess);
                const float* Re = R.data + (long long)epochs[e].ref_row0 * R.ld + epochs[e].ref_col0;
                TRY(launch_ref_stats(Re, epochs[e].rows, epochs[e].cols, R.ld, sel, cs) == hipSuccess);
            }
            if (rc != DIA_OK) break;
            TRY(launch_init_fit(st0, v0, m, 1, o.init, o.init_phi, theta, sel0, cs, n, (long long)L.stride) ==
                hipSuccess);
            TRY(launch_zero_ints(ints, 16, cs) == hipSuccess);

            const int* done0 = &st0->done;
            int variant = 0;
            int n_chunks = 0, grid = 0;
            BatchedArgs b;
            std::vector<Bf16x3Args> g;
            int rows_per = 0;
            if (precision == DIA_PREC_FP32) {
                const std::vector<EpochDev> d = epoch_descs(R, epochs, n, m, v0.theta_eval, (long long)L.stride,
                                                            v0.theta_eval64, (long long)L.stride, done0,
                                                            (long long)L.stride);
                TRY(upload(base + L.epochs, d.data(), sizeof(EpochDev) * n, cs));
                variant = choose_batched_variant(base, L, R, epochs, n, m, *obj, cs);
                const Plan p = make_plan(m, epochs, n, variant);
                TRY(upload_plan(base, L, p, cs));
                n_chunks = (int)p.chunks.size();
                grid = batched_grid(m, variant, n_chunks);
                b = batched_args(base, L, R, *obj, n_chunks);
            } else {
                TRY(bf16x3_prepare(R, epochs, n, m, *obj, v0.theta_eval, (long long)L.stride,
                                   reinterpret_cast<double*>(base + L.partial), &g, done0,
                                   (long long)L.stride) == DIA_OK);
                rows_per = bf16x3_partial_rows(m, epochs[0].rows, epochs[0].cols, n) / n;
            }
            TRY(launch_zero_ints(ints, 16, cs) == hipSuccess);

            BatchReduceArgs br;
            std::memset(&br, 0, sizeof(br));
            br.partial = reinterpret_cast<const double*>(base + L.partial);
            br.cbeg = rows_per > 0 ? nullptr : reinterpret_cast<const int*>(base + L.cbeg);
            br.cend = rows_per > 0 ? nullptr : reinterpret_cast<const int*>(base + L.cend);
            br.rows_per = rows_per;
            br.npp = L.npp;
            br.gt = reinterpret_cast<double*>(base + L.gt);
            br.st = st0;
            br.v = v0;
            br.stride = (long long)L.stride;
            br.o = opts_dev(o);
            br.n = L.n;
            br.m = m;
            br.queue = ints;
            br.n_done = ints + 1;

            // poll_every optimiser iterations as one graph
            auto capture = [&]() -> bool {
                if (exec) (void)hipGraphExecDestroy(exec);
                if (graph) (void)hipGraphDestroy(graph);
                exec = nullptr;
                graph = nullptr;
                if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
                bool ok = true;
                for (int k = 0; k < o.poll_every; ++k) {
                    if (precision == DIA_PREC_FP32)
                        ok = ok && launch_batched_eval(m, grid, b, cs, variant) == hipSuccess;
                    else
                        ok = ok && bf16x3_launch_eval(g, cs) == hipSuccess;
                    ok = ok && launch_reduce_batched(br, n, cs) == hipSuccess;
                }
                if (hipStreamEndCapture(cs, &graph) != hipSuccess || !ok) return false;
                return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            };
            TRY(capture());
            const int max_reps = o.max_eval / o.poll_every + 2;
            int n_done = 0;
            std::vector<int> done_h(n), live;
            for (int rep = 0; rep < max_reps && n_done < n && rc == DIA_OK; ++rep) {
                TRY(hipGraphLaunch(exec, cs) == hipSuccess);
                TRY(hipMemcpyAsync(&n_done, ints + 1, sizeof(int), hipMemcpyDeviceToHost, cs) == hipSuccess);
                TRY(hipStreamSynchronize(cs) == hipSuccess);
                // split precision: once the unconverged epochs fit in fewer blocks of 32, gather
                // them into full blocks (a block costs the same however many of its epochs still run)
                if (precision == DIA_PREC_BF16X3 && n_done < n &&
                    (n - n_done + kBf16x3Block - 1) / kBf16x3Block < (int)g.size()) {
                    TRY(hipMemcpy2DAsync(done_h.data(), sizeof(int), &st0->done, (size_t)L.stride, sizeof(int), n,
                                         hipMemcpyDeviceToHost, cs) == hipSuccess);
                    TRY(hipStreamSynchronize(cs) == hipSuccess);
                    live.clear();
                    for (int e = 0; e < n; ++e)
                        if (done_h[e] == 0) live.push_back(e);
                    if (live.empty()) break;
                    TRY(bf16x3_prepare(R, epochs, n, m, *obj, v0.theta_eval, (long long)L.stride,
                                       reinterpret_cast<double*>(base + L.partial), &g, done0, (long long)L.stride,
                                       &live) == DIA_OK);
                    TRY(capture());
                }
            }
            if (rc != DIA_OK) break;
            std::vector<NewtonOutcome> nw(n);
            if (o.max_newton > 0) {
                // exact-Hessian polish of every epoch that finished without error, kNewtonLanes at a
                // time: each lane is a host thread with its own stream and workspace region, taking
                // epochs from a shared counter (the epochs' states and vectors are disjoint)
                const bool quad = obj->rho == DIA_RHO_GAUSS && obj->var != DIA_VAR_CCD_MODEL &&
                                  obj->var != DIA_VAR_EMCCD_MODEL;
                std::vector<int> status_h(n);
                TRY(hipMemcpy2DAsync(status_h.data(), sizeof(int), &st0->status, (size_t)L.stride, sizeof(int), n,
                                     hipMemcpyDeviceToHost, cs) == hipSuccess);
                TRY(hipStreamSynchronize(cs) == hipSuccess);
                int device = 0;
                TRY(hipGetDevice(&device) == hipSuccess);
                const int lanes = std::min(kNewtonLanes, n);
                std::atomic<int> next{0};
                std::vector<int> lane_rc(lanes, DIA_OK);
                auto lane = [&](int w) {
                    hipStream_t ls = nullptr;
                    if (hipSetDevice(device) != hipSuccess ||
                        hipStreamCreateWithFlags(&ls, hipStreamNonBlocking) != hipSuccess) {
                        lane_rc[w] = DIA_E_HIP;
                        return;
                    }
                    char* nb = base + L.newton + (size_t)w * L.newton_each;
                    for (;;) {
                        const int e = next.fetch_add(1);
                        if (e >= n) break;
                        if (status_h[e] < 0) continue;
                        FitState* st = reinterpret_cast<FitState*>(reinterpret_cast<char*>(st0) + e * L.stride);
                        dia_image Re{R.data + (long long)epochs[e].ref_row0 * R.ld + epochs[e].ref_col0,
                                     epochs[e].rows, epochs[e].cols, R.ld};
                        dia_image Ie{epochs[e].I, epochs[e].rows, epochs[e].cols, epochs[e].ld};
                        dia_objective oe = *obj;
                        oe.weights = epochs[e].weights;
                        oe.flat = epochs[e].flat;
                        oe.mask = epochs[e].mask;
                        const NewtonLayout NL = newton_layout(m, Ie.rows, Ie.cols, true, true);
                        const int ge = eval_grid(m, tile_grid_tiles(m, Ie.rows, Ie.cols, 0), 0);
                        const int pr = newton_polish(Re, Ie, to_params(oe), 0.0, m, 0, ge, 0, st,
                                                     offset_vecs(v0, (long long)e * L.stride),
                                                     reinterpret_cast<double*>(nb + NL.part), nb, NL, o.max_newton,
                                                     quad, ls, &nw[e]);
                        if (pr != DIA_OK) {
                            lane_rc[w] = pr;
                            break;
                        }
                    }
                    (void)hipStreamSynchronize(ls);
                    (void)hipStreamDestroy(ls);
                };
                std::vector<std::thread> pool;
                try {
                    for (int w = 1; w < lanes; ++w) pool.emplace_back(lane, w);
                } catch (...) {
                    // fewer lanes: the started ones and this thread take every epoch from the counter
                }
                lane(0);
                for (auto& t : pool) t.join();
                for (int w = 0; w < lanes; ++w)
                    if (lane_rc[w] != DIA_OK && rc == DIA_OK) rc = lane_rc[w];
                if (rc != DIA_OK) break;
            }
            TRY(launch_finalize(st0, v0, m, theta, cs, n, (long long)L.stride) == hipSuccess);
            std::vector<FitState> fs(n);
            for (int e = 0; e < n; ++e)
                TRY(hipMemcpyAsync(&fs[e], reinterpret_cast<char*>(st0) + e * L.stride, sizeof(FitState),
                                   hipMemcpyDeviceToHost, cs) == hipSuccess);
            if (rc != DIA_OK) break;
            TRY(hipStreamSynchronize(cs) == hipSuccess);
            int worst_neg = 0, worst_pos = 0;
            for (int e = 0; e < n; ++e) {
                int se = fs[e].done ? fs[e].status : DIA_W_NOT_CONVERGED;
                int stop = fs[e].done ? fs[e].stop : STOP_CAP;
                const int first_stop = stop;
                if (se >= 0 && nw[e].converged) se = DIA_OK, stop = STOP_NEWTON;
                if (se < worst_neg) worst_neg = se;
                if (se > worst_pos) worst_pos = se;
                if (res != nullptr) {
                    res[e].loss = fs[e].out_loss;
                    res[e].P = fs[e].out_P;
                    res[e].B0 = fs[e].out_B0;
                    res[e].n_eval = fs[e].n_eval + nw[e].evals;
                    res[e].n_adam = fs[e].n_adam;
                    res[e].n_lbfgs = fs[e].n_lbfgs;
                    res[e].n_outer = 1;
                    res[e].n_masked = 0;
                    res[e].stop = stop;
                    res[e].status = se;
                    res[e].n_newton = nw[e].steps;
                    res[e].n_hessian = nw[e].hessians;
                    res[e].first_order_stop = first_stop;
                    res[e].reserved = 0;
                }
            }
            rc = worst_neg < 0 ? worst_neg : worst_pos;
        } while (false);
    } catch (...) {
        rc = DIA_E_HIP;
    }
#undef TRY
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    return rc;
}

}  // extern "C"

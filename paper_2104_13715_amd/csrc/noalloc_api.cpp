// dia_loss_grad_noalloc: the fused loss and gradient with the library's own static scratch in place
// of a caller workspace, for callers that cannot allocate device memory.
//
// The scratch is a file-scope device array.  In host code its name is a host-side stand-in, not a
// device address, so the array is only ever reached through the pointer that hipGetSymbolAddress
// returns on each device (each GPU holds its own copy at its own address), looked up once per
// device on the first call there, with that device current.
#include <mutex>

#include "api_util.h"

namespace dia {
namespace {

constexpr size_t kScratchBytes = DIA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's scratch (nullptr on failure).
void* scratch_on_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace dia

using namespace dia;

extern "C" int dia_loss_grad_noalloc(dia_image R, dia_image I, const dia_objective* obj, const float* theta,
                                     int32_t m, double* loss, float* grad, void* stream) {
    // the same argument checks as dia_loss_grad, then the workspace it would need
    int c = check_image(R);
    if (c != DIA_OK) return c;
    if ((c = check_image(I)) != DIA_OK) return c;
    if (R.rows != I.rows || R.cols != I.cols) return DIA_E_SIZE;
    if ((c = check_m(m, R.rows, R.cols)) != DIA_OK) return c;
    if ((c = check_obj(obj)) != DIA_OK) return c;
    if (theta == nullptr || loss == nullptr || grad == nullptr) return DIA_E_ARG;
    size_t need = 0;
    if ((c = dia_workspace_size(DIA_OP_LOSS_GRAD, I.rows, I.cols, I.ld, m, &need)) != DIA_OK) return c;
    if (need > kScratchBytes) return DIA_E_SCRATCH;
    void* ws = scratch_on_current_device();
    if (ws == nullptr) return DIA_E_HIP;
    return loss_grad_impl(R, I, obj, theta, nullptr, m, loss, grad, nullptr, ws, kScratchBytes, stream,
                          /*may_time=*/false);
}

// Allocation-free variant of the bank adjoint: the same launches as
// gabor_bank_apply_adjoint with the workspace taken from a fixed device
// array of this library instead of memory the plan allocates.  For callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops).
#include <mutex>

#include "gabor_plan_impl.h"

namespace {

constexpr int64_t kScratchBytes = int64_t(64) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU the library runs on, held until the process ends.  In
// host code `scratch` names a host-side stand-in, never the device memory:
// only the address from hipGetSymbolAddress is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device
// with that device current.
hipError_t scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" gabor_status gabor_bank_apply_adjoint_noalloc(gabor_plan p, const void* d_grad_out, float* d_grad_image,
                                                         int64_t grad_row_stride_elems, void* hip_stream)
{
    if (!p || !d_grad_out || !d_grad_image) return GABOR_ERR_INVALID_ARG;
    if (grad_row_stride_elems < p->W) return GABOR_ERR_INVALID_ARG;
    gabor::AdjLayout L;
    const gabor_status st = gabor::adjoint_layout(p, &L);
    if (st != GABOR_OK) return st;
    if (L.bytes > kScratchBytes) return GABOR_ERR_UNSUPPORTED;
    void* ws = nullptr;
    if (scratch_address(&ws) != hipSuccess) return GABOR_ERR_DEVICE;
    return gabor::adjoint_run(p, L, ws, d_grad_out, 1, 0, d_grad_image, 0, grad_row_stride_elems,
                              (hipStream_t)hip_stream, false);
}

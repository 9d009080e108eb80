// The reverse step for callers that cannot allocate device memory (code under
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// bfvm_step_adjoint keeps its workspace (three sweep outputs, reduction
// partials and results) in allocations it makes on first use.  This variant
// takes the same workspace from `scratch`, a file-scope device array that the
// code object carries: every GPU on which the library runs holds one copy
// until the process ends.  Host code must not pass the array's name to a
// kernel or a copy (on the host it is only a stand-in for the symbol); the
// device address is looked up once per device with hipGetSymbolAddress and
// used from then on.
//
// Nothing in the workspace has to start at zero: the recomputed sweep
// outputs are written in full before they are read, every reduction block
// writes its own partial sums, and the final reduction writes the results.
// Every call on one GPU shares that GPU's array, so calls that overlap on
// one GPU (from several threads, or on several streams) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

// 96 MiB for the three sweep outputs (the 128^3 x 2 FP64 differentiation
// grid uses exactly that) plus 2 MiB for the per-line sums (1.5 MiB on that
// grid) and the results.
constexpr size_t kScratchBytes = (98ull << 20);
constexpr size_t kAlign = 256;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

size_t round_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int nf_fail(int code, const std::string& msg)
{
    bfvm::set_error(msg);
    return code;
}

// the device address of this device's copy of `scratch`
int scratch_ptr(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return nf_fail(BFVM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return nf_fail(BFVM_EDEVICE, "hipGetDevice");
        if (cur != device && hipSetDevice(device) != hipSuccess) return nf_fail(BFVM_EDEVICE, "hipSetDevice");
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return nf_fail(BFVM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return BFVM_OK;
}

}  // namespace

extern "C" int bfvm_step_adjoint_noalloc(bfvm_grid g, const void* field_in, void* grad, double* grad_D,
                                         double* grad_lambda)
{
    if (!g) return nf_fail(BFVM_EINVAL, "grid is NULL");
    if (!field_in || !grad || !grad_D || !grad_lambda) return nf_fail(BFVM_EINVAL, "NULL pointer");
    if (!g->have_params) return nf_fail(BFVM_ESTATE, "set_params must come before step_adjoint_noalloc");
    const size_t field = round_up((size_t)g->nelem() * bfvm::dtype_size(g->dtype));
    const size_t parts = round_up(sizeof(double) * (size_t)bfvm::adjoint_partials_count(g));
    const size_t outs = round_up(sizeof(double) * 6 * (size_t)g->S);
    const size_t need = 3 * field + parts + outs;
    if (need > kScratchBytes)
        return nf_fail(BFVM_EINVAL, "grid too large for the allocation-free reverse step: it needs " +
                                        std::to_string(need) + " bytes of workspace, the scratch array holds " +
                                        std::to_string(kScratchBytes));
    void* base = nullptr;
    if (int st = scratch_ptr(g->device, &base)) return st;
    char* b = static_cast<char*>(base);
    void* work[3] = {b, b + field, b + 2 * field};
    double* partials = reinterpret_cast<double*>(b + 3 * field);
    double* red_out = reinterpret_cast<double*>(b + 3 * field + parts);
    // stage timing would create events: off for this call
    const bool timing = g->timing;
    g->timing = false;
    const int st = bfvm::adjoint_step_into(g, field_in, grad, work, partials, red_out, grad_D, grad_lambda);
    g->timing = timing;
    return st;
}

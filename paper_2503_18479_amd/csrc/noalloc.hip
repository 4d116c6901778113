// cosim_loss_and_grad_noalloc: cosim_loss_and_grad without any allocation,
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The call's device buffers (currents, factor records, partial sums and
// per-system gradient terms) live in one file-scope device array instead of
// the plan's workspace.  Each device holds its own copy of the array at its
// own address, taken once per device with hipGetSymbolAddress while that
// device is current; host code uses only that address.  Every call on a
// device shares its copy, so calls that overlap on one device race.  Nothing
// in the array needs to start at zero: every element a call reads was written
// earlier in the same call.
#include <mutex>

#include "internal.h"

static constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

// Address of this device's copy of `scratch`; the device must be current.
int scratch_ptr(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return cosim::set_error(COSIM_EUNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return cosim::set_error(COSIM_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
        }
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return COSIM_OK;
}

}  // namespace

extern "C" {

size_t cosim_noalloc_scratch_bytes(void) { return kScratchBytes; }

int cosim_loss_and_grad_noalloc(cosim_plan_t p, int B, int F, const double *C_d,
                                const double *omega_d, const double *T_d, int loss_mode,
                                int precision, double *loss_d, double *grad_d, int32_t *status_d,
                                void *stream) {
    if (!p) return cosim::set_error(COSIM_EINVAL, "null plan");
    int device = -1;
    int rc = cosim::plan_device(p, &device);
    if (rc) return rc;
    void *ptr = nullptr;
    if ((rc = scratch_ptr(device, &ptr))) return rc;
    return cosim::loss_and_grad_scratch(p, B, F, C_d, omega_d, T_d, loss_mode, precision, loss_d,
                                        grad_d, status_d, stream, ptr, kScratchBytes);
}

}  // extern "C"

// Allocation-free decode: the decoder's workspace for the call is a static
// per-device array of this library instead of caller memory, so the call
// itself allocates nothing (for callers that cannot allocate).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qcmet.h"
#include "qcmet_internal.h"

namespace {

// The array itself.  In host code its name stands for a host-side shadow,
// not a device address: kernels and copies take the address that
// hipGetSymbolAddress returns for the current device, kept per device below.
__device__ __align__(256) char scratch[QM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return qm_set_error(QM_ERR_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return qm_set_error(QM_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return qm_set_error(QM_ERR_HIP, e != hipSuccess ? hipGetErrorString(e) : "no scratch address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return QM_OK;
}

}  // namespace

extern "C" int qm_decode_noalloc(qm_decoder *dec, const float *llr, const uint8_t *syndrome, int32_t iters,
                                 uint8_t *hard, float *app, uint8_t *flags, void *stream) {
    if (!dec) return qm_set_error(QM_ERR_INVALID_ARG, "decoder is NULL");
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != QM_OK) return rc;
    return qm_decode_on_workspace(dec, static_cast<char *>(ws), QM_NOALLOC_SCRATCH_BYTES, llr, syndrome, iters, hard,
                                  app, flags, static_cast<hipStream_t>(stream));
}

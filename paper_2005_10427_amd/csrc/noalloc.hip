// Transposition without a caller-supplied workspace, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that forbid it).  The
// workspace is one fixed array in device memory: each GPU the library runs on holds its own
// copy for the life of the process.  Calls on one GPU share it, so calls that overlap on one
// GPU (different streams, or different host threads) race and must not be issued.
#include "../../include/qsd.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace {

constexpr size_t kScratchBytes = QSD_NOALLOC_MAX_WORKSPACE;
constexpr int kMaxDevices = 64;

// The workspace of qsd_transpose_noalloc.  In host code this name is only a handle for the
// runtime: the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this GPU's copy, looked up once per device with that device current.
qsd_status scratch_on(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return QSD_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return QSD_ERR_HIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return QSD_ERR_HIP;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev && hipSetDevice(cur) != hipSuccess) return QSD_ERR_HIP;
        if (e != hipSuccess || !p) return QSD_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return QSD_OK;
}

}  // namespace

extern "C" qsd_status qsd_transpose_noalloc(qsd_plan_t plan, int64_t nnz, const void* const* in_crd,
                                            const void* in_val, void* const* out_crd, void* out_val,
                                            hipStream_t stream) {
    if (!plan) return QSD_ERR_NULL;
    size_t need = 0;
    const qsd_status st = qsd_plan_workspace(plan, &need);
    if (st != QSD_OK) return st;
    if (need > kScratchBytes) return QSD_ERR_WORKSPACE;  // the plan needs more than the fixed array
    int dev = 0;
    if (stream) {
        if (hipStreamGetDevice(stream, &dev) != hipSuccess) return QSD_ERR_HIP;
    } else if (hipGetDevice(&dev) != hipSuccess) {
        return QSD_ERR_HIP;
    }
    void* ws = nullptr;
    const qsd_status s2 = scratch_on(dev, &ws);
    if (s2 != QSD_OK) return s2;
    // qsd_transpose clears the parts of the workspace that must start at zero (control block,
    // histograms, look-back words) with kernels on `stream`; it allocates nothing
    return qsd_transpose(plan, nnz, in_crd, in_val, out_crd, out_val, ws, kScratchBytes, stream);
}

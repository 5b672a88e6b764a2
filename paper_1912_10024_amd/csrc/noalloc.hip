// sse_backward_noalloc: the adjoint with its workspace in a file-scope device
// array instead of a caller-provided buffer, for callers that cannot allocate.
//
// The array (kScratchBytes) is part of the library's code object: every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never uses the array's name as a device address: on the
// first call on a device (with that device current) hipGetSymbolAddress gives
// that device's address, which is kept per device and passed to the kernels.
// Nothing here allocates.  Every call on a GPU shares that GPU's array, so
// calls that overlap on one GPU race; the kernels overwrite every part of the
// array they read (the reverse adjacency is built by a zeroing kernel, then
// counts, scan and fill; every d grad H share that the reduction reads is
// written first), so no clearing between calls is needed.
#include <mutex>

#include "sse_kernels.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of the array (resolved once per device)
hipError_t scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t sse_noalloc_scratch_bytes(void) { return kScratchBytes; }

int sse_backward_noalloc(const sse_dims* dims, const double* G, const double* D, const double* dH,
                         const int32_t* nbr, double alpha_re, double alpha_im, const double* dSigma, double* dG,
                         double* dD, double* ddH, void* stream) {
    // argument checks as for sse_backward (its messages via sse_last_error)
    size_t full = 0;  // (validates dims)
    int rc = sse_workspace_bytes(dims, SSE_FP64, 1, &full);
    if (rc) return rc;
    // the part of the workspace this call uses: without ddH, the reverse adjacency only
    const size_t need = sse::bwd_workspace_bytes_for(sse::to_dims(*dims), false, ddH != nullptr);
    if (need > kScratchBytes)
        return sse::set_error(SSE_ERR_WORKSPACE, "sse_backward_noalloc: these dims need %zu bytes of workspace, above its %zu",
                              need, kScratchBytes);
    void* ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return sse::set_error(SSE_ERR_HIP, "sse_backward_noalloc: scratch address: %s", hipGetErrorString(e));
    // the D gradient reads g in the caller's layout: its atom-major copy would not fit the array
    return sse::backward_one_table(dims, G, D, dH, nbr, alpha_re, alpha_im, dSigma, dG, dD, ddH, ws, kScratchBytes,
                                   stream, false);
}

}  // extern "C"

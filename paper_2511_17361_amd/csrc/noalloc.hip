// sq_render_fwd_noalloc: the forward render of sq_render_fwd with its scratch
// space in a fixed device array of this library instead of a caller
// workspace, for callers that cannot allocate device memory (code under
// hipGraph capture, serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol); it asks the runtime for the device address once per device
// (hipGetSymbolAddress, with that device current) and passes that pointer as
// the workspace of the ordinary forward.  No call here allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/sqr.h"
#include "sqr_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SQ_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (looked up once).
hipError_t scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

sq_status sq_render_fwd_noalloc(const sq_grid* grid, const sq_index* idx, const sq_prims* prims,
                                const sq_rays* rays, const sq_march* march, float* depth, float* sem, float* probs,
                                float* t_final, float* ckpt, int64_t* stats, const sq_tuning* tuning,
                                hipStream_t stream) {
    // the size check is host arithmetic only: an oversized call touches no device
    const size_t need = sq_render_workspace(grid, prims, rays, march);
    if (need == 0) {
        // invalid arguments: let the full call report which (it launches nothing)
        return sq_render_fwd(grid, idx, prims, rays, march, depth, sem, probs, t_final, ckpt, stats, tuning,
                             nullptr, 0, stream);
    }
    if (need > (size_t)SQ_NOALLOC_SCRATCH_BYTES)
        return sqr::set_error(SQ_ERR_CAPACITY, "sq_render_fwd_noalloc: %zu bytes of scratch needed, the fixed "
                                               "array holds %zu", need, (size_t)SQ_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess)
        return sqr::set_error(SQ_ERR_HIP, "sq_render_fwd_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    return sq_render_fwd(grid, idx, prims, rays, march, depth, sem, probs, t_final, ckpt, stats, tuning, ws,
                         (size_t)SQ_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"

// rad_batch_static: rad_batch for callers that cannot allocate (code under hipGraph
// capture, tight serving loops, harnesses that forbid allocation).  Its workspace --
// segment descriptors and the chunk partial amplitudes -- is one file-scope device
// array, `scratch`, of kStaticScratchBytes per GPU, loaded with the library and held
// until the process ends.  The host code never passes the array's name to a kernel
// (on the host it names a stand-in, not device memory): the array's device address is
// looked up with hipGetSymbolAddress once per device, with that device current, and
// that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rad.h"
#include "rad_internal.h"

namespace rad {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU

__device__ __align__(256) char scratch[kStaticScratchBytes];

rad_status run_in_scratch(const rad_grid *grid, const rad_segment *segs, int n_segs, const int *out_index,
                          int n_out, int kinds, rad_precision prec, double *out, char *scratch_ptr, size_t cap,
                          hipStream_t st);

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};
bool g_tried[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the first call
// on that device), or nullptr with the lookup's error.
char *scratch_on_current(hipError_t &err)
{
    int dev = -1;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_tried[dev]) {
        void *p = nullptr;
        g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_err[dev] == hipSuccess ? (char *)p : nullptr;
        g_tried[dev] = true;
    }
    err = g_err[dev];
    return g_ptr[dev];
}

}  // namespace
}  // namespace rad

extern "C" {

size_t rad_static_scratch_bytes(void) { return rad::kStaticScratchBytes; }

rad_status rad_batch_static(const rad_grid *grid, const rad_segment *segs, int n_segs, const int *out_index,
                            int n_out, int kinds, rad_precision prec, double *out, void *stream)
{
    hipError_t e = hipSuccess;
    char *p = rad::scratch_on_current(e);
    if (!p) {
        rad_err::set(e == hipSuccess ? "no fixed scratch on this device" : hipGetErrorString(e));
        return RAD_EDEVICE;
    }
    return rad::run_in_scratch(grid, segs, n_segs, out_index, n_out, kinds, prec, out, p,
                               rad::kStaticScratchBytes, (hipStream_t)stream);
}

}  // extern "C"

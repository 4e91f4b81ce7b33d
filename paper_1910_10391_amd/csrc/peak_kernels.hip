// Issue-rate microbenchmarks: the ceilings the radiation-integral kernels are
// measured against.  The integral path is bound by vector ALU work -- the phase
// factors and the complex accumulation (Sec. II; the paper finds double-precision
// throughput decisive, Sec. V) -- so the ceilings are the chip's FP64 and FP32 FMA
// rates, the FP32 hardware sine/cosine rate and the two phase-factor routines of the
// kernels.  Each thread runs kChains independent dependency chains (enough
// independent work to hide the pipeline latency at 8 waves per CU); results are
// summed into out[] so that nothing is optimised away.
#include <hip/hip_runtime.h>

#include "rad_internal.h"
#include "rad_math.h"
#include "rad_peaks.h"

namespace rad {
namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 4;

__global__ __launch_bounds__(256) void peak_fma64(double m, double c, int64_t iters, double *out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = 1.0 + 1e-3 * (double)((tid + j) & 255);
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int j = 0; j < kChains; ++j) a[j] = __builtin_fma(a[j], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[tid] = s;
}

__global__ __launch_bounds__(256) void peak_fma32(float m, float c, int64_t iters, double *out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = 1.0f + 1e-3f * (float)((tid + j) & 255);
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int j = 0; j < kChains; ++j) a[j] = __builtin_fmaf(a[j], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[tid] = (double)s;
}

// half the chains take the sine, half the cosine (revolutions in, values in [-1, 1] out:
// the chain stays in the instruction's domain)
__global__ __launch_bounds__(256) void peak_sincos32(int64_t iters, double *out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = 1e-3f * (float)((tid + j) & 255);
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int j = 0; j < kChains; ++j)
                a[j] = (j & 1) ? __builtin_amdgcn_cosf(a[j]) : __builtin_amdgcn_sinf(a[j]);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[tid] = (double)s;
}

// The kernels' phase factors on independent arguments: u advances by a step per
// evaluation (one FP64 add, as the phase product of the kernels is one multiply) and
// the factors are summed.
template <bool MIXED>
__global__ __launch_bounds__(256) void peak_phase(double du, int64_t iters, double *out)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double u[kChains], acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        u[j] = 1e3 * (double)((tid * kChains + j) & 4095) + 0.1234;
        acc[j] = 0.0;
    }
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u_ = 0; u_ < kUnroll; ++u_)
#pragma unroll
            for (int j = 0; j < kChains; ++j) {
                u[j] += du;
                double cr, ci;
                if constexpr (MIXED) {
                    float cf, sf;
                    cis_revolutions_f32(u[j], cf, sf);
                    cr = (double)cf;
                    ci = (double)sf;
                } else {
                    cis_halfturns(u[j], cr, ci);
                }
                acc[j] += cr + ci;
            }
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j];
    out[tid] = s;
}

}  // namespace
}  // namespace rad

extern "C" {

rad_status rad_peak(int which, int64_t iters, double *out, int64_t n_threads, double *ops, void *stream)
{
    using namespace rad;
    if (which < 0 || which >= RAD_PEAK_COUNT || iters < 1 || n_threads < 256 || n_threads % 256 ||
        n_threads > ((int64_t)1 << 31) || !out || !ops) {
        rad_err::set("rad_peak: invalid which, iters, n_threads (a positive multiple of 256) or pointer");
        return RAD_EINVAL;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)out) != hipSuccess ||
        (const char *)out + (size_t)n_threads * sizeof(double) > (const char *)base + size) {
        (void)hipGetLastError();
        rad_err::set("rad_peak: out is not n_threads doubles of device memory");
        return RAD_EINVAL;
    }
    const dim3 grid((unsigned)(n_threads / 256)), block(256);
    hipStream_t st = (hipStream_t)stream;
    const double per_thread = (double)iters * kUnroll * kChains;
    switch (which) {
    case RAD_PEAK_FMA64:
        hipLaunchKernelGGL(peak_fma64, grid, block, 0, st, 0.9999999, 1e-7, iters, out);
        *ops = 2.0 * per_thread * (double)n_threads;
        break;
    case RAD_PEAK_FMA32:
        hipLaunchKernelGGL(peak_fma32, grid, block, 0, st, 0.9999f, 1e-4f, iters, out);
        *ops = 2.0 * per_thread * (double)n_threads;
        break;
    case RAD_PEAK_SINCOS32:
        hipLaunchKernelGGL(peak_sincos32, grid, block, 0, st, iters, out);
        *ops = per_thread * (double)n_threads;
        break;
    case RAD_PEAK_PHASE64:
        hipLaunchKernelGGL(peak_phase<false>, grid, block, 0, st, 0.618033988749895, iters, out);
        *ops = per_thread * (double)n_threads;
        break;
    case RAD_PEAK_PHASE_MIXED:
        hipLaunchKernelGGL(peak_phase<true>, grid, block, 0, st, 0.618033988749895, iters, out);
        *ops = per_thread * (double)n_threads;
        break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        rad_err::set(hipGetErrorString(e));
        return RAD_EDEVICE;
    }
    return RAD_OK;
}

}  // extern "C"

/*
 * rad_peaks.h -- issue-rate microbenchmarks of librad (measurement only).
 *
 * The radiation integrals (include/rad.h) are bound by vector arithmetic, not by
 * memory or matrix units: per (time, photon energy, direction) term a phase
 * factor exp(i kappa psi) and a complex multiply-accumulate (Sec. II; the paper
 * finds double-precision throughput decisive for its GPU timings, Sec. V).  These
 * kernels measure the ceilings that work is compared with on the GPU at hand:
 *
 *   RAD_PEAK_FMA64       FP64 fused multiply-adds        (ops = 2 flops per FMA)
 *   RAD_PEAK_FMA32       FP32 fused multiply-adds, no packed instructions (2 per FMA)
 *   RAD_PEAK_SINCOS32    hardware FP32 sine / cosine of revolutions (1 per instruction)
 *   RAD_PEAK_PHASE64     the FP64 kernels' phase factor exp(i pi u) (1 per factor)
 *   RAD_PEAK_PHASE_MIXED the mixed form's phase factor (FP64 reduction, FP32 sin/cos; 1 per factor)
 *
 * rad_peak launches n_threads threads (a positive multiple of 256, at most 2^31)
 * that each run `iters` rounds of 32 independent operations, writes one value per
 * thread to out (DEVICE double [n_threads], so that nothing is optimised away) and
 * stores the number of operations of the launch in *ops (HOST).  The launch is
 * asynchronous on `stream`; time it with events on that stream.
 * Errors: RAD_EINVAL for an unknown `which`, iters < 1, a bad thread count or a
 * NULL / too small out; RAD_EDEVICE if the launch fails.
 */
#ifndef RAD_PEAKS_H
#define RAD_PEAKS_H

#include <stdint.h>

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RAD_PEAK_FMA64 = 0,
    RAD_PEAK_FMA32 = 1,
    RAD_PEAK_SINCOS32 = 2,
    RAD_PEAK_PHASE64 = 3,
    RAD_PEAK_PHASE_MIXED = 4,
    RAD_PEAK_COUNT = 5
};

rad_status rad_peak(int which, int64_t iters, double *out, int64_t n_threads, double *ops, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAD_PEAKS_H */

// Phase factors exp(i phi) for the radiation-integral kernels.
//
// FP64 form: the phase arrives as a count of half turns u = phi / pi (the
// kernels multiply the FP64 phase by kappa / pi), is reduced exactly to
// f = u - rint(u) in [-1/2, 1/2], and
//     sin(pi f) = f PS(f^2),   cos(pi f) = PC(f^2)
// with Chebyshev-fitted polynomials (sincos_coeffs.h, written by
// gen_sincos_coeffs.py).  exp(i pi u) = (-1)^rint(u) (cos(pi f) + i sin(pi f)),
// so the only quadrant work is one sign flip of both parts.
//
// FP32 form (mixed precision): the phase is reduced in FP64 to revolutions
// r = phi/(2 pi) - rint(phi/(2 pi)) in [-1/2, 1/2] and the hardware
// v_sin_f32 / v_cos_f32 (which take revolutions) give sin(2 pi r), cos(2 pi r).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sincos_coeffs.h"

namespace rad {

// exp(i pi u) for |u| < 2^31 half turns.
__host__ __device__ __forceinline__ void cis_halfturns(double u, double &c, double &s)
{
    const double q = __builtin_rint(u);
    const double f = u - q;           // exact: q is the nearest integer to u
    const double z = f * f;
    double ps = RAD_SIN_C[RAD_SIN_NC - 1];
#pragma unroll
    for (int k = RAD_SIN_NC - 2; k >= 0; --k) ps = __builtin_fma(ps, z, RAD_SIN_C[k]);
    double pc = RAD_COS_C[RAD_COS_NC - 1];
#pragma unroll
    for (int k = RAD_COS_NC - 2; k >= 0; --k) pc = __builtin_fma(pc, z, RAD_COS_C[k]);
    ps *= f;
    // (-1)^q: flip the sign bit of both parts when q is odd
    const uint32_t qi = (uint32_t)(int32_t)q;
    uint32_t ws[2], wc[2];
    __builtin_memcpy(ws, &ps, 8);
    __builtin_memcpy(wc, &pc, 8);
#if defined(__HIP_DEVICE_COMPILE__)
    // high word + (q << 31) flips bit 31 exactly when q is odd (the carry leaves the
    // word): one shift-and-add per part instead of a shared shift and two xors
    __asm__("v_lshl_add_u32 %0, %1, 31, %0" : "+v"(ws[1]) : "v"(qi));
    __asm__("v_lshl_add_u32 %0, %1, 31, %0" : "+v"(wc[1]) : "v"(qi));
#else
    ws[1] ^= qi << 31;
    wc[1] ^= qi << 31;
#endif
    __builtin_memcpy(&s, ws, 8);
    __builtin_memcpy(&c, wc, 8);
}

// sin, cos of 2 pi r for an FP64 revolution count r (any size < 2^52):
// exact FP64 reduction, then the FP32 hardware transcendental unit.
__device__ __forceinline__ void cis_revolutions_f32(double r, float &c, float &s)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float rf = (float)(r - __builtin_rint(r));
    s = __builtin_amdgcn_sinf(rf);
    c = __builtin_amdgcn_cosf(rf);
#else
    (void)r;
    c = s = 0.0f;  // the host pass never executes device code
#endif
}

}  // namespace rad

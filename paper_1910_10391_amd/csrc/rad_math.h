// Phase factors exp(i phi) for the radiation-integral kernels.
//
// FP64 form: the phase arrives as a count of half turns u = phi / pi (the
// kernels multiply the FP64 phase by kappa / pi), is reduced exactly to
// f = u - q in [-1/2, 1/2] with q the integer nearest to u, and
//     sin(pi f) = f PS(f^2),   cos(pi f) = PC(f^2)
// with Chebyshev-fitted polynomials (sincos_coeffs.h, written by
// gen_sincos_coeffs.py).  exp(i pi u) = (-1)^q (cos(pi f) + i sin(pi f)),
// so the only quadrant work is one sign flip of both parts.  The parity of q
// comes from one FP64 addition of 1.5 * 2^52: for an integer |q| < 2^51 the
// sum 1.5 * 2^52 + q is exact (its unit in the last place is 1), and its low
// mantissa bit is the parity of q.  Exact for |u| < 2^51 (no 32-bit integer
// conversion, which would saturate past 2^31 half turns).
//
// FP32 form (mixed precision): the phase is reduced in FP64 to revolutions
// r = phi/(2 pi) - rint(phi/(2 pi)) in [-1/2, 1/2] and the hardware
// v_sin_f32 / v_cos_f32 (which take revolutions) give sin(2 pi r), cos(2 pi r).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sincos_coeffs.h"

namespace rad {

// 1.5 * 2^52: added to an integer |q| < 2^51 it leaves q in the low mantissa bits.
constexpr double kRoundShift = 6755399441055744.0;

// exp(i pi u) for |u| < 2^51 half turns.
__host__ __device__ __forceinline__ void cis_halfturns(double u, double &c, double &s)
{
    const double q = __builtin_rint(u);
    const double f = u - q;              // exact: q is the nearest integer to u
    const double sh = q + kRoundShift;   // 1.5 * 2^52 + q, exact
    // (q from rint and the shift added to q, not to u: this form keeps the register
    // allocation of the amplitude kernels' hot loops free of spills)
    const double z = f * f;
    double ps = RAD_SIN_C[RAD_SIN_NC - 1];
#pragma unroll
    for (int k = RAD_SIN_NC - 2; k >= 0; --k) ps = __builtin_fma(ps, z, RAD_SIN_C[k]);
    double pc = RAD_COS_C[RAD_COS_NC - 1];
#pragma unroll
    for (int k = RAD_COS_NC - 2; k >= 0; --k) pc = __builtin_fma(pc, z, RAD_COS_C[k]);
    ps *= f;
    // (-1)^q: flip the sign bit of both parts when q is odd; the low word of sh is
    // q mod 2^32 (1.5 * 2^52 has no bits below 2^51), so its bit 0 is q's parity
    uint32_t shw[2];
    __builtin_memcpy(shw, &sh, 8);
    const uint32_t qi = shw[0];
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

// GPU trajectory generator (gfx950): one thread integrates one particle.
//
// The transverse motion is sequential in time, so the parallelism is across
// particles; a thread keeps its state in registers and streams its samples to
// HBM (88 bytes per step).  Arithmetic is kept in program order (no FMA
// contraction) and the normal draws use no library transcendental (traj_internal.h),
// so that the CPU generator, which takes the same steps, gives the same bits.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "traj_internal.h"

#pragma clang fp contract(off)

namespace radtraj {

// dU/dx of the periodic well for unit positive charge [eV/m]; inv_d = 1 / d (a step's
// slopes are on its critical path, and an IEEE division is a long dependent sequence here)
__device__ inline double slope(const rad_traj_params &p, double x, double inv_d)
{
    const double d = p.d_m;
    const double xr = x - d * floor(x * inv_d + 0.5);
    const double u = 2.0 * xr * inv_d;
    return p.U0_eV * ((1.0 - p.q) * 2.0 * u + p.q * 4.0 * u * u * u) * (2.0 * inv_d);
}

__device__ inline double gaussian(Stream &r)
{
    const double u1 = r.uniform(), u2 = r.uniform();
    return sqrt(-2.0 * det_log(u1)) * det_cos2pi(u2);
}

// The unit normals of every scattering kick, in parallel over (step, particle): the
// same draws (Box-Muller on uniforms j, j+1 and j+2, j+3 of the particle's stream) that
// the sequential integration would make, so the trajectories do not change.
__global__ __launch_bounds__(256) void kicks_kernel(TrajLaunch L)
{
    const int64_t total = L.max_steps * L.n_particles;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int pi = (int)(i % L.n_particles);
        const int64_t k = i / L.n_particles;
        if (k >= L.desc[pi].n) continue;
        const uint64_t s = particle_stream(L.p.seed, L.first + pi).s;
        const uint64_t j = first_kick_draw(L.p) + 4u * (uint64_t)k;
        const double u1 = uniform_at(s, j), u2 = uniform_at(s, j + 1);
        const double u3 = uniform_at(s, j + 2), u4 = uniform_at(s, j + 3);
        L.kicks[2 * i] = sqrt(-2.0 * det_log(u1)) * det_cos2pi(u2);
        L.kicks[2 * i + 1] = sqrt(-2.0 * det_log(u3)) * det_cos2pi(u4);
    }
}

// steps whose kicks are loaded ahead of use
constexpr int kKickAhead = 8;

__global__ __launch_bounds__(64) void traj_kernel(TrajLaunch L)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n_particles) return;
    const rad_traj_params &p = L.p;
    const TrajDesc D = L.desc[i];
    Stream r = particle_stream(p.seed, L.first + i);
    if (draw_steps(p, r) != D.n) return;   // the host drew the same count; never taken
    const int64_t n = D.n;
    double *const c = L.cols + D.off;
    double *const ct = c, *const cx = c + L.total, *const cy = c + 2 * L.total, *const cdz = c + 3 * L.total;
    double *const cvx = c + 4 * L.total, *const cvy = c + 5 * L.total, *const cdvz = c + 6 * L.total;
    double *const cax = c + 7 * L.total, *const cay = c + 8 * L.total, *const caz = c + 9 * L.total;
    double *const cen = c + 10 * L.total;

    const double h = p.length_m / (double)n;
    const double g_ref = p.energy_eV / kMe_eV;
    const double inv2g2_ref = 0.5 / (g_ref * g_ref);
    const double inv_me = 1.0 / kMe_eV, inv_d = 1.0 / p.d_m;
    const double s = p.charge;
    double E = p.energy_eV;
    double x = (r.uniform() - 0.5) * p.d_m;
    double vx = p.theta_sigma * gaussian(r);
    double vy = p.theta_sigma * gaussian(r);
    double y = 0.0, dz = 0.0;
    // velocities of the two previous samples, for the central-difference accelerations
    double v1x = 0.0, v1y = 0.0, v1z = 0.0, v2x = 0.0, v2y = 0.0, v2z = 0.0;
    // sample k and step k -> k + 1 (the kick's unit normals given); false after the last sample
    auto step = [&](int64_t k, double2 kick) -> bool {
        const double g = E * inv_me;
        const double dvz = inv2g2_ref - 0.5 / (g * g) - 0.5 * (vx * vx + vy * vy);
        ct[k] = h * (double)k;
        cx[k] = x;
        cy[k] = y;
        cvx[k] = vx;
        cvy[k] = vy;
        cdvz[k] = dvz;
        cdz[k] = dz;
        cen[k] = E;
        if (k >= 1) {
            // sample k-1: central difference between samples max(k-2, 0) and k
            const int64_t lo = k >= 2 ? k - 2 : 0;
            const double dt = h * (double)k - h * (double)lo;
            cax[k - 1] = (vx - (k >= 2 ? v2x : v1x)) / dt;
            cay[k - 1] = (vy - (k >= 2 ? v2y : v1y)) / dt;
            caz[k - 1] = (dvz - (k >= 2 ? v2z : v1z)) / dt;
        }
        if (k == n) {
            // last sample: one-sided difference with sample n-1
            const double dt = h * (double)n - h * (double)(n - 1);
            cax[n] = (vx - v1x) / dt;
            cay[n] = (vy - v1y) / dt;
            caz[n] = (dvz - v1z) / dt;
            return false;
        }
        v2x = v1x;
        v2y = v1y;
        v2z = v1z;
        v1x = vx;
        v1y = vy;
        v1z = dvz;
        // RK4 on (x, vx) with E frozen over the step
        const double f = -s / E;
        const double k1x = vx, k1v = f * slope(p, x, inv_d);
        const double k2x = vx + 0.5 * h * k1v, k2v = f * slope(p, x + 0.5 * h * k1x, inv_d);
        const double k3x = vx + 0.5 * h * k2v, k3v = f * slope(p, x + 0.5 * h * k2x, inv_d);
        const double k4x = vx + h * k3v, k4v = f * slope(p, x + h * k3x, inv_d);
        x += h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        vx += h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
        y += h * vy;
        if (p.loss_on) {
            const double a_mean = (k1v + 2.0 * k2v + 2.0 * k3v + k4v) / 6.0;
            E -= h * (2.0 / 3.0) * kAlpha * kHbarC * g * g * g * g * a_mean * a_mean;
        }
        if (p.ms_on) {
            const double sig = (p.eps_s_eV / E) * sqrt(h / p.X0_m);
            double gx = kick.x, gy = kick.y;
            if (!L.kicks) {
                gx = gaussian(r);
                gy = gaussian(r);
            }
            const double dtx = sig * gx, dty = sig * gy;
            vx += dtx;
            vy += dty;
            if (p.loss_on) E -= kMe_eV * kAlpha / (2.0 * kPi) * g * g * g * (dtx * dtx + dty * dty);
        }
        const double g1 = E * inv_me;
        const double dvz1 = inv2g2_ref - 0.5 / (g1 * g1) - 0.5 * (vx * vx + vy * vy);
        dz += 0.5 * h * (dvz + dvz1);
        return true;
    };
    // The kicks of a group of kKickAhead steps are loaded while the group before it runs:
    // a step's own load from HBM would otherwise sit on the critical path of the sequence.
    double2 cur[kKickAhead], nxt[kKickAhead];
    auto load_group = [&](int64_t k0, double2 (&dst)[kKickAhead]) {
#pragma unroll
        for (int j = 0; j < kKickAhead; ++j) {
            const int64_t k = k0 + j;
            dst[j] = make_double2(0.0, 0.0);
            if (L.kicks && k < n) {
                const double *kk = L.kicks + 2 * (k * L.n_particles + i);
                dst[j] = make_double2(kk[0], kk[1]);
            }
        }
    };
    load_group(0, cur);
    for (int64_t k0 = 0;; k0 += kKickAhead) {
        load_group(k0 + kKickAhead, nxt);
        bool more = true;
#pragma unroll
        for (int j = 0; j < kKickAhead; ++j)
            if (more) more = step(k0 + j, cur[j]);
        if (!more) break;
#pragma unroll
        for (int j = 0; j < kKickAhead; ++j) cur[j] = nxt[j];
    }
}

// One block per section: the entry energy, then the columns of samples k0..k1 with dvz
// and dz re-referenced to the section's own gamma (same operation order as the
// host-side cut of the CPU generator's trajectories).
__global__ __launch_bounds__(256) void sections_kernel(SecLaunch L)
{
    const SecDesc D = L.desc[blockIdx.x];
    const double *src = L.cols + D.src_off;
    double *dst = L.sec_cols + D.dst_off;
    const double E = src[10 * L.total + D.k0];
    const double g = E / kMe_eV;
    const double shift = 0.5 / (g * g) - 0.5 / (L.g_ref * L.g_ref);
    if (threadIdx.x == 0) L.entry_energy[blockIdx.x] = E;
    const int64_t n = D.k1 - D.k0 + 1;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        const int64_t i = D.k0 + k;
#pragma unroll
        for (int c = 0; c < 11; ++c) {
            double v = src[c * L.total + i];
            if (c == 6) v = v + shift;                                 // dvz
            if (c == 3) v = v + shift * src[i];                        // dz + shift t
            dst[c * L.sec_total + k] = v;
        }
    }
}

hipError_t launch_sections(const SecLaunch &L, hipStream_t st)
{
    hipLaunchKernelGGL(sections_kernel, dim3((unsigned)L.n_sec), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_kicks(const TrajLaunch &L, hipStream_t st)
{
    const int64_t total = L.max_steps * L.n_particles;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(kicks_kernel, dim3(blocks), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_traj(const TrajLaunch &L, hipStream_t st)
{
    hipLaunchKernelGGL(traj_kernel, dim3((unsigned)((L.n_particles + 63) / 64)), dim3(64), 0, st, L);
    return hipGetLastError();
}

}  // namespace radtraj

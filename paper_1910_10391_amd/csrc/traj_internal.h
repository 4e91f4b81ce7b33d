// Internal pieces of the trajectory generator shared by its host side and its kernel:
// the random-number streams (host: step counts; device: everything).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "rad_traj.h"

namespace radtraj {

constexpr double kMe_eV = 0.51099895e6;         // CODATA 2018
constexpr double kAlpha = 7.2973525693e-3;
constexpr double kHbarC = 1.973269804e-7;
constexpr double kPi = 3.14159265358979323846;

// splitmix64 (Steele, Lea, Flood 2014): state advances by the golden-ratio
// increment; output is the state passed through two xor-shift-multiply rounds.
struct Stream {
    uint64_t s;
    __host__ __device__ inline uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // uniform on (0, 1]: the top 53 bits plus one, times 2^-53
    __host__ __device__ inline double uniform() { return ((double)(next() >> 11) + 1.0) * 0x1.0p-53; }
};

// splitmix64 is counter-based: draw j (0-based) after a state s is mix(s + (j + 1) g),
// which lets the kicks of every step be drawn in parallel.
__host__ __device__ inline double uniform_at(uint64_t s, uint64_t j)
{
    Stream r{s + j * 0x9E3779B97F4A7C15ull};
    return r.uniform();
}

__host__ __device__ inline Stream particle_stream(uint64_t seed, int64_t particle)
{
    Stream r;
    r.s = (seed * 0x9E3779B97F4A7C15ull) ^ (((uint64_t)particle + 1ull) * 0xD1B54A32D192ED03ull);
    (void)r.next();
    return r;
}

// Normal draws: Box-Muller with a logarithm and a cosine evaluated from IEEE operations
// only (+ - * / sqrt, exact bit manipulation, no FMA contraction), in the same order as the CPU generator's, so that both draw the same
// bits (the host's and the device's library log and cos differ in the last bit now and
// then, and one such bit can decide on which side of a plane's kink a step lands).
//
// log u, u in (0, 1]: u = m 2^e, m in [sqrt(1/2), sqrt(2)): e ln 2 + 2 atanh(s),
// s = (m - 1) / (m + 1), |s| <= 0.172, the atanh series to s^23.
__host__ __device__ inline double det_log(double u)
{
#pragma clang fp contract(off)
    uint64_t b = (uint64_t)__builtin_bit_cast(uint64_t, u);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    b = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m = __builtin_bit_cast(double, b);
    if (m > 1.4142135623730951) {
        m = 0.5 * m;
        e = e + 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    return (double)e * 0.6931471805599453 + (2.0 * s + 2.0 * s * (z * p));
}

// cos(2 pi u), u in [0, 1]: v = min(u, 1 - u), w = v - 1/4 (exact on the 2^-53 grid),
// -sin(x) at x = 2 pi w, |x| <= pi/2, the sine's Taylor series to x^23.
__host__ __device__ inline double det_cos2pi(double u)
{
#pragma clang fp contract(off)
    const double v = u <= 0.5 ? u : 1.0 - u;
    const double w = v - 0.25;
    const double x = w * 6.283185307179586;
    const double z = x * x;
    double p = -1.0 / 25852016738884976640000.0;
    p = p * z + 1.0 / 51090942171709440000.0;
    p = p * z - 1.0 / 121645100408832000.0;
    p = p * z + 1.0 / 355687428096000.0;
    p = p * z - 1.0 / 1307674368000.0;
    p = p * z + 1.0 / 6227020800.0;
    p = p * z - 1.0 / 39916800.0;
    p = p * z + 1.0 / 362880.0;
    p = p * z - 1.0 / 5040.0;
    p = p * z + 1.0 / 120.0;
    p = p * z - 1.0 / 6.0;
    return -(x + x * (z * p));
}

// the first draw of a particle's stream: its step count, uniform in [n_min, n_max]
__host__ __device__ inline int64_t draw_steps(const rad_traj_params &p, Stream &r)
{
    if (p.n_max <= p.n_min) return p.n_min;
    const double u = r.uniform() - 1e-300;
    int64_t n = p.n_min + (int64_t)floor((double)(p.n_max - p.n_min + 1) * u);
    return n > p.n_max ? p.n_max : n;
}

struct TrajDesc {
    int64_t n;     // steps
    int64_t off;   // first sample in the packed columns
};

struct TrajLaunch {
    rad_traj_params p;
    int64_t first;
    int n_particles;
    int64_t total;
    const TrajDesc *desc;
    double *cols;   // [RAD_TRAJ_NCOL][total]
    double *kicks;  // [max_steps][n_particles][2] unit normals of the scattering kicks, or null
    int64_t max_steps;
};

// Index of a particle's first kick draw in its stream: the step count (when drawn),
// the entry x, two normals for the entry angles.
__host__ __device__ inline uint64_t first_kick_draw(const rad_traj_params &p)
{
    return (p.n_max > p.n_min ? 1u : 0u) + 5u;
}

// One section: source samples [k0, k1] of the trajectory at src_off, destination offset.
struct SecDesc {
    int64_t src_off, k0, k1, dst_off;
};

struct SecLaunch {
    const SecDesc *desc;
    int n_sec;
    double g_ref;
    const double *cols;     // [RAD_TRAJ_NCOL][total]
    int64_t total;
    double *sec_cols;       // [RAD_TRAJ_NCOL][sec_total]
    int64_t sec_total;
    double *entry_energy;   // [n_sec] (device)
};

hipError_t launch_traj(const TrajLaunch &L, hipStream_t st);
hipError_t launch_kicks(const TrajLaunch &L, hipStream_t st);
hipError_t launch_sections(const SecLaunch &L, hipStream_t st);

}  // namespace radtraj

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

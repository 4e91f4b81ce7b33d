/*
 * rad_traj.h -- C ABI of the GPU trajectory generator (part of librad).
 *
 * Planar channeling trajectories for the radiation integrals of include/rad.h,
 * generated on the GPU so that they never cross PCIe.  The model follows the
 * transverse equation of motion of Sec. III (continuum potential, multiple
 * Coulomb scattering, radiative energy loss) with a synthetic planar well, since
 * the paper's potential tables are not reproduced here:
 *
 *   U(x) = U0 [ (1-q) (2x/d)^2 + q (2x/d)^4 ],   x reduced to [-d/2, d/2) with period d;
 *   d vx / dt = -charge U'(x) / E  (t and lengths in metres, velocities in units of c),
 *   integrated by classical RK4 with a fixed step h = length / n and E frozen over a step;
 *   after each step a Gaussian kick of vx and vy, mean square (eps_s/E)^2 h / X0
 *   (Sec. III, the scattering on nuclei with a uniform density);
 *   energy loss per step: the leading term of the Landau-Lifshitz force (Sec. III),
 *   h (2/3) alpha hbar c gamma^4 a^2 with a the RK4 mean acceleration, plus
 *   (m_e alpha / 2 pi) gamma^3 (dthx^2 + dthy^2) per kick (Sec. III).
 *
 * Output columns per particle (n+1 samples for n steps): t, x, y, dz, vx, vy, dvz,
 * ax, ay, az, energy, in the small-angle variables of Sec. II relative to
 * beta_ref = 1 - 1/(2 gamma_ref^2), gamma_ref = energy_eV / m_e:
 * dvz = 1/(2 gamma_ref^2) - 1/(2 gamma^2) - (vx^2 + vy^2)/2, dz its trapezoid
 * integral, accelerations central differences of the stored (post-kick)
 * velocities, one-sided at the ends.  The particle's segment for rad_batch is the
 * whole trajectory with gamma = gamma_ref and energy = energy_eV.
 *
 * Random numbers: one splitmix64 stream (Steele, Lea and Flood, 2014) per
 * particle keyed by (seed, particle index); uniforms (0, 1] from the top 53 bits;
 * normals by Box-Muller.  Draw order per particle: the step count (uniform in
 * [n_min, n_max]), entry x (uniform over the channel), entry angles thx, thy
 * (normal, sigma theta_sigma), then per step dthx, dthy.
 *
 * Conventions as in rad.h.
 */
#ifndef RAD_TRAJ_H
#define RAD_TRAJ_H

#include <stddef.h>
#include <stdint.h>

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double energy_eV;   /* entry energy E (> m_e) */
    double charge;      /* +1 positron (feels U), -1 electron (feels -U) */
    double U0_eV;       /* well depth */
    double d_m;         /* plane spacing d (> 0) */
    double q;           /* quartic fraction in [0, 1] */
    double length_m;    /* crystal thickness (> 0) */
    double theta_sigma; /* entry angle standard deviation [rad] */
    double X0_m;        /* radiation length (> 0) */
    double eps_s_eV;    /* scattering energy constant (10.6 MeV in Sec. III) */
    int32_t ms_on;      /* multiple scattering on/off */
    int32_t loss_on;    /* radiative loss on/off */
    int64_t n_min;      /* steps per particle drawn uniformly in [n_min, n_max], n_min >= 1 */
    int64_t n_max;
    uint64_t seed;
} rad_traj_params;

#define RAD_TRAJ_NCOL 11

/* Steps n_i of particles first .. first + n_particles - 1 (HOST int64 out[n_particles]);
 * particle i has n_i + 1 samples.  Pure host computation. */
rad_status rad_traj_lengths(const rad_traj_params *p, int64_t first, int n_particles, int64_t *out);

/* DEVICE workspace bytes of rad_traj_generate for particles first .. first +
 * n_particles - 1: their descriptors and, with scattering on, the unit normals of
 * every kick (16 bytes per step and particle, drawn in parallel before the
 * integration).  0 for invalid arguments. */
size_t rad_traj_workspace_bytes(const rad_traj_params *p, int64_t first, int n_particles);

/* DEVICE workspace bytes of rad_traj_sections (40 bytes per section). */
size_t rad_traj_sections_workspace_bytes(int n_particles, int n_sections);

/*
 * Generate particles first .. first + n_particles - 1 into cols (DEVICE double
 * [RAD_TRAJ_NCOL][total_samples], column-major over all samples: column c of
 * particle i starts at cols + c * total_samples + off_i, off_i = sum_{j<i} (n_j + 1)).
 * total_samples must equal sum_i (n_i + 1) (rad_traj_lengths).  The kick normals
 * are drawn first, in parallel over (step, particle) (splitmix64 is counter-based),
 * then one GPU thread integrates each particle; asynchronous on `stream` (returns
 * once the small descriptor upload has completed); deterministic.
 * RAD_EINVAL on invalid parameters or sizes.
 */
rad_status rad_traj_generate(const rad_traj_params *p, int64_t first, int n_particles, double *cols,
                             int64_t total_samples, void *ws, size_t ws_bytes, void *stream);

/*
 * Cut the trajectories that rad_traj_generate wrote into `cols` into n_sections
 * sections each (the paper's sections, Sec. II: the energy is fixed per section and
 * the section spectra add).  Section s of particle i holds samples k_s .. k_{s+1}
 * (both ends; k_s = floor(s n_i / n_sections)), with gamma_s = E(k_s) / m_e and dz,
 * dvz re-referenced to beta_s = 1 - 1/(2 gamma_s^2): dvz += 1/(2 gamma_s^2) -
 * 1/(2 gamma_ref^2), dz += (the same) t; t, x, y, vx, vy and the accelerations are
 * copied.  sec_cols (DEVICE double [RAD_TRAJ_NCOL][total_section_samples]) receives
 * the sections in (particle, section) order, packed like cols; total_section_samples
 * must equal sum_i (n_i + n_sections).  entry_energy (HOST double
 * [n_particles][n_sections]) receives E(k_s), from which the caller forms the
 * segments' gamma and energy.  Needs n_min >= n_sections.  ws: DEVICE workspace of
 * rad_traj_sections_workspace_bytes(n_particles, n_sections) bytes.  Synchronises
 * `stream` (the entry energies are copied to the host).
 */
rad_status rad_traj_sections(const rad_traj_params *p, int64_t first, int n_particles, int n_sections,
                             const double *cols, int64_t total_samples, double *sec_cols,
                             int64_t total_section_samples, double *entry_energy, void *ws, size_t ws_bytes,
                             void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAD_TRAJ_H */

/*
 * Seeded synthetic channeling trajectories (inputs only; no radiation integral
 * is evaluated here).
 *
 * Model, after Sec. III of Nielsen (arXiv:1910.10391), simplified where the
 * paper's tables are not available:
 *   - planar continuum well, periodic with the plane spacing d:
 *       U(x) = U0 [ (1-q) (2x/d)^2 + q (2x/d)^4 ],  x reduced to [-d/2, d/2);
 *     positrons (charge +1) feel U, electrons (charge -1) feel -U, which puts
 *     their minimum on the planes with a cusp;
 *   - transverse motion d(vx)/dt = -charge U'(x) / E, RK4 with a fixed step
 *     (the paper uses adaptive RK45 with a step floor, Sec. IV);
 *   - multiple Coulomb scattering on nuclei as Gaussian kicks of vx and vy
 *     after every step, mean square (eps_s/E)^2 dz / X0 (Sec. III, the nuclear
 *     term with a uniform density; the electron term needs X-ray tables that
 *     are not available);
 *   - radiative energy loss: the leading (Larmor) term of the Landau-Lifshitz
 *     force, dE/dt = -(2/3) alpha hbar c gamma^4 ax^2, plus the loss per
 *     deflection dE_MS = (m_e alpha / 2 pi) gamma^3 theta^2 (Sec. III);
 *   - accelerations are central differences of the stored post-kick velocity
 *     (one-sided at the ends), so the kicks radiate.
 * Longitudinal variables are kept relative to beta_ref = 1 - 1/(2 gamma_ref^2)
 * with gamma_ref the entry Lorentz factor: dvz = 1/(2g_ref^2) - 1/(2g^2) -
 * (vx^2+vy^2)/2, dz = int dvz dt (trapezoid).
 *
 * Random numbers: splitmix64 (Steele, Lea, Flood 2014) keyed by (seed,
 * particle), normals by Box-Muller with the logarithm and cosine below.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double energy_eV;   /* entry energy */
    double charge;      /* +1 positron, -1 electron */
    double U0_eV;       /* well depth */
    double d_m;         /* plane spacing */
    double q;           /* quartic fraction */
    double length_m;    /* crystal thickness */
    double theta_sigma; /* entry angle sigma [rad] */
    double X0_m;        /* radiation length */
    double eps_s_eV;    /* multiple-scattering energy constant */
    int32_t ms_on;
    int32_t loss_on;
    int64_t n_min;      /* steps per trajectory drawn uniformly in [n_min, n_max] */
    int64_t n_max;
    uint64_t seed;
} chan_params;

static const double SYN_ME_EV = 0.51099895e6;
static const double SYN_ALPHA = 7.2973525693e-3;
static const double SYN_HBARC = 1.973269804e-7;
static const double SYN_PI = 3.14159265358979323846;

typedef struct { uint64_t s; } rng_t;

static uint64_t splitmix64(rng_t *r)
{
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double u01(rng_t *r) /* (0, 1] */
{
    return ((double)(splitmix64(r) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

/*
 * log and cos for the normal draws, from IEEE operations only (+ - * / sqrt and exact
 * bit manipulation; this file is built without FMA contraction), so that another
 * implementation that evaluates the same series in the same order -- the GPU
 * generator's -- draws the same bits; the C library's log and cos and a device's round
 * differently in the last bit now and then.
 *
 * log u, u in (0, 1]: u = m 2^e with m in [sqrt(1/2), sqrt(2)), log u = e ln 2 +
 * 2 atanh s, s = (m - 1) / (m + 1), |s| <= 0.172, by the atanh series to s^23 (the next
 * term is below 2^-60 of the sum).
 */
double syn_log(double u)
{
    uint64_t b;
    memcpy(&b, &u, sizeof b);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    b = (b & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &b, sizeof m);
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

/*
 * cos(2 pi u), u in [0, 1]: v = min(u, 1 - u) in [0, 1/2] and w = v - 1/4 (both exact
 * for u on the 2^-53 grid), cos(2 pi u) = -sin(x) with x = 2 pi w, |x| <= pi/2, by the
 * sine's Taylor series to x^23.
 */
double syn_cos2pi(double u)
{
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

static double normal(rng_t *r)
{
    const double u1 = u01(r), u2 = u01(r);
    return sqrt(-2.0 * syn_log(u1)) * syn_cos2pi(u2);
}

static rng_t particle_rng(uint64_t seed, int64_t particle)
{
    rng_t r;
    r.s = seed * 0x9E3779B97F4A7C15ull ^ ((uint64_t)particle + 1ull) * 0xD1B54A32D192ED03ull;
    (void)splitmix64(&r);
    return r;
}

static int64_t draw_length(const chan_params *p, rng_t *r)
{
    if (p->n_max <= p->n_min) return p->n_min;
    const double u = u01(r) - 1e-300;
    int64_t n = p->n_min + (int64_t)floor((double)(p->n_max - p->n_min + 1) * u);
    if (n > p->n_max) n = p->n_max;
    return n;
}

/* dU/dx of the periodic well for unit positive charge; inv_d = 1 / d (multiplications
 * instead of divisions: the GPU generator, whose steps are latency-bound, takes the same
 * operations) */
static double well_slope(const chan_params *p, double x, double inv_d)
{
    const double d = p->d_m;
    const double xr = x - d * floor(x * inv_d + 0.5);
    const double u = 2.0 * xr * inv_d;
    return p->U0_eV * ((1.0 - p->q) * 2.0 * u + p->q * 4.0 * u * u * u) * (2.0 * inv_d);
}

/* Number of steps of each particle (the first draw of its stream). */
int chan_lengths(const chan_params *p, int64_t n_particles, int64_t first, int64_t *n_out)
{
    for (int64_t i = 0; i < n_particles; ++i) {
        rng_t r = particle_rng(p->seed, first + i);
        n_out[i] = draw_length(p, &r);
    }
    return 0;
}

/*
 * One trajectory of n steps (n+1 samples).  Columns (each n+1 doubles):
 * t, x, y, dz_ref, vx, vy, dvz_ref, ax, ay, az, energy.
 */
int chan_generate(const chan_params *p, int64_t particle, int64_t n, double *t, double *x,
                  double *y, double *dz, double *vx, double *vy, double *dvz, double *ax,
                  double *ay, double *az, double *energy)
{
    rng_t r = particle_rng(p->seed, particle);
    const int64_t n_drawn = draw_length(p, &r);
    if (n != n_drawn || n < 1) return 1;
    const double h = p->length_m / (double)n;
    const double g_ref = p->energy_eV / SYN_ME_EV;
    const double inv2g2_ref = 0.5 / (g_ref * g_ref);
    const double inv_me = 1.0 / SYN_ME_EV, inv_d = 1.0 / p->d_m;
    const double s = p->charge;
    double E = p->energy_eV;
    double xc = (u01(&r) - 0.5) * p->d_m;
    double vxc = p->theta_sigma * normal(&r);
    double vyc = p->theta_sigma * normal(&r);
    double yc = 0.0, dzc = 0.0;
    for (int64_t k = 0; k <= n; ++k) {
        const double g = E * inv_me;
        const double dvzc = inv2g2_ref - 0.5 / (g * g) - 0.5 * (vxc * vxc + vyc * vyc);
        t[k] = h * (double)k;
        x[k] = xc; y[k] = yc; vx[k] = vxc; vy[k] = vyc; dvz[k] = dvzc; dz[k] = dzc;
        energy[k] = E;
        if (k == n) break;
        /* RK4 on (x, vx) with E frozen over the step */
        const double f = -s / E;
        const double k1x = vxc, k1v = f * well_slope(p, xc, inv_d);
        const double k2x = vxc + 0.5 * h * k1v, k2v = f * well_slope(p, xc + 0.5 * h * k1x, inv_d);
        const double k3x = vxc + 0.5 * h * k2v, k3v = f * well_slope(p, xc + 0.5 * h * k2x, inv_d);
        const double k4x = vxc + h * k3v, k4v = f * well_slope(p, xc + h * k3x, inv_d);
        xc += h / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        vxc += h / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
        yc += h * vyc;
        /* radiative loss over the step: Larmor term with the mean acceleration */
        if (p->loss_on) {
            const double a_mean = (k1v + 2.0 * k2v + 2.0 * k3v + k4v) / 6.0;
            E -= h * (2.0 / 3.0) * SYN_ALPHA * SYN_HBARC * g * g * g * g * a_mean * a_mean;
        }
        /* multiple scattering kick and its energy loss */
        if (p->ms_on) {
            const double sig = (p->eps_s_eV / E) * sqrt(h / p->X0_m);
            const double dtx = sig * normal(&r), dty = sig * normal(&r);
            vxc += dtx;
            vyc += dty;
            if (p->loss_on)
                E -= SYN_ME_EV * SYN_ALPHA / (2.0 * SYN_PI) * g * g * g * (dtx * dtx + dty * dty);
        }
        const double g1 = E * inv_me;
        const double dvz1 = inv2g2_ref - 0.5 / (g1 * g1) - 0.5 * (vxc * vxc + vyc * vyc);
        dzc += 0.5 * h * (dvzc + dvz1);
    }
    /* accelerations: central differences of the stored velocities */
    for (int64_t k = 0; k <= n; ++k) {
        const int64_t lo = k > 0 ? k - 1 : 0, hi = k < n ? k + 1 : n;
        const double dt = t[hi] - t[lo];
        ax[k] = (vx[hi] - vx[lo]) / dt;
        ay[k] = (vy[hi] - vy[lo]) / dt;
        az[k] = (dvz[hi] - dvz[lo]) / dt;
    }
    (void)SYN_HBARC;
    return 0;
}

int chan_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Direct-sum CPU oracle for the radiation integrals.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * library: the constants below are typed in again on purpose.
 *
 * What it computes (Nielsen, "GPU accelerated simulation of channeling
 * radiation of relativistic particles", arXiv:1910.10391):
 *
 *   Sec. II, eq. (integralrad1)-(integralrad2): the classical spectrum
 *     d2I/(dw dOmega) = e^2/(4 pi^2) |int f(t,n) exp(i w (t - n.x(t))) dt|^2
 *   Sec. II, small-angle expansion (the f_x, f_y, f_z, g and phase displays
 *     that follow eq. (integralrad2)), in the variables dz = z - beta0 t,
 *     dvz = v_z - beta0, beta0 = 1 - 1/(2 gamma^2), theta^2 = nx^2 + ny^2.
 *   Sec. II, eq. (Lindhard_substi): spin-0 by the substitution
 *     w -> w* = w / (1 - hw/E), dI_q/dhw(w) = (w / w*) dI_c/dhw(w*).
 *   Sec. II, eq. (cue)-(Iterm): spin-1/2 (BCK) spectrum
 *     e^2/(4 pi^2) [ (E*^2+E^2)/(2E^2) |I|^2 + hw^2/(2 E^2 gamma^2) |J|^2 ]
 *     with E* = E - hw and I, J integrated with exp(i w* (t - n.r)).
 *
 * Units: c = 1, t and lengths in metres, photon energies in eV, the
 * wavenumber kappa = hw / (hbar c) in 1/m.  Output spectra are
 * d2I/(d(hbar w) dOmega), dimensionless: alpha/(4 pi^2) |A|^2.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - quadrature in t: trapezoid weights from t unless explicit weights are
 *     given;
 *   - J's numerator n.beta_dot is expanded with n_z -> 1, the same order as
 *     the (a_z + ...) factors of f_x and f_y:  Q = (nx ax + ny ay + az) g;
 *   - |I|^2 includes the z component;
 *   - spin-0 is applied direction by direction: (E* over E) times |A(kappa*)|^2, E* = E - hw;
 *   - hw >= E in a quantum spectrum gives 0.
 *
 * Plain scalar loops, libm sin/cos, compiled without fast-math and without
 * FMA contraction.  One (kappa, direction) integral per loop iteration,
 * parallel over iterations with OpenMP, like the paper's CPU twin (Sec. V).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 */
static const double ORACLE_HBARC_EVM = 1.973269804e-7; /* hbar c [eV m] */
static const double ORACLE_ALPHA = 7.2973525693e-3;    /* fine-structure constant */
static const double ORACLE_PI = 3.14159265358979323846;

typedef struct {
    int64_t n;
    const double *t, *x, *y, *dz, *vx, *vy, *dvz, *ax, *ay, *az;
    const double *w; /* NULL -> trapezoid from t */
    double gamma;
} oracle_seg;

/* Trapezoid weight of sample k (reading: the paper does not name its rule). */
static double oracle_weight(const oracle_seg *s, int64_t k)
{
    if (s->w) return s->w[k];
    if (s->n < 2) return 0.0;
    if (k == 0) return 0.5 * (s->t[1] - s->t[0]);
    if (k == s->n - 1) return 0.5 * (s->t[s->n - 1] - s->t[s->n - 2]);
    return 0.5 * (s->t[k + 1] - s->t[k - 1]);
}

/*
 * Amplitudes for one wavenumber kappa and one direction (nx, ny):
 *   A = sum_k w_k f(t_k, n) exp(i kappa psi_k)          (3 complex components)
 *   J = sum_k w_k (n.beta_dot)/(1-n.beta)^2 exp(i kappa psi_k)
 * with f, g and psi written exactly as in the Sec. II expansion:
 *   g   = (1/(2g^2) + th^2/2 - dvz - nx vx - ny vy)^-2
 *   f_x = [(az + ny ay)(nx - vx) - (ny (ny - vy) + C) ax] g
 *   f_y = [(az + nx ax)(ny - vy) - (nx (nx - vx) + C) ay] g
 *   f_z = [C (nx ax + ny ay) - (nx (nx - vx) + ny (ny - vy)) az] g
 *   C   = -th^2/2 - dvz + 1/(2 gamma^2)
 *   psi = (1/(2 gamma^2) + th^2/2) t - dz - nx x - ny y
 */
static void oracle_amplitude(const oracle_seg *s, double kappa, double nx, double ny,
                             double A[6], double J[2])
{
    const double c0 = 1.0 / (2.0 * s->gamma * s->gamma);
    const double th2 = nx * nx + ny * ny;
    double axr = 0, axi = 0, ayr = 0, ayi = 0, azr = 0, azi = 0, jr = 0, ji = 0;
    for (int64_t k = 0; k < s->n; ++k) {
        const double vx = s->vx[k], vy = s->vy[k], dvz = s->dvz[k];
        const double ax = s->ax[k], ay = s->ay[k], az = s->az[k];
        const double den = c0 + th2 / 2.0 - dvz - nx * vx - ny * vy;
        const double g = 1.0 / (den * den);
        const double C = -th2 / 2.0 - dvz + c0;
        const double fx = ((az + ny * ay) * (nx - vx) - (ny * (ny - vy) + C) * ax) * g;
        const double fy = ((az + nx * ax) * (ny - vy) - (nx * (nx - vx) + C) * ay) * g;
        const double fz = (C * (nx * ax + ny * ay) - (nx * (nx - vx) + ny * (ny - vy)) * az) * g;
        const double q = (nx * ax + ny * ay + az) * g;
        const double psi = (c0 + th2 / 2.0) * s->t[k] - s->dz[k] - nx * s->x[k] - ny * s->y[k];
        const double ph = kappa * psi;
        const double c = cos(ph), sn = sin(ph);
        const double wk = oracle_weight(s, k);
        axr += wk * fx * c; axi += wk * fx * sn;
        ayr += wk * fy * c; ayi += wk * fy * sn;
        azr += wk * fz * c; azi += wk * fz * sn;
        jr += wk * q * c;   ji += wk * q * sn;
    }
    A[0] = axr; A[1] = axi; A[2] = ayr; A[3] = ayi; A[4] = azr; A[5] = azi;
    J[0] = jr; J[1] = ji;
}

static void oracle_set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Raw amplitudes on a list of wavenumbers and a list of directions.
 * A_out: [n_kappa][n_dir][6] (x re, x im, y re, y im, z re, z im)
 * J_out: [n_kappa][n_dir][2] or NULL.
 */
int oracle_amplitudes(int64_t n, const double *t, const double *x, const double *y,
                      const double *dz, const double *vx, const double *vy, const double *dvz,
                      const double *ax, const double *ay, const double *az, const double *w,
                      double gamma, int64_t n_kappa, const double *kappa, int64_t n_dir,
                      const double *nx, const double *ny, double *A_out, double *J_out,
                      int n_threads)
{
    oracle_seg s = {n, t, x, y, dz, vx, vy, dvz, ax, ay, az, w, gamma};
    if (n < 0 || n_kappa < 0 || n_dir < 0) return 1;
    oracle_set_threads(n_threads);
    const int64_t total = n_kappa * n_dir;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t it = 0; it < total; ++it) {
        const int64_t i = it / n_dir, j = it % n_dir;
        double A[6], J[2];
        oracle_amplitude(&s, kappa[i], nx[j], ny[j], A, J);
        for (int c = 0; c < 6; ++c) A_out[it * 6 + c] = A[c];
        if (J_out) { J_out[it * 2] = J[0]; J_out[it * 2 + 1] = J[1]; }
    }
    return 0;
}

/*
 * Spectra of one segment on the grid hw[n_w] x thy[n_y] x thx[n_x].
 * kinds: bit 1 classical, bit 2 spin-0, bit 4 spin-1/2.  out holds one cube
 * [n_w][n_y][n_x] per requested kind, in the order classical, spin-0, spin-1/2.
 * energy_eV is the particle energy E fixed for the segment (Sec. II, sections).
 */
int oracle_spectrum(int64_t n, const double *t, const double *x, const double *y,
                    const double *dz, const double *vx, const double *vy, const double *dvz,
                    const double *ax, const double *ay, const double *az, const double *w,
                    double gamma, double energy_eV, int n_w, const double *hw, int n_x,
                    const double *thx, int n_y, const double *thy, int kinds, double *out,
                    int n_threads)
{
    oracle_seg s = {n, t, x, y, dz, vx, vy, dvz, ax, ay, az, w, gamma};
    if (n < 0 || n_w < 0 || n_x < 0 || n_y < 0 || (kinds & ~7) || !kinds) return 1;
    oracle_set_threads(n_threads);
    const int want_c = kinds & 1, want_0 = (kinds >> 1) & 1, want_h = (kinds >> 2) & 1;
    const int64_t cube = (int64_t)n_w * n_y * n_x;
    double *out_c = out;
    double *out_0 = out + (int64_t)want_c * cube;
    double *out_h = out + (int64_t)(want_c + want_0) * cube;
    const double pref = ORACLE_ALPHA / (4.0 * ORACLE_PI * ORACLE_PI);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t it = 0; it < cube; ++it) {
        const int64_t i = it / ((int64_t)n_y * n_x);
        const int64_t jy = (it / n_x) % n_y;
        const int64_t jx = it % n_x;
        const double e_ph = hw[i];
        const double k = e_ph / ORACLE_HBARC_EVM;
        double A[6], J[2];
        if (want_c) {
            oracle_amplitude(&s, k, thx[jx], thy[jy], A, J);
            const double S = A[0] * A[0] + A[1] * A[1] + A[2] * A[2] + A[3] * A[3] +
                             A[4] * A[4] + A[5] * A[5];
            out_c[it] = pref * S;
        }
        if (want_0 || want_h) {
            double s0 = 0.0, sh = 0.0;
            if (e_ph < energy_eV) {
                const double E = energy_eV, Es = energy_eV - e_ph;
                const double kstar = k * E / Es; /* w* = w / (1 - hw/E) */
                oracle_amplitude(&s, kstar, thx[jx], thy[jy], A, J);
                const double S = A[0] * A[0] + A[1] * A[1] + A[2] * A[2] + A[3] * A[3] +
                                 A[4] * A[4] + A[5] * A[5];
                const double SJ = J[0] * J[0] + J[1] * J[1];
                s0 = pref * (Es / E) * S;
                sh = pref * ((Es * Es + E * E) / (2.0 * E * E) * S +
                             e_ph * e_ph / (2.0 * E * E * gamma * gamma) * SJ);
            }
            if (want_0) out_0[it] = s0;
            if (want_h) out_h[it] = sh;
        }
    }
    return 0;
}

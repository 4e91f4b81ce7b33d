/*
 * rad.h -- C ABI of librad, the MI355X (gfx950) radiation-integral library.
 *
 * The library evaluates, on one GPU, the radiation integrals of Nielsen,
 * "GPU accelerated simulation of channeling radiation of relativistic
 * particles" (arXiv:1910.10391), Sec. II:
 *
 *   classical (eq. (integralrad1)-(integralrad2)), in the Sec. II small-angle
 *   expansion:  d2I/(d hw dOmega) = alpha/(4 pi^2) |A(k)|^2,
 *     A(kappa) = int f(t, n) exp(i kappa psi(t, n)) dt,  k = hw / (hbar c),
 *     psi = (1/(2 gamma^2) + theta^2/2) t - dz - n_x x - n_y y;
 *   spin-0, substitution model (eq. (Lindhard_substi)):
 *     alpha/(4 pi^2) (E* / E) |A(k*)|^2,  k* = k E / (E - hw),  E* = E - hw;
 *   spin-1/2, BCK model (eq. (cue)-(Iterm)):
 *     alpha/(4 pi^2) [ (E*^2 + E^2)/(2 E^2) |A(k*)|^2 + hw^2/(2 E^2 gamma^2) |J(k*)|^2 ],
 *     J(kappa) = int (n . beta_dot)/(1 - n . beta)^2 exp(i kappa psi) dt,
 *     with n . beta_dot expanded as n_x a_x + n_y a_y + a_z;
 *   sections (Sec. II, end): a trajectory is cut into segments with the energy
 *   fixed at each segment's entry; the spectrum of the trajectory is the sum
 *   of the segment spectra;
 *   dI/d hw (Sec. IV): the sum of the cube over the angular cells.
 *
 * Conventions shared by every call:
 *   - Units: c = 1, t and lengths in metres, velocities are beta, accelerations
 *     are d(beta)/dt in 1/m, photon and particle energies in eV.  Output spectra
 *     are d2I/(d hw dOmega), dimensionless.
 *   - Cube layout: [n_w][n_y][n_x], row-major (x fastest), FP64.
 *   - Pointers marked DEVICE are GPU global-memory pointers on the current HIP
 *     device (e.g. torch's data_ptr()); HOST pointers are CPU memory.  The
 *     caller owns every buffer.  A grid handle owns only its own device copy of
 *     the grid.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Compute
 *     calls are asynchronous on it and make no host synchronisation.
 *   - Workspaces are caller-provided device memory; compute calls allocate no
 *     device memory.  They stage their launch descriptors through the grid's
 *     pinned host buffer (1 MiB from rad_setup_grid, about 1000 segments' worth);
 *     only a call whose descriptors need more grows it to that size.
 *     rad_batch_static allocates nothing at all.
 *   - Errors: every call returns a status and never aborts or throws across the
 *     ABI.  Arguments are validated before any launch; on error nothing is
 *     launched and rad_last_error() holds a message (thread-local).
 *   - A photon energy hw >= E is kinematically forbidden in the quantum
 *     spectra: those entries are 0, not an error.
 *   - Results are bitwise reproducible run to run (fixed-order reductions, no
 *     floating-point atomics).
 */
#ifndef RAD_H
#define RAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rad_grid rad_grid; /* opaque, immutable after setup */

typedef enum {
    RAD_OK = 0,
    RAD_EINVAL = 1,       /* invalid argument (null pointer, bad size, bad value) */
    RAD_ENOMEM = 2,       /* workspace too small, or device allocation failed in setup */
    RAD_EDEVICE = 3,      /* HIP runtime error (no device, launch failure) */
    RAD_EUNSUPPORTED = 4  /* valid request the library does not implement */
} rad_status;

typedef enum { RAD_CLASSICAL = 1, RAD_SPIN0 = 2, RAD_SPINHALF = 4 } rad_kind; /* bitmask */

typedef enum {
    RAD_FP64 = 0,  /* FP64 throughout */
    RAD_MIXED = 1  /* FP64 phase, range reduction and accumulation; FP32 integrand and sincos */
} rad_precision;

/*
 * One trajectory segment (the paper's section, Sec. II), columns as DEVICE
 * pointers, each n FP64 values (structure of arrays), in the small-angle
 * variables of Sec. II: dz = z - beta0 t, dvz = v_z - beta0 with
 * beta0 = 1 - 1/(2 gamma^2).
 */
typedef struct {
    int64_t n;               /* samples, >= 2 */
    const double *t;         /* time (= path length, c = 1) [m], increasing */
    const double *x, *y;     /* transverse position [m] */
    const double *dz;        /* z - beta0 t [m] */
    const double *vx, *vy;   /* transverse beta */
    const double *dvz;       /* v_z - beta0 */
    const double *ax, *ay, *az; /* d(beta)/dt [1/m] */
    const double *w;         /* quadrature weights [m], or NULL for the trapezoid rule from t */
    double gamma;            /* Lorentz factor of the expansion reference (> 0) */
    double energy_eV;        /* particle energy E at segment entry (> 0; quantum kinds only) */
} rad_segment;

/*
 * Build a grid handle: photon energies hw_eV[n_w] (> 0), directions
 * thx[n_x] = n_x and thy[n_y] = n_y [rad] (HOST arrays, copied).  The angle
 * integral uses cell widths half-way between neighbours (a single point has
 * width 1).  When thx and thy are uniform with one common spacing d (to within
 * 8 units in the last place of the largest angle), the FP64 kernels form the
 * phase factors of a direction tile by recurrence along each axis (the phase is
 * quadratic in the direction index; Sec. II), see rad_grid_step.  Allocates
 * device memory and 1 MiB of pinned host memory through which compute calls upload
 * their launch descriptors; may synchronise `stream`.
 * Errors: RAD_EINVAL for null pointers, sizes < 1 or non-finite values;
 * RAD_ENOMEM / RAD_EDEVICE on allocation or copy failure.
 */
rad_status rad_setup_grid(const double *hw_eV, int n_w, const double *thx, int n_x,
                          const double *thy, int n_y, void *stream, rad_grid **out);

/* Release a grid handle (NULL is ignored).  The caller must not free it while
 * calls that use it are still running on a stream. */
void rad_free_grid(rad_grid *grid);

/* Grid sizes (any pointer may be NULL). */
rad_status rad_grid_dims(const rad_grid *grid, int *n_w, int *n_x, int *n_y);

/* The common direction spacing d the FP64 kernels use for their phase recurrence,
 * or 0 when thx or thy is not uniform or their spacings differ (phase factors are
 * then evaluated directly).  Errors: RAD_EINVAL for a NULL grid or dth. */
rad_status rad_grid_step(const rad_grid *grid, double *dth);

/*
 * Workspace bytes that rad_classical / rad_quantum need for any segment with
 * n <= max_n samples and the given kinds (RAD_CLASSICAL for rad_classical, a
 * subset of RAD_SPIN0|RAD_SPINHALF for rad_quantum) and precision.  0 on
 * invalid arguments.
 */
size_t rad_workspace_bytes(const rad_grid *grid, int64_t max_n, int kinds, rad_precision prec);

/* Workspace bytes rad_batch needs for exactly this list of segments (HOST array)
 * and n_out outputs.  0 on invalid arguments. */
size_t rad_batch_workspace_bytes(const rad_grid *grid, const rad_segment *segs, int n_segs,
                                 int n_out, int kinds, rad_precision prec);

/*
 * Classical spectrum of one segment (Sec. II eq. (integralrad1)).
 * out: DEVICE [n_w][n_y][n_x] FP64, overwritten.  ws: DEVICE workspace of
 * ws_bytes >= rad_workspace_bytes(grid, seg->n, RAD_CLASSICAL, prec).
 * Errors: RAD_EINVAL (null pointers, n < 2, gamma <= 0), RAD_ENOMEM (ws too
 * small), RAD_EDEVICE (launch failure).
 */
rad_status rad_classical(const rad_grid *grid, const rad_segment *seg, rad_precision prec,
                         double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Semi-classical spectra of one segment: kinds is a non-empty subset of
 * RAD_SPIN0 | RAD_SPINHALF (Sec. II eq. (Lindhard_substi) and eq. (cue)).
 * out: DEVICE [popcount(kinds)][n_w][n_y][n_x], spin-0 first, overwritten.
 * Needs seg->energy_eV > 0.  Errors as rad_classical.
 */
rad_status rad_quantum(const rad_grid *grid, const rad_segment *seg, int kinds, rad_precision prec,
                       double *out, void *ws, size_t ws_bytes, void *stream);

/*
 * Many segments in one call (uneven lengths), summed per output: segment s is
 * added to output out_index[s] (HOST array, 0 <= out_index[s] < n_out); the
 * sum runs in segment order, so it is deterministic (Sec. II, sections).
 * kinds: any non-empty subset of RAD_CLASSICAL | RAD_SPIN0 | RAD_SPINHALF.
 * out: DEVICE [n_out][popcount(kinds)][n_w][n_y][n_x], kinds in the order
 * classical, spin-0, spin-1/2; overwritten (outputs with no segment are 0).
 * ws_bytes >= rad_batch_workspace_bytes(grid, segs, n_segs, kinds, prec).
 */
rad_status rad_batch(const rad_grid *grid, const rad_segment *segs, int n_segs,
                     const int *out_index, int n_out, int kinds, rad_precision prec, double *out,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * rad_batch for callers that cannot allocate: code under hipGraph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * errors as rad_batch, without the workspace: the segment descriptors and partial
 * amplitudes live in a fixed device array of rad_static_scratch_bytes() (64 MiB)
 * that the library holds on every GPU it runs on until the process ends; the
 * descriptors are written into it by kernels (no host staging buffer), and the
 * call allocates no device or pinned host memory.  The time chunks are coarsened
 * (down to one per segment) until the work fits, so results equal rad_batch's to
 * rounding (bitwise where the chunking is the same).  Errors: as rad_batch, and
 * RAD_ENOMEM when even one chunk per segment needs more than the fixed scratch
 * (then nothing is launched).  All calls on one GPU share its array and it keeps
 * the last call's contents: calls that overlap in time on one GPU (two streams,
 * two threads) race and give wrong results; serialise them.
 */
size_t rad_static_scratch_bytes(void);
rad_status rad_batch_static(const rad_grid *grid, const rad_segment *segs, int n_segs,
                            const int *out_index, int n_out, int kinds, rad_precision prec,
                            double *out, void *stream);

/*
 * Persistent, replayable batches.  A plan fixes one rad_batch call's segments,
 * outputs, kinds, precision and workspace: rad_plan_create validates, orders the
 * work longest segment first and writes the work list into `ws` (synchronising
 * `stream` once).  rad_plan_launch then issues only kernels -- a ticket reset, a
 * persistent amplitude kernel per integral set whose resident blocks pull work
 * items from the list, and the finalize kernel -- with no host copy and no
 * allocation.  rad_plan_launch_graph captures that sequence into a hipGraph on
 * its first call for a given `out` and replays the graph afterwards; it needs a
 * created (non-default) stream.  The plan keeps pointers to the grid, the
 * segment columns and `ws`: they must stay valid and unchanged while the plan
 * is used.  Calls on one plan must not overlap in time (they share the work
 * list's tickets).  Results equal rad_batch's to rounding; repeated launches of
 * one plan, eager or from the graph, are bitwise identical.
 * ws_bytes >= rad_batch_workspace_bytes(grid, segs, n_segs, n_out, kinds, prec).
 */
typedef struct rad_plan rad_plan;
rad_status rad_plan_create(const rad_grid *grid, const rad_segment *segs, int n_segs,
                           const int *out_index, int n_out, int kinds, rad_precision prec,
                           void *ws, size_t ws_bytes, void *stream, rad_plan **plan);
rad_status rad_plan_launch(rad_plan *plan, double *out, void *stream);
rad_status rad_plan_launch_graph(rad_plan *plan, double *out, void *stream);
void rad_plan_free(rad_plan *plan);

/*
 * The phase factor e^{i phi} as the integral kernels compute it, on given arguments,
 * for measuring its accuracy.  RAD_FP64: turns[k] = phi/pi (half turns); cos(pi u) and
 * sin(pi u) from the exact reduction f = u - rint(u) and Chebyshev fits in f on
 * [-1/2, 1/2].  RAD_MIXED: turns[k] = phi/(2 pi) (revolutions); the FP64 reduction
 * r - rint(r), rounded to FP32, then the hardware FP32 sine and cosine of revolutions.
 * turns, c, s: DEVICE double [n]; c[k] = cos, s[k] = sin.  |turns[k]| must stay below
 * 2^51.  Errors: RAD_EINVAL for an unknown precision, n outside [0, 2^40] or a buffer
 * that is not n doubles of device memory; nothing is launched for n = 0.
 */
rad_status rad_phase_factors(const double *turns, int64_t n, rad_precision prec, double *c, double *s,
                             void *stream);

/*
 * Angle integral (Sec. IV): dIdw[c][i] = sum_{jy,jx} cube[c][i][jy][jx] dthx[jx] dthy[jy]
 * for n_cubes consecutive DEVICE cubes; dIdw is DEVICE [n_cubes][n_w].
 */
rad_status rad_angle_integrate(const rad_grid *grid, const double *cube, int n_cubes, double *dIdw,
                               void *stream);

/*
 * Exact cell integrals for the learned angular sampler's refinement.  The
 * directions of `grid` are split into cells of cx x cy (8 x 8 supported; n_x, n_y
 * must be multiples): cell c = (ci, cj) covers thx[ci*cx .. ci*cx+cx-1] x
 * thy[cj*cy .. cj*cy+cy-1], cells numbered c = cj * (n_x/cx) + ci.  For every
 * segment s, photon energy w and cell c with mask[s][w][c] != 0 (HOST uint8
 * [n_segs][n_w][n_cells]) it writes
 *   cell_out[s][w][c] = sum over the cell's directions of the `kind` spectrum
 *                       (exactly one of RAD_CLASSICAL, RAD_SPIN0, RAD_SPINHALF)
 *                       times dthx dthy (the grid's angle-cell widths),
 * and 0 where the mask is 0 (cell_out: DEVICE [n_segs][n_w][n_cells]).  Only the
 * masked cells are computed (per block of 64 photon energies); segments are
 * single sections (no summing across segments).  ws_bytes >=
 * rad_cells_workspace_bytes(...) for the same mask.  Errors as rad_batch.
 */
size_t rad_cells_workspace_bytes(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                                 rad_precision prec, int cx, int cy, const uint8_t *mask);
rad_status rad_cells(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                     rad_precision prec, int cx, int cy, const uint8_t *mask, double *cell_out,
                     void *ws, size_t ws_bytes, void *stream);

/*
 * rad_cells with the mask in DEVICE memory (uint8 [n_segs][n_w][n_cells]), read by the
 * kernels when they run, so that a mask computed on the device (the sampler's
 * selection) needs no copy to the host and nothing waits for `stream`.  The launch
 * covers every (segment, cell, block of 64 photon energies); a block whose energies
 * have no mask bit set leaves at once, so the work done is that of rad_cells.  The
 * sums are those of rad_cells, but the time axis is cut into chunks planned for every
 * cell (rad_cells plans them for the masked cells only, and cuts finer when few are
 * masked), so the results equal rad_cells' to rounding, bitwise where the two plans
 * coincide (a full mask).  The workspace holds partial amplitudes for every cell
 * (ws_bytes >= rad_cells_device_workspace_bytes(...), which needs no mask).  Errors as rad_cells, plus RAD_EINVAL for a mask that is not
 * n_segs * n_w * n_cells bytes of device memory.
 */
size_t rad_cells_device_workspace_bytes(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                                        rad_precision prec, int cx, int cy);
rad_status rad_cells_device(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                            rad_precision prec, int cx, int cy, const uint8_t *mask, double *cell_out,
                            void *ws, size_t ws_bytes, void *stream);

/* Static text of a status code. */
const char *rad_status_string(rad_status status);

/* Message of the last failed call on this thread ("" if none). */
const char *rad_last_error(void);

/*
 * Tuning knobs of the amplitude kernel (process-wide), set by the autotuner.  A
 * variant fixes the direction tile each lane owns (0: 4x4, 1: 4x3, 2: 4x4 at one
 * resident block per CU, 3: 4x2, 4: 4x6) and the resident blocks per CU it is
 * compiled for (two unless stated).  It is chosen per form
 * (`persistent`: rad_plan_* vs the one-block-per-item calls), per precision
 * (`mixed`) and per integral set (`with_j`: the set that also carries J for
 * spin-1/2).  Every variant computes the same sums; only the speed differs.
 * A plan keeps the variants in force when it was created.
 * rad_tune_set_variant: RAD_EINVAL for an unknown variant; RAD_EUNSUPPORTED for
 * variant 4 with with_j set (its 24 directions leave no registers for J).
 */
rad_status rad_tune_set_variant(int persistent, int mixed, int with_j, int variant);
rad_status rad_tune_get_variant(int persistent, int mixed, int with_j, int *variant);
int rad_tune_num_variants(void);

/*
 * Launch-shape knobs (process-wide), also set by the autotuner.
 * rad_tune_set_shape: the waves of a block spread over photon energies, wg = 1, 2 or 4
 * (the block's other waves take further direction tiles: 4 / wg of them), per form and
 * precision; 0 (the default) chooses by the grid: 4 above 128 energies, 2 above 64, else
 * 1.  Every wg computes the same sums in the same order (the same bits).
 * rad_tune_set_chunk_target: segments are cut into time chunks until a launch has this
 * many work items (0, the default: 2048); the chunk sums then come in another order, so
 * results change by rounding only.  It applies to every form, and changes the workspace
 * sizes: query them after setting it.  RAD_EINVAL for wg outside {0, 1, 2, 4} or a target
 * outside [0, 2^24].  rad_tune_get_chunk_target returns the target in force.
 */
rad_status rad_tune_set_shape(int persistent, int mixed, int wg);
/*
 * The cell integrals' block shape (rad_cells, rad_cells_device).  A cell is evaluated
 * for each block of 64 photon energies that holds a selected energy.  0, the default,
 * groups these blocks: those of one (segment, cell, time chunk) are taken in order by
 * four, then two, then one, and a group of k blocks runs as k work items, each of whose
 * 4 waves takes one block and whose 4 / k direction tiles are among the cell's four
 * 4 x 4 tiles, so that each staged direction serves up to 256 energies; the sums are
 * those of wg = 1, bit for bit (grids of more than 256 blocks run as wg = 1).  wg = 1,
 * 2 or 4 fixes a block's spread: wg adjacent energy blocks for 4 / wg tiles (wg = 1: the
 * whole 8 x 8 cell for 64 energies), so wg > 1 evaluates a cell for whole groups of
 * 64 wg energies; its sums are those of wg = 1 to rounding (the time chunking follows the
 * item count, and so may the workspace sizes: query them after setting it).  RAD_EINVAL
 * for other values.  rad_tune_get_cell_spread returns the setting (0: grouped).
 */
rad_status rad_tune_set_cell_spread(int wg);
int rad_tune_get_cell_spread(void);
rad_status rad_tune_get_shape(int persistent, int mixed, int *wg);
rad_status rad_tune_set_chunk_target(int64_t target_blocks);
int64_t rad_tune_get_chunk_target(void);

/*
 * Index checks of the debug build (compiled with -DRAD_DEBUG=1, librad_debug.so): the
 * kernels check descriptor, time-chunk and partial-amplitude indices against the
 * launch's bounds, count each violation and skip that access.  Returns the count since
 * the last reset on the current device (synchronising it; reset != 0 clears the count),
 * -1 in a release build (no checks compiled), -2 if the device cannot be read.
 */
int64_t rad_debug_violations(int reset);

/*
 * Kernel timing for benchmarks: when enabled, every launch of the amplitude
 * kernel is bracketed by HIP events on the caller's stream.  rad_profile_read
 * waits for the recorded events and returns the summed kernel time [ms] and
 * the number of launches since the last reset.
 */
rad_status rad_profile_enable(int on);
rad_status rad_profile_read(double *kernel_ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* RAD_H */

/*
 * rad_sampler.h -- C ABI of the learned angular sampler's kernels (part of librad).
 *
 * The sampler estimates dI/d hw on a fine angular grid (n_x x n_y directions,
 * split into cells of cx x cy) from (1) the exact spectrum at the cell centres
 * (rad_batch on a coarse grid), (2) the MLP's predicted log intensity at every
 * fine direction (include/rad_mlp.h), (3) exact cell integrals on the cells the
 * prediction selects (rad_cells in include/rad.h); cells left out count as their
 * predicted mass, their centre value times their area, or their centre value
 * corrected by the predicted sub-cell shape.  Two selection rules: by predicted
 * mass (rad_sampler_select, where a prediction that disagrees with the exact centre
 * values makes a photon energy fall back to the full grid, the exact reference),
 * and by the predicted error of the midpoint value (rad_sampler_select_error).
 * Conventions as in rad.h.
 */
#ifndef RAD_SAMPLER_H
#define RAD_SAMPLER_H

#include <stddef.h>
#include <stdint.h>

#include "rad.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RAD_N_FEATURES 38

/*
 * Trajectory features for the network, one row of RAD_N_FEATURES floats per
 * segment (DEVICE feat [n_segs][38]): log(gamma / 1e4); a 32-bin histogram, over
 * [0, d/2] with d = plane_spacing_m, of the transverse oscillation amplitudes
 * (half the distance between consecutive sign changes of v_x; amplitudes >= d/2,
 * over-barrier motion, fall in the last bin), normalised to sum 1;
 * log(omega_osc / 1e5 m^-1) with omega_osc = pi (sign changes of v_x) / (t_end -
 * t_0); and the direction of motion in units of 1/gamma: gamma mean(v_x),
 * gamma mean(v_y), gamma std(v_x), gamma std(v_y) over the samples (the spread
 * about the mean, in two passes).  Uses t, x, vx, vy, n and gamma of each segment.
 * ws: DEVICE workspace of at least n_segs * 48 bytes.  Asynchronous: the segment
 * descriptors travel as kernel arguments, nothing waits for `stream`.
 */
rad_status rad_features(const rad_segment *segs, int n_segs, double plane_spacing_m, float *feat, void *ws,
                        size_t ws_bytes, void *stream);

/*
 * Cell selection per (trajectory, photon energy) of the fine grid `fine`:
 * pred (DEVICE float [n_traj][n_w][n_y][n_x]) is the network's output, the
 * predicted angular shape being exp(mu + sigma * pred) up to a scale; coarse
 * (DEVICE double [n_traj][n_w][n_cells]) the exact spectrum at the cell centres.
 * The predicted centre value P_c of a cell is the mean predicted value of the fine
 * directions nearest its centre (the central 2 x 2 of an even cell); the scale is
 * lambda = sum_c coarse_c A_c / sum_c P_c A_c (A_c the cell area).  Check: the
 * energy falls back to the full grid (every cell selected) when
 * sum_c |lambda P_c - coarse_c| A_c > tau * sum_c coarse_c A_c, or a sum is 0.
 * Otherwise cells are taken in decreasing predicted mass (lambda times the sum over
 * the cell's fine directions of the predicted value x dthx dthy) while the predicted
 * mass before them is below coverage * the total, at most `cap` cells.  The
 * selection is then widened to whole blocks of 64 photon energies (w / 64): a cell
 * selected for one energy of a block is selected for all of them, since rad_cells
 * evaluates a cell for a whole block at the cost of one.  Writes mask (DEVICE uint8
 * [n_traj][n_w][n_cells]), fallback (DEVICE uint8 [n_traj][n_w]) and, if cell_pred
 * is not NULL, the scaled predicted cell masses (DEVICE double
 * [n_traj][n_w][n_cells]).  Needs n_cells = (n_x/cx)(n_y/cy) <= 64.
 */
rad_status rad_sampler_select(const rad_grid *fine, int n_traj, const float *pred, float mu, float sigma,
                              const double *coarse, int cx, int cy, float coverage, int cap, float tau,
                              uint8_t *mask, uint8_t *fallback, double *cell_pred, void *stream);

/*
 * Error-driven cell selection, with the inputs of rad_sampler_select.  The
 * predicted sub-cell shape corrects each exact centre value: with M_c the predicted
 * cell mass (sum over the cell's fine directions of exp(mu + sigma pred) x dthx
 * dthy) and P_c the predicted centre value, the cell estimate is
 * E_c = coarse_c M_c / P_c (coarse_c A_c where P_c is 0); it does not depend on the
 * prediction's scale, and it is the exact cell integral when the prediction is the
 * true map and the centre value is a fine direction (odd cells).  e_c = |E_c -
 * coarse_c A_c| estimates the error of leaving the cell at its midpoint value.
 * Cells are taken in decreasing e_c (ties by index) while the estimated error of
 * the cells not yet taken (e_c plus that of every cell after it) exceeds
 * eps * sum_c E_c, at most `cap` cells; then widened to blocks of 64 photon
 * energies as in rad_sampler_select.  Writes mask (DEVICE uint8
 * [n_traj][n_w][n_cells]) and cell_est (DEVICE double [n_traj][n_w][n_cells],
 * E_c, to pass to rad_sampler_combine as cell_pred).  No fallback check.  eps >= 0,
 * cap >= 1; n_cells <= 64.  This rule is not in the paper (it extends the angular
 * grid of Sec. IV).
 */
rad_status rad_sampler_select_error(const rad_grid *fine, int n_traj, const float *pred, float mu, float sigma,
                                    const double *coarse, int cx, int cy, float eps, int cap, uint8_t *mask,
                                    double *cell_est, void *stream);

/*
 * dIdw (DEVICE double [n_traj][n_w]) = sum over cells of the exact cell integral
 * (cells, DEVICE [n_traj][n_w][n_cells], from rad_cells) where mask is set; else
 * cell_pred (the predicted cell masses of rad_sampler_select or the estimates E_c of
 * rad_sampler_select_error) if it is not NULL, else the coarse centre value times
 * the cell's area.  Fallback: where fallback[t][w] (DEVICE uint8 [n_traj][n_w]) is
 * set, dIdw[t][w] = full[t][w] (DEVICE double [n_traj][n_w]), the full-grid angle
 * integral (rad_batch on the fine grid, then rad_angle_integrate), copied bit for
 * bit.  fallback and full are both NULL or both given (else RAD_EINVAL).
 */
rad_status rad_sampler_combine(const rad_grid *fine, int n_traj, int cx, int cy, const double *cells,
                               const uint8_t *mask, const double *coarse, const double *cell_pred,
                               const uint8_t *fallback, const double *full, double *dIdw, void *stream);

/*
 * Refinement without a network, the comparison the sampler has to beat: a stand-in
 * prediction that ranks cells by their exact centre values.  pred (DEVICE float
 * [n_traj][n_w][n_y][n_x]) = log(coarse[t][w][cell of the direction]) computed in FP64
 * (-inf where the value is not positive); coarse: DEVICE double [n_traj][n_w][n_cells].
 * With mu = 0, sigma = 1, rad_sampler_select then ranks cells by centre value x area.
 * Errors: RAD_EINVAL for sizes or buffers out of range, cells that do not tile the grid.
 */
rad_status rad_sampler_coarse_pred(const rad_grid *fine, int n_traj, const double *coarse, int cx, int cy,
                                   float *pred, void *stream);

/*
 * Training data of the network (spectra the method itself computes).
 *
 * rad_sampler_targets: the angular shape of each of n_maps spectra S (DEVICE double
 * [n_maps][n_dirs], e.g. one photon energy of a cube on the fine grid):
 * y[m][d] = log(max(S, 0) / max_d max(S, 0) + floor_rel) (DEVICE float, same shape),
 * computed in FP64.  floor_rel > 0 keeps the logarithm finite where S is 0.
 *
 * rad_sampler_moments: mean and standard deviation (population) of n floats y
 * (DEVICE), in FP64 by two fixed-order passes, into moments (DEVICE double [2]); ws:
 * DEVICE workspace of rad_sampler_moments_workspace_bytes().
 *
 * rad_sampler_minibatch: `batch` training points drawn uniformly with replacement: a
 * map (trajectory t in [0, n), energy slot e in [0, nwt)) and a direction p in
 * [0, npix), by splitmix64 of (seed, step, point) -- batch `step` is reproducible.
 * Writes traj[b] = t (DEVICE int [batch]), the point inputs x[b] = point_x[W[t][e] npix
 * + p] (DEVICE float [batch][3]; W: DEVICE int [n][nwt] energy indices into the point
 * table point_x, DEVICE float [n_points][3], n_points a multiple of npix; an index
 * outside the table is clamped into it) and target[b] = (Y[t][e][p] - mean) / std
 * (Y: DEVICE float [n][nwt][npix]; moments from rad_sampler_moments).
 *
 * Errors: RAD_EINVAL for sizes out of range or buffers that are not device memory of
 * the stated size; RAD_ENOMEM for a small workspace.  No host synchronisation.
 */
rad_status rad_sampler_targets(const double *S, int64_t n_maps, int n_dirs, float floor_rel, float *y, void *stream);
size_t rad_sampler_moments_workspace_bytes(void);
rad_status rad_sampler_moments(const float *y, int64_t n, double *moments, void *ws, size_t ws_bytes, void *stream);
rad_status rad_sampler_minibatch(const float *Y, const int *W, int64_t n, int nwt, int npix, const float *point_x,
                                 int64_t n_points, const double *moments, int batch, uint64_t seed, uint64_t step,
                                 int *traj, float *x, float *target, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAD_SAMPLER_H */

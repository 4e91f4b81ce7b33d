// Internal data structures of the learned-sampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radsmp {

constexpr int kHistBins = 32;
constexpr int kFeatures = 6 + kHistBins;   // log gamma, histogram, log omega_osc, 4 direction moments
constexpr int kMaxTurning = 4096;           // turning points kept per trajectory
constexpr int kWBlock = 64;                 // photon energies rad_cells evaluates together
constexpr int kMomentParts = 1024;          // first-pass blocks of the target moments
constexpr double kPi = 3.14159265358979323846;

struct FeatSeg {
    const double *t, *x, *vx, *vy;
    int64_t n;
    double gamma;
};

struct FeatLaunch {
    const FeatSeg *segs;
    double plane_spacing;
    float *feat;   // [n_segs][kFeatures]
};

struct SelectLaunch {
    const float *pred;     // [n_traj][n_w][n_y][n_x] normalised log intensity
    float mu, sigma;       // log intensity = mu + sigma * pred
    const double *coarse;  // [n_traj][n_w][n_cells] spectrum at the cell centres
    const double *wx, *wy; // direction cell widths of the fine grid
    int n_traj, n_w, n_x, n_y, cx, cy, n_cells;
    float coverage, tau;   // coverage: eps in the error-driven selection
    int cap;
    uint8_t *mask;         // [n_traj][n_w][n_cells]
    uint8_t *fallback;     // [n_traj][n_w]
    double *cell_pred;     // [n_traj][n_w][n_cells] predicted cell masses (or estimates E_c), or null
};

struct CombineLaunch {
    const double *cells, *coarse, *wx, *wy;
    const double *cell_pred;   // null: unselected cells count as centre value x area
    const uint8_t *mask;
    const uint8_t *fallback;   // [n_traj][n_w] or null: where set, the full-grid value
    const double *full;        // [n_traj][n_w] full-grid dI/dhw (with fallback)
    int n_traj, n_w, n_x, cx, cy, n_cells;
    double *out;           // [n_traj][n_w]
};

// Training data of the network: per map the angular shape log(S / max S + floor) of a
// spectrum, the moments of all targets, and minibatches drawn from them.
struct BatchLaunch {
    const float *Y;        // [n][nwt][npix] targets
    const int *W;          // [n][nwt] photon-energy index (into the point table) of each map
    const float *point_x;  // [n_w * npix][3] network point inputs
    int64_t n_points;      // n_w * npix
    int64_t n;
    int nwt, npix;
    const double *moments; // [2]: mean and standard deviation of Y
    int batch;
    uint64_t seed, step;
    int *traj;             // [batch]
    float *x;              // [batch][3]
    float *target;         // [batch] standardised
};

hipError_t launch_features(const FeatLaunch &F, int n_segs, hipStream_t st);
hipError_t launch_targets(const double *S, int64_t n_maps, int n_dirs, float floor_rel, float *y, hipStream_t st);
hipError_t launch_moments(const float *y, int64_t n, double *part, int parts, double *out, hipStream_t st);
hipError_t launch_minibatch(const BatchLaunch &L, hipStream_t st);
hipError_t launch_select(const SelectLaunch &L, hipStream_t st);
hipError_t launch_select_error(const SelectLaunch &L, hipStream_t st);
hipError_t launch_widen(uint8_t *mask, int n_traj, int n_w, int n_cells, hipStream_t st);
hipError_t launch_coarse_pred(const double *coarse, int64_t n_maps, int n_x, int n_y, int cx, int cy, float *pred,
                              hipStream_t st);
hipError_t launch_combine(const CombineLaunch &L, hipStream_t st);

}  // namespace radsmp

// Internal data structures of the learned-sampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radsmp {

constexpr int kHistBins = 32;
constexpr int kFeatures = 6 + kHistBins;   // log gamma, histogram, log omega_osc, 4 direction moments
constexpr int kMaxTurning = 4096;           // turning points kept per trajectory
constexpr int kWBlock = 64;                 // photon energies rad_cells evaluates together
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
    int n_traj, n_w, n_x, cx, cy, n_cells;
    double *out;           // [n_traj][n_w]
};

hipError_t launch_features(const FeatLaunch &F, int n_segs, hipStream_t st);
hipError_t launch_select(const SelectLaunch &L, hipStream_t st);
hipError_t launch_select_error(const SelectLaunch &L, hipStream_t st);
hipError_t launch_widen(uint8_t *mask, int n_traj, int n_w, int n_cells, hipStream_t st);
hipError_t launch_combine(const CombineLaunch &L, hipStream_t st);

}  // namespace radsmp

// Internal data structures shared by the host library and the kernels of librad.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rad {

// CODATA 2018
constexpr double kHbarC_eVm = 1.973269804e-7;   // hbar c [eV m]
constexpr double kAlpha = 7.2973525693e-3;      // fine-structure constant
constexpr double kPi = 3.14159265358979323846;

// Kernel tile shape: each lane owns one photon energy and a TX x TY block of
// directions; a wave is 64 photon energies; a block is 4 waves.
constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLogSlots = 7;
constexpr int kSlots = 1 << kLogSlots;  // time-steps x direction-tiles staged in LDS per pass

// Amplitude-kernel variants: direction tile TX x TY and minimum resident blocks per CU.
enum Variant { kVar44x2 = 0, kVar43x2 = 1, kVar44x1 = 2, kVar42x2 = 3, kVar46x2 = 4, kNumVariants = 5 };
constexpr int kVarTX[kNumVariants] = {4, 4, 4, 4, 4};
constexpr int kVarTY[kNumVariants] = {4, 3, 4, 2, 6};
// whether a variant serves the integral set with J: the 4x6 tile's 24 directions fill the
// VGPRs with the A_x, A_y accumulators alone, so it serves only sets without J
constexpr bool kVarJ[kNumVariants] = {true, true, true, true, false};

enum Column { C_T = 0, C_X, C_Y, C_DZ, C_VX, C_VY, C_DVZ, C_AX, C_AY, C_AZ, C_NCOL };

// One segment as the kernels see it: a trajectory piece and the (hw, direction)
// grid it is integrated on (all segments of a rad_batch call share one grid; the
// cell refinement gives each (trajectory, cell) its own view of the fine grid).
struct SegDesc {
    const double *col[C_NCOL];
    const double *w;       // nullable -> trapezoid
    int64_t n;
    double c0;             // 1 / (2 gamma^2)
    double gamma;
    double energy;         // eV
    int64_t part_off;      // offset (in double2) of this segment's partial amplitudes in the set
    int32_t n_chunks;
    int32_t chunk_len;
    int64_t block_begin;   // first block of this segment in the amplitude launch
    const double *hw;      // [n_w] eV
    const double *k;       // [n_w] 1/m
    const double *thx;     // [n_x]
    const double *thy;     // [n_y]
    int32_t n_w, n_x, n_y;
    int32_t n_tx, n_ty;    // direction tiles along x, y
    int32_t n_groups;      // ceil(n_tx * n_ty / nt)
    int32_t n_wblocks;     // ceil(n_w / (64 wg))
    int32_t pad_;
    double dth;            // common spacing of uniform thx and thy grids, or 0
};

// One amplitude launch: one "set" (classical kappa = k, or quantum kappa = k*).
struct AmpLaunch {
    const SegDesc *segs;   // in launch (longest-first) order
    const int4 *items;     // explicit work items (segment, chunk, group, w block) or null
    int n_segs;
    int64_t n_blocks;      // work items
    int wg;                // waves per block spread over photon energies (1, 2, 4)
    int nt;                // direction tiles per block (4 / wg)
    int quantum;           // 0: kappa = k; 1: kappa = k E/(E - hw)
    int comps;             // 2 (A_x, A_y) or 3 (A_x, A_y, J)
    double2 *part;         // partial amplitudes [seg][chunk][comp][n][w]
    int64_t part_len;      // elements of `part` (index checks of the RAD_DEBUG build)
    unsigned *counter;     // ticket of the persistent form (zeroed before the launch)
    int rec;               // FP64: phase factors by recurrence (every segment's dth != 0)
    // cell refinement with a device mask: the items were compacted on the device and
    // only the first *n_live of them run (the blocks past it return at once); null
    // otherwise
    const int *n_live;
};

// Device-side compaction of the cell refinement's items: items (in launch order) whose
// photon-energy block has a mask bit set, for pseudo-segment p = (p / n_cells, p % n_cells)
// = (segment, cell), keep their order in `live`, their number in *n_live.  wg = 0: the
// grouped form, whose dense items come in rows of n_wb (one per (pseudo-segment, time
// chunk), blocks 0 .. n_wb - 1) and are first regrouped row by row into `grouped`.
struct CellCompact {
    const int4 *items;
    int64_t n_items;
    const uint8_t *mask;     // [n_segs][n_w][n_cells]
    int n_cells, n_w, wg;
    int n_wb;                // 64-energy blocks per row (grouped form)
    int4 *grouped;           // [n_items] (grouped form)
    int *flags;              // [n_items]
    int4 *live;              // [n_items]
    int *n_live;
};

// Finalize: per output, the segments that feed it, in segment order.
struct FinLaunch {
    const int *out_seg_begin;   // [n_out + 1]
    const int *out_seg_list;    // segment ids (index into cls/qsegs) in order
    const SegDesc *cls;         // classical-set descriptors by segment id (or null)
    const SegDesc *qs;          // quantum-set descriptors by segment id (or null)
    const double2 *part_c;      // classical partials
    const double2 *part_q;      // quantum partials
    int64_t part_c_len, part_q_len;   // their elements (index checks of the RAD_DEBUG build)
    int comps_q;                // 2 or 3
    const double *hw, *thx, *thy;
    int n_w, n_x, n_y;
    int n_out;
    int kinds;
    int n_kinds;
    int one_chunk;              // every segment is a single time chunk
    double *out;                // [n_out][n_kinds][n_w][n_y][n_x]
};

// Cell integrals of the refinement: for each (segment, photon energy, cell) with
// its mask set, the spectrum summed over the cell's directions times their
// solid-angle weights.
struct CellsFin {
    const SegDesc *segs;        // active (segment, cell) pseudo-segments
    const int *psof;            // [n_segs][n_cells] -> pseudo-segment or -1
    const uint8_t *mask;        // [n_segs][n_w][n_cells]
    const double2 *part;
    int64_t part_len;           // elements of `part` (index checks of the RAD_DEBUG build)
    int comps, kind;
    const double *wx, *wy;      // direction cell widths of the fine grid
    const double *hw;
    int n_segs, n_w, n_x, ncx, n_cells, cx, cy;
    double *out;                // [n_segs][n_w][n_cells]
};

// Read-only view of a grid handle's device arrays (for the sampler's host code).
struct GridView {
    const double *hw, *k, *thx, *thy, *wx, *wy;
    int n_w, n_x, n_y, device;
};

}  // namespace rad

struct rad_grid;
bool rad_grid_view(const rad_grid *g, rad::GridView *v);
namespace rad_err {
void set(const char *msg);
}

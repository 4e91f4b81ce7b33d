// Kernels of the learned angular sampler (gfx950): trajectory features, cell
// selection from the network's prediction, and the refined angle integral.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sampler_internal.h"

namespace radsmp {

// ---------------------------------------------------------------- features
// One block per trajectory.  Turning points are the sign changes of v_x
// (between samples k and k+1, position x[k+1]); a half oscillation runs between
// consecutive turning points and its amplitude is half the distance between
// them.  Features: log(gamma / 1e4); a kHistBins-bin histogram of the amplitudes
// over [0, d/2] (amplitudes >= d/2, over-barrier motion, fall in the last bin),
// normalised to sum 1 (with fewer than two turning points the only entry is half
// the total x excursion); log(omega_osc / 1e5 m^-1) with
// omega_osc = pi (number of sign changes) / (t_end - t_0); and the direction of
// motion in units of 1/gamma: gamma mean(v_x), gamma mean(v_y), gamma std(v_x),
// gamma std(v_y) over the samples (the radiation cone follows the direction).
__global__ __launch_bounds__(256) void features_kernel(FeatLaunch F)
{
    __shared__ int s_cnt[256];
    __shared__ float s_tp[kMaxTurning];
    __shared__ double s_min[256], s_max[256];
    __shared__ double s_mom[4][256];
    const FeatSeg &S = F.segs[blockIdx.x];
    const int64_t n = S.n;
    const int tid = threadIdx.x;
    const int64_t per = (n - 1 + 255) / 256;             // pairs (k, k+1), k in [0, n-1)
    const int64_t k0 = tid * per, k1 = min(n - 1, k0 + per);
    int cnt = 0;
    double xmn = 1e300, xmx = -1e300;
    for (int64_t k = k0; k < k1; ++k) {
        const bool a = S.vx[k] >= 0.0, b = S.vx[k + 1] >= 0.0;
        cnt += (a != b);
    }
    double m[2] = {0.0, 0.0};   // sums of vx, vy
    for (int64_t k = tid; k < n; k += 256) {
        xmn = fmin(xmn, S.x[k]);
        xmx = fmax(xmx, S.x[k]);
        m[0] += S.vx[k];
        m[1] += S.vy[k];
    }
    s_cnt[tid] = cnt;
    s_min[tid] = xmn;
    s_max[tid] = xmx;
    for (int j = 0; j < 2; ++j) s_mom[j][tid] = m[j];
    __syncthreads();
    // means first, then the spreads about them (two passes: no cancellation when the
    // spread is small beside the mean)
    if (tid < 2) {
        double t = 0.0;
        for (int i = 0; i < 256; ++i) t += s_mom[tid][i];
        s_mom[tid + 2][0] = t / (double)n;
    }
    __syncthreads();
    {
        const double mx = s_mom[2][0], my = s_mom[3][0];
        double q[2] = {0.0, 0.0};
        for (int64_t k = tid; k < n; k += 256) {
            const double dx = S.vx[k] - mx, dy = S.vy[k] - my;
            q[0] += dx * dx;
            q[1] += dy * dy;
        }
        __syncthreads();   // the means are read before the slots are reused
        s_mom[0][tid] = q[0];
        s_mom[1][tid] = q[1];
        if (tid == 0) {
            s_mom[2][1] = mx;
            s_mom[3][1] = my;
        }
    }
    __syncthreads();
    // exclusive prefix of the counts (in chunk order = time order), extrema, moments
    if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < 256; ++i) {
            const int c = s_cnt[i];
            s_cnt[i] = acc;
            acc += c;
        }
        double a = 1e300, b = -1e300;
        for (int i = 0; i < 256; ++i) {
            a = fmin(a, s_min[i]);
            b = fmax(b, s_max[i]);
        }
        s_min[0] = a;
        s_max[0] = b;
        for (int j = 0; j < 2; ++j) {
            double t = 0.0;
            for (int i = 0; i < 256; ++i) t += s_mom[j][i];
            s_mom[j][0] = t;   // sums of squared deviations
        }
    }
    __syncthreads();
    int o = s_cnt[tid];
    for (int64_t k = k0; k < k1; ++k) {
        const bool a = S.vx[k] >= 0.0, b = S.vx[k + 1] >= 0.0;
        if (a != b) {
            if (o < kMaxTurning) s_tp[o] = (float)S.x[k + 1];
            ++o;
        }
    }
    __syncthreads();
    // the last thread's end offset is the total number of sign changes
    __shared__ int s_total;
    if (tid == 255) s_total = o;
    __syncthreads();
    if (tid != 0) return;
    const int total = s_total;
    const int stored = min(total, kMaxTurning);
    float hist[kHistBins];
    for (int i = 0; i < kHistBins; ++i) hist[i] = 0.0f;
    const double half = 0.5 * F.plane_spacing;
    int runs = 0;
    auto put = [&](double amp) {
        int bin = (int)(amp / half * kHistBins);
        bin = bin < 0 ? 0 : (bin >= kHistBins ? kHistBins - 1 : bin);
        hist[bin] += 1.0f;
        ++runs;
    };
    for (int i = 0; i + 1 < stored; ++i) put(0.5 * fabs((double)s_tp[i + 1] - (double)s_tp[i]));
    if (runs == 0) put(0.5 * (s_max[0] - s_min[0]));
    float *f = F.feat + (int64_t)blockIdx.x * kFeatures;
    f[0] = (float)log(S.gamma / 1e4);
    for (int i = 0; i < kHistBins; ++i) f[1 + i] = hist[i] / (float)runs;
    const double span = S.t[n - 1] - S.t[0];
    const double w_osc = span > 0.0 ? kPi * (double)total / span : 0.0;
    f[1 + kHistBins] = (float)log(fmax(w_osc, 1.0) / 1e5);
    const double mx = s_mom[2][1], my = s_mom[3][1];
    const double vxx = s_mom[0][0] / (double)n, vyy = s_mom[1][0] / (double)n;
    f[2 + kHistBins] = (float)(S.gamma * mx);
    f[3 + kHistBins] = (float)(S.gamma * my);
    f[4 + kHistBins] = (float)(S.gamma * sqrt(vxx));
    f[5 + kHistBins] = (float)(S.gamma * sqrt(vyy));
}

// ---------------------------------------------------------------- selection
// The network's view of cell c of item (trajectory, photon energy), from the
// predicted intensities exp(mu + sigma * pred) of its fine directions: the mass
// pm (sum of value x dthx dthy), the centre value pc (mean value of the fine
// directions nearest the centre: the central 2 x 2 of an even cell, the middle
// point of an odd one) and the cell area.
__device__ __forceinline__ void cell_prediction(const SelectLaunch &L, int64_t item, int c, double &pm,
                                                double &pc, double &area)
{
    const int ncx = L.n_x / L.cx;
    const int ci = c % ncx, cj = c / ncx;
    const float *pred = L.pred + item * (int64_t)L.n_x * L.n_y;
    const int xa = (L.cx - 1) / 2, xb = L.cx / 2, ya = (L.cy - 1) / 2, yb = L.cy / 2;
    int npc = 0;
    pm = pc = area = 0.0;
    for (int jy = 0; jy < L.cy; ++jy)
        for (int jx = 0; jx < L.cx; ++jx) {
            const int gx = ci * L.cx + jx, gy = cj * L.cy + jy;
            const double v = exp((double)L.mu + (double)L.sigma * (double)pred[(int64_t)gy * L.n_x + gx]);
            const double dA = L.wx[gx] * L.wy[gy];
            pm += v * dA;
            area += dA;
            if ((jx == xa || jx == xb) && (jy == ya || jy == yb)) {
                pc += v;
                ++npc;
            }
        }
    pc /= (double)npc;
}

// Wave-wide sums over the cells of one item.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per (trajectory, photon energy); lane c < n_cells owns cell c.  The
// network predicts the angular shape up to a scale; the scale lambda comes from
// the exact spectrum at the cell centres C_c: lambda = sum_c C_c A_c / sum_c P_c A_c
// (P_c the predicted centre value, A_c the cell area).  Check: the energy falls
// back to the full grid (every cell selected) when sum_c |lambda P_c - C_c| A_c
// exceeds tau sum_c C_c A_c (or either sum is 0).  Otherwise cells are taken in
// decreasing predicted mass (lambda times the predicted cell mass; ties by index)
// while the mass before them is below coverage times the total, at most `cap`.
__global__ __launch_bounds__(256) void select_kernel(SelectLaunch L)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;   // traj * n_w + w
    if (item >= (int64_t)L.n_traj * L.n_w) return;
    const int c = lane;
    const bool live = c < L.n_cells;
    double pm = 0.0, pc = 0.0, cc = 0.0, area = 0.0;
    if (live) {
        cell_prediction(L, item, c, pm, pc, area);
        cc = L.coarse[item * L.n_cells + c];
    }
    const double P = wave_sum(pc * area), C = wave_sum(cc * area);
    const double lambda = P > 0.0 ? C / P : 0.0;
    pm *= lambda;
    const double D = wave_sum(fabs(lambda * pc - cc) * area), Mp = wave_sum(pm);
    if (live && L.cell_pred) L.cell_pred[item * L.n_cells + c] = pm;
    const bool fb = !(C > 0.0) || !(P > 0.0) || D > (double)L.tau * C;
    // rank and predicted mass ahead of this cell
    int rank = 0;
    double ahead = 0.0;
    for (int j = 0; j < 64; ++j) {
        const double mj = __shfl(pm, j, 64);
        const bool lj = j < L.n_cells;
        const bool before = lj && (mj > pm || (mj == pm && j < c));
        if (before) {
            ++rank;
            ahead += mj;
        }
    }
    const bool sel = live && (fb || (rank < L.cap && ahead < (double)L.coverage * Mp));
    if (live) L.mask[item * L.n_cells + c] = sel ? 1 : 0;
    if (lane == 0) L.fallback[item] = fb ? 1 : 0;
}

// Error-driven selection, same layout: the predicted sub-cell shape corrects the
// exact centre value, E_c = C_c pm_c / pc_c (C_c A_c where pc_c is 0; the ratio
// does not depend on the prediction's scale), and e_c = |E_c - C_c A_c| estimates
// the error of leaving the cell at its midpoint value.  Cells are taken in
// decreasing e_c (ties by index) while the estimated error of the cells not yet
// taken, sum of e_j over this cell and those after it, exceeds eps sum_c E_c, at
// most `cap`.  E_c goes to cell_pred for the combination.
__global__ __launch_bounds__(256) void select_error_kernel(SelectLaunch L)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= (int64_t)L.n_traj * L.n_w) return;
    const int c = lane;
    const bool live = c < L.n_cells;
    double est = 0.0, e = 0.0;
    if (live) {
        double pm, pc, area;
        cell_prediction(L, item, c, pm, pc, area);
        const double cc = L.coarse[item * L.n_cells + c];
        const double mid = cc * area;
        est = pc > 0.0 ? cc * pm / pc : mid;
        e = fabs(est - mid);
        L.cell_pred[item * L.n_cells + c] = est;
    }
    const double budget = (double)L.coverage * wave_sum(est);
    int rank = 0;
    double left = 0.0;
    for (int j = 0; j < 64; ++j) {
        const double ej = __shfl(e, j, 64);
        const bool lj = j < L.n_cells;
        const bool before = lj && (ej > e || (ej == e && j < c));
        if (before) ++rank;
        else if (lj) left += ej;
    }
    if (live) L.mask[item * L.n_cells + c] = (rank < L.cap && left > budget) ? 1 : 0;
}

// Widen the selection to whole blocks of kWBlock photon energies: rad_cells
// evaluates a cell for a whole block at the cost of one energy, so every energy of
// a block whose cell is selected anywhere in the block takes the exact value.
// One thread per (trajectory, energy block, cell); in place.
__global__ __launch_bounds__(256) void widen_kernel(uint8_t *mask, int n_traj, int n_w, int n_cells)
{
    const int n_wb = (n_w + kWBlock - 1) / kWBlock;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_traj * n_wb * n_cells) return;
    const int c = (int)(i % n_cells);
    const int b = (int)((i / n_cells) % n_wb);
    const int64_t s = i / ((int64_t)n_cells * n_wb);
    const int w0 = b * kWBlock, w1 = min(n_w, w0 + kWBlock);
    uint8_t *m = mask + (s * n_w) * n_cells + c;
    uint8_t any = 0;
    for (int w = w0; w < w1; ++w) any |= m[(int64_t)w * n_cells];
    if (any)
        for (int w = w0; w < w1; ++w) m[(int64_t)w * n_cells] = 1;
}

// ---------------------------------------------------------------- combine
// dI/dhw[traj][w] = sum_c (mask ? exact cell integral : estimate), the estimate
// being the predicted cell mass when cell_pred is given, else the coarse centre
// value times the cell's area; an energy that fell back takes the full-grid value.
__global__ __launch_bounds__(256) void combine_kernel(CombineLaunch L)
{
    const int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= (int64_t)L.n_traj * L.n_w) return;
    if (L.fallback && L.fallback[item]) {
        L.out[item] = L.full[item];
        return;
    }
    const int ncx = L.n_x / L.cx;
    double acc = 0.0;
    for (int c = 0; c < L.n_cells; ++c) {
        const int64_t i = item * L.n_cells + c;
        if (L.mask[i]) {
            acc += L.cells[i];
        } else if (L.cell_pred) {
            acc += L.cell_pred[i];
        } else {
            const int ci = c % ncx, cj = c / ncx;
            double ax = 0.0, ay = 0.0;
            for (int j = 0; j < L.cx; ++j) ax += L.wx[ci * L.cx + j];
            for (int j = 0; j < L.cy; ++j) ay += L.wy[cj * L.cy + j];
            acc += L.coarse[i] * ax * ay;
        }
    }
    L.out[item] = acc;
}

// ---------------------------------------------------------------- training data
// y[m][d] = log(S+ / max_d S+ + floor) with S+ = max(S, 0): one block per map, the maximum
// over its directions by a fixed LDS tree, then the transform (FP64, stored as FP32).
__global__ __launch_bounds__(256) void targets_kernel(const double *__restrict__ S, int n_dirs, float floor_rel,
                                                      float *__restrict__ y)
{
    __shared__ double red[256];
    const double *s = S + (int64_t)blockIdx.x * n_dirs;
    double mx = 0.0;
    for (int d = threadIdx.x; d < n_dirs; d += 256) mx = fmax(mx, s[d]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const double peak = fmax(red[0], 1e-300);
    float *out = y + (int64_t)blockIdx.x * n_dirs;
    for (int d = threadIdx.x; d < n_dirs; d += 256) out[d] = (float)log(fmax(s[d], 0.0) / peak + (double)floor_rel);
}

// Mean and standard deviation of n values in FP64, two passes (mean, then squared
// deviations), each a fixed-order sum: `parts` blocks of 256 strided partial sums, then
// one block adds the parts.  mode 0: sums of y; mode 1: sums of (y - mean)^2.
__global__ __launch_bounds__(256) void moments_kernel(const float *__restrict__ y, int64_t n, int mode,
                                                      const double *__restrict__ mean, double *__restrict__ part)
{
    __shared__ double red[256];
    const double m = mode ? mean[0] : 0.0;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = (double)y[i] - m;
        acc += mode ? v * v : v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void moments_finish(const double *__restrict__ part, int parts, int64_t n, int mode,
                                                      double *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < parts; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[mode] = mode ? sqrt(red[0] / (double)n) : red[0] / (double)n;
}

// splitmix64 (Steele, Lea and Flood, 2014) of a counter: draw i of step `step`
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Minibatch point b: a map (trajectory t, its energy slot e) and a direction p drawn
// uniformly, the point inputs of (energy W[t][e], direction p) and the standardised
// target (Y - mean) / std.  Draws are counter-based, so batch `step` is reproducible.
__global__ __launch_bounds__(256) void minibatch_kernel(BatchLaunch L)
{
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= L.batch) return;
    const uint64_t base = mix64(L.seed ^ mix64(L.step)) + 3ull * (uint64_t)b;
    const uint64_t r0 = mix64(base), r1 = mix64(base + 1), r2 = mix64(base + 2);
    const int64_t t = (int64_t)((r0 >> 11) % (uint64_t)L.n);
    const int e = (int)((r1 >> 11) % (uint64_t)L.nwt);
    const int p = (int)((r2 >> 11) % (uint64_t)L.npix);
    // an energy index outside the table is clamped into it (the host cannot see W)
    const int64_t n_energy = L.n_points / L.npix;
    int64_t we = L.W[t * L.nwt + e];
    we = we < 0 ? 0 : (we >= n_energy ? n_energy - 1 : we);
    const int64_t pt = we * L.npix + p;
#pragma unroll
    for (int j = 0; j < 3; ++j) L.x[(int64_t)b * 3 + j] = L.point_x[pt * 3 + j];
    L.traj[b] = (int)t;
    const float v = L.Y[(t * L.nwt + e) * (int64_t)L.npix + p];
    L.target[b] = (float)(((double)v - L.moments[0]) / L.moments[1]);
}

// pred[m][y][x] = log(coarse[m][cell of (y, x)]) in FP64, stored as FP32 (-inf where the
// value is not positive): one thread per fine direction.
__global__ __launch_bounds__(256) void coarse_pred_kernel(const double *__restrict__ coarse, int64_t n, int n_x,
                                                          int n_y, int cx, int cy, float *__restrict__ pred)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t dirs = (int64_t)n_x * n_y;
    const int64_t m = i / dirs;
    const int d = (int)(i % dirs), y = d / n_x, x = d % n_x;
    const int ncx = n_x / cx, n_cells = ncx * (n_y / cy);
    const double v = coarse[m * n_cells + (y / cy) * ncx + x / cx];
    pred[i] = v > 0.0 ? (float)log(v) : -__builtin_huge_valf();
}

hipError_t launch_coarse_pred(const double *coarse, int64_t n_maps, int n_x, int n_y, int cx, int cy, float *pred,
                              hipStream_t st)
{
    const int64_t n = n_maps * n_x * n_y;
    hipLaunchKernelGGL(coarse_pred_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, coarse, n, n_x, n_y,
                       cx, cy, pred);
    return hipGetLastError();
}

hipError_t launch_targets(const double *S, int64_t n_maps, int n_dirs, float floor_rel, float *y, hipStream_t st)
{
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)n_maps), dim3(256), 0, st, S, n_dirs, floor_rel, y);
    return hipGetLastError();
}

hipError_t launch_moments(const float *y, int64_t n, double *part, int parts, double *out, hipStream_t st)
{
    for (int mode = 0; mode < 2; ++mode) {
        hipLaunchKernelGGL(moments_kernel, dim3((unsigned)parts), dim3(256), 0, st, y, n, mode, out, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(moments_finish, dim3(1), dim3(256), 0, st, part, parts, n, mode, out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_minibatch(const BatchLaunch &L, hipStream_t st)
{
    hipLaunchKernelGGL(minibatch_kernel, dim3((unsigned)((L.batch + 255) / 256)), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_features(const FeatLaunch &F, int n_segs, hipStream_t st)
{
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)n_segs), dim3(256), 0, st, F);
    return hipGetLastError();
}

hipError_t launch_select(const SelectLaunch &L, hipStream_t st)
{
    const int64_t items = (int64_t)L.n_traj * L.n_w;
    hipLaunchKernelGGL(select_kernel, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_select_error(const SelectLaunch &L, hipStream_t st)
{
    const int64_t items = (int64_t)L.n_traj * L.n_w;
    hipLaunchKernelGGL(select_error_kernel, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_widen(uint8_t *mask, int n_traj, int n_w, int n_cells, hipStream_t st)
{
    const int64_t items = (int64_t)n_traj * ((n_w + kWBlock - 1) / kWBlock) * n_cells;
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, mask, n_traj, n_w,
                       n_cells);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineLaunch &L, hipStream_t st)
{
    const int64_t items = (int64_t)L.n_traj * L.n_w;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, L);
    return hipGetLastError();
}

}  // namespace radsmp

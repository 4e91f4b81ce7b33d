// librad: host side of the sampler C ABI (include/rad_sampler.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "rad_internal.h"
#include "rad_sampler.h"
#include "sampler_internal.h"

using namespace radsmp;

namespace rad {
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st);
}

static_assert(sizeof(FeatSeg) == 48, "rad_features documents 48 workspace bytes per segment");

namespace {

rad_status sfail(rad_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    rad_err::set(buf);
    return st;
}

rad_status srange(const void *p, size_t bytes, const char *name)
{
    if (!p) return sfail(RAD_EINVAL, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(RAD_EINVAL, "%s (%p) is not a device allocation", name, p);
    }
    if ((const char *)p + bytes > (const char *)base + size)
        return sfail(RAD_EINVAL, "%s: %zu bytes exceed its device allocation", name, bytes);
    return RAD_OK;
}

rad_status view_of(const rad_grid *g, rad::GridView &v)
{
    if (!rad_grid_view(g, &v)) return sfail(RAD_EINVAL, "grid is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return sfail(RAD_EDEVICE, "no HIP device");
    if (dev != v.device) return sfail(RAD_EINVAL, "grid lives on device %d, current device is %d", v.device, dev);
    return RAD_OK;
}

rad_status cells_shape(const rad::GridView &v, int cx, int cy, int &n_cells)
{
    if (cx <= 0 || cy <= 0 || v.n_x % cx || v.n_y % cy)
        return sfail(RAD_EINVAL, "cells of %d x %d do not tile the %d x %d grid", cx, cy, v.n_x, v.n_y);
    n_cells = (v.n_x / cx) * (v.n_y / cy);
    if (n_cells > 64) return sfail(RAD_EUNSUPPORTED, "%d cells (at most 64)", n_cells);
    return RAD_OK;
}

}  // namespace

extern "C" {

rad_status rad_features(const rad_segment *segs, int n_segs, double plane_spacing_m, float *feat, void *ws,
                        size_t ws_bytes, void *stream)
{
    if (!segs || n_segs <= 0) return sfail(RAD_EINVAL, "no segments");
    if (!(plane_spacing_m > 0.0) || !std::isfinite(plane_spacing_m))
        return sfail(RAD_EINVAL, "plane_spacing_m must be finite and > 0");
    const size_t need = sizeof(FeatSeg) * (size_t)n_segs;
    if (ws_bytes < need) return sfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    rad_status rs = srange(ws, need, "workspace");
    if (rs != RAD_OK) return rs;
    if ((rs = srange(feat, (size_t)n_segs * kFeatures * sizeof(float), "feat")) != RAD_OK) return rs;
    std::vector<FeatSeg> h(n_segs);
    for (int s = 0; s < n_segs; ++s) {
        const rad_segment &sg = segs[s];
        if (sg.n < 2) return sfail(RAD_EINVAL, "segment %d: n < 2", s);
        if (!(sg.gamma > 0.0)) return sfail(RAD_EINVAL, "segment %d: gamma must be > 0", s);
        const size_t b = (size_t)sg.n * sizeof(double);
        if ((rs = srange(sg.t, b, "t")) != RAD_OK || (rs = srange(sg.x, b, "x")) != RAD_OK ||
            (rs = srange(sg.vx, b, "vx")) != RAD_OK || (rs = srange(sg.vy, b, "vy")) != RAD_OK)
            return rs;
        h[s] = FeatSeg{sg.t, sg.x, sg.vx, sg.vy, sg.n, sg.gamma};
    }
    hipStream_t st = (hipStream_t)stream;
    // the descriptors travel as kernel arguments: no host buffer has to outlive the call,
    // so nothing waits for the stream
    hipError_t e = rad::launch_upload(ws, h.data(), need, st);
    FeatLaunch F{(const FeatSeg *)ws, plane_spacing_m, feat};
    if (e == hipSuccess) e = launch_features(F, n_segs, st);
    if (e != hipSuccess) return sfail(RAD_EDEVICE, "features: %s", hipGetErrorString(e));
    return RAD_OK;
}

rad_status rad_sampler_select(const rad_grid *fine, int n_traj, const float *pred, float mu, float sigma,
                              const double *coarse, int cx, int cy, float coverage, int cap, float tau,
                              uint8_t *mask, uint8_t *fallback, double *cell_pred, void *stream)
{
    rad::GridView v;
    rad_status rs = view_of(fine, v);
    if (rs != RAD_OK) return rs;
    int n_cells = 0;
    if ((rs = cells_shape(v, cx, cy, n_cells)) != RAD_OK) return rs;
    if (n_traj <= 0) return sfail(RAD_EINVAL, "n_traj must be > 0");
    if (!(coverage > 0.0f && coverage <= 1.0f) || cap < 1 || !(tau >= 0.0f) || !std::isfinite(mu) ||
        !std::isfinite(sigma))
        return sfail(RAD_EINVAL, "invalid coverage, cap, tau, mu or sigma");
    const size_t items = (size_t)n_traj * v.n_w;
    if ((rs = srange(pred, items * v.n_x * v.n_y * sizeof(float), "pred")) != RAD_OK) return rs;
    if ((rs = srange(coarse, items * n_cells * sizeof(double), "coarse")) != RAD_OK) return rs;
    if ((rs = srange(mask, items * n_cells, "mask")) != RAD_OK) return rs;
    if ((rs = srange(fallback, items, "fallback")) != RAD_OK) return rs;
    if (cell_pred && (rs = srange(cell_pred, items * n_cells * sizeof(double), "cell_pred")) != RAD_OK) return rs;
    SelectLaunch L{pred, mu, sigma, coarse, v.wx, v.wy, n_traj, v.n_w, v.n_x, v.n_y, cx, cy, n_cells,
                   coverage, tau, cap, mask, fallback, cell_pred};
    hipError_t e = launch_select(L, (hipStream_t)stream);
    if (e == hipSuccess) e = launch_widen(mask, n_traj, v.n_w, n_cells, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "select: %s", hipGetErrorString(e));
}

rad_status rad_sampler_select_error(const rad_grid *fine, int n_traj, const float *pred, float mu, float sigma,
                                    const double *coarse, int cx, int cy, float eps, int cap, uint8_t *mask,
                                    double *cell_est, void *stream)
{
    rad::GridView v;
    rad_status rs = view_of(fine, v);
    if (rs != RAD_OK) return rs;
    int n_cells = 0;
    if ((rs = cells_shape(v, cx, cy, n_cells)) != RAD_OK) return rs;
    if (n_traj <= 0) return sfail(RAD_EINVAL, "n_traj must be > 0");
    if (!(eps >= 0.0f) || !std::isfinite(eps) || cap < 1 || !std::isfinite(mu) || !std::isfinite(sigma))
        return sfail(RAD_EINVAL, "invalid eps, cap, mu or sigma");
    const size_t items = (size_t)n_traj * v.n_w;
    if ((rs = srange(pred, items * v.n_x * v.n_y * sizeof(float), "pred")) != RAD_OK) return rs;
    if ((rs = srange(coarse, items * n_cells * sizeof(double), "coarse")) != RAD_OK) return rs;
    if ((rs = srange(mask, items * n_cells, "mask")) != RAD_OK) return rs;
    if ((rs = srange(cell_est, items * n_cells * sizeof(double), "cell_est")) != RAD_OK) return rs;
    SelectLaunch L{pred, mu, sigma, coarse, v.wx, v.wy, n_traj, v.n_w, v.n_x, v.n_y, cx, cy, n_cells,
                   eps, 0.0f, cap, mask, nullptr, cell_est};
    hipError_t e = launch_select_error(L, (hipStream_t)stream);
    if (e == hipSuccess) e = launch_widen(mask, n_traj, v.n_w, n_cells, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "select_error: %s", hipGetErrorString(e));
}

rad_status rad_sampler_coarse_pred(const rad_grid *fine, int n_traj, const double *coarse, int cx, int cy, float *pred,
                                   void *stream)
{
    rad::GridView v;
    rad_status rs = view_of(fine, v);
    if (rs != RAD_OK) return rs;
    int n_cells = 0;
    if ((rs = cells_shape(v, cx, cy, n_cells)) != RAD_OK) return rs;
    if (n_traj <= 0) return sfail(RAD_EINVAL, "n_traj must be > 0");
    const size_t maps = (size_t)n_traj * v.n_w;
    if ((rs = srange(coarse, maps * n_cells * sizeof(double), "coarse")) != RAD_OK) return rs;
    if ((rs = srange(pred, maps * v.n_x * v.n_y * sizeof(float), "pred")) != RAD_OK) return rs;
    hipError_t e = launch_coarse_pred(coarse, (int64_t)maps, v.n_x, v.n_y, cx, cy, pred, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "coarse_pred: %s", hipGetErrorString(e));
}

rad_status rad_sampler_combine(const rad_grid *fine, int n_traj, int cx, int cy, const double *cells,
                               const uint8_t *mask, const double *coarse, const double *cell_pred,
                               const uint8_t *fallback, const double *full, double *dIdw, void *stream)
{
    rad::GridView v;
    rad_status rs = view_of(fine, v);
    if (rs != RAD_OK) return rs;
    int n_cells = 0;
    if ((rs = cells_shape(v, cx, cy, n_cells)) != RAD_OK) return rs;
    if (n_traj <= 0) return sfail(RAD_EINVAL, "n_traj must be > 0");
    const size_t items = (size_t)n_traj * v.n_w;
    if ((rs = srange(cells, items * n_cells * sizeof(double), "cells")) != RAD_OK) return rs;
    if ((rs = srange(coarse, items * n_cells * sizeof(double), "coarse")) != RAD_OK) return rs;
    if ((rs = srange(mask, items * n_cells, "mask")) != RAD_OK) return rs;
    if ((rs = srange(dIdw, items * sizeof(double), "dIdw")) != RAD_OK) return rs;
    if (cell_pred && (rs = srange(cell_pred, items * n_cells * sizeof(double), "cell_pred")) != RAD_OK) return rs;
    if ((fallback == nullptr) != (full == nullptr)) return sfail(RAD_EINVAL, "fallback and full go together");
    if (fallback && ((rs = srange(fallback, items, "fallback")) != RAD_OK ||
                     (rs = srange(full, items * sizeof(double), "full")) != RAD_OK))
        return rs;
    CombineLaunch L{cells, coarse, v.wx, v.wy, cell_pred, mask, fallback, full, n_traj, v.n_w, v.n_x, cx, cy,
                    n_cells, dIdw};
    hipError_t e = launch_combine(L, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "combine: %s", hipGetErrorString(e));
}

rad_status rad_sampler_targets(const double *S, int64_t n_maps, int n_dirs, float floor_rel, float *y, void *stream)
{
    if (n_maps <= 0 || n_maps > ((int64_t)1 << 31) - 1 || n_dirs <= 0 || !(floor_rel > 0.0f) || !std::isfinite(floor_rel))
        return sfail(RAD_EINVAL, "need n_maps in [1, 2^31), n_dirs >= 1 and a finite floor_rel > 0");
    rad_status rs;
    const size_t n = (size_t)n_maps * n_dirs;
    if ((rs = srange(S, n * sizeof(double), "S")) != RAD_OK || (rs = srange(y, n * sizeof(float), "y")) != RAD_OK)
        return rs;
    hipError_t e = launch_targets(S, n_maps, n_dirs, floor_rel, y, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "targets: %s", hipGetErrorString(e));
}

size_t rad_sampler_moments_workspace_bytes(void) { return (size_t)kMomentParts * sizeof(double); }

rad_status rad_sampler_moments(const float *y, int64_t n, double *moments, void *ws, size_t ws_bytes, void *stream)
{
    if (n <= 0) return sfail(RAD_EINVAL, "n must be > 0");
    if (ws_bytes < rad_sampler_moments_workspace_bytes())
        return sfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, rad_sampler_moments_workspace_bytes());
    rad_status rs;
    if ((rs = srange(y, (size_t)n * sizeof(float), "y")) != RAD_OK ||
        (rs = srange(moments, 2 * sizeof(double), "moments")) != RAD_OK ||
        (rs = srange(ws, rad_sampler_moments_workspace_bytes(), "workspace")) != RAD_OK)
        return rs;
    hipError_t e = launch_moments(y, n, (double *)ws, kMomentParts, moments, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "moments: %s", hipGetErrorString(e));
}

rad_status rad_sampler_minibatch(const float *Y, const int *W, int64_t n, int nwt, int npix, const float *point_x,
                                 int64_t n_points, const double *moments, int batch, uint64_t seed, uint64_t step,
                                 int *traj, float *x, float *target, void *stream)
{
    if (n <= 0 || n > ((int64_t)1 << 31) - 1 || nwt <= 0 || npix <= 0 || batch <= 0 || n_points <= 0)
        return sfail(RAD_EINVAL, "need n in [1, 2^31), nwt, npix, batch, n_points >= 1");
    rad_status rs;
    if ((rs = srange(Y, (size_t)n * nwt * npix * sizeof(float), "Y")) != RAD_OK ||
        (rs = srange(W, (size_t)n * nwt * sizeof(int), "W")) != RAD_OK ||
        (rs = srange(point_x, (size_t)n_points * 3 * sizeof(float), "point_x")) != RAD_OK ||
        (rs = srange(moments, 2 * sizeof(double), "moments")) != RAD_OK ||
        (rs = srange(traj, (size_t)batch * sizeof(int), "traj")) != RAD_OK ||
        (rs = srange(x, (size_t)batch * 3 * sizeof(float), "x")) != RAD_OK ||
        (rs = srange(target, (size_t)batch * sizeof(float), "target")) != RAD_OK)
        return rs;
    if (n_points % npix) return sfail(RAD_EINVAL, "the point table is not whole energies of npix directions");
    BatchLaunch L{Y, W, point_x, n_points, n, nwt, npix, moments, batch, seed, step, traj, x, target};
    hipError_t e = launch_minibatch(L, (hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : sfail(RAD_EDEVICE, "minibatch: %s", hipGetErrorString(e));
}

}  // extern "C"

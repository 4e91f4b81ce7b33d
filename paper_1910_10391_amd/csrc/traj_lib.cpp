// librad: host side of the trajectory generator C ABI (include/rad_traj.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "rad_internal.h"
#include "rad_traj.h"
#include "traj_internal.h"

using namespace radtraj;

namespace {

rad_status tfail(rad_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    rad_err::set(buf);
    return st;
}

rad_status trange(const void *p, size_t bytes, const char *name)
{
    if (!p) return tfail(RAD_EINVAL, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return tfail(RAD_EINVAL, "%s (%p) is not a device allocation", name, p);
    }
    if ((const char *)p + bytes > (const char *)base + size)
        return tfail(RAD_EINVAL, "%s: %zu bytes exceed its device allocation", name, bytes);
    return RAD_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

rad_status check_params(const rad_traj_params *p)
{
    if (!p) return tfail(RAD_EINVAL, "params is NULL");
    if (!(std::isfinite(p->energy_eV) && p->energy_eV > kMe_eV)) return tfail(RAD_EINVAL, "energy_eV must exceed m_e");
    if (!(p->charge == 1.0 || p->charge == -1.0)) return tfail(RAD_EINVAL, "charge must be +1 or -1");
    if (!std::isfinite(p->U0_eV) || !finite_pos(p->d_m) || !(p->q >= 0.0 && p->q <= 1.0) ||
        !finite_pos(p->length_m) || !(std::isfinite(p->theta_sigma) && p->theta_sigma >= 0.0) ||
        !finite_pos(p->X0_m) || !(std::isfinite(p->eps_s_eV) && p->eps_s_eV >= 0.0))
        return tfail(RAD_EINVAL, "invalid well, crystal or scattering parameter");
    if (p->n_min < 1 || p->n_max < p->n_min || p->n_max > (int64_t)1 << 40)
        return tfail(RAD_EINVAL, "need 1 <= n_min <= n_max");
    return RAD_OK;
}

}  // namespace

extern "C" {

rad_status rad_traj_lengths(const rad_traj_params *p, int64_t first, int n_particles, int64_t *out)
{
    rad_status rs = check_params(p);
    if (rs != RAD_OK) return rs;
    if (n_particles <= 0 || !out || first < 0) return tfail(RAD_EINVAL, "need n_particles > 0, first >= 0, out");
    for (int i = 0; i < n_particles; ++i) {
        Stream r = particle_stream(p->seed, first + i);
        out[i] = draw_steps(*p, r);
    }
    return RAD_OK;
}

namespace {
// Workspace: the descriptors, then (with scattering) the kick normals [max_steps][n][2].
size_t desc_bytes(int n_particles) { return ((sizeof(TrajDesc) * (size_t)n_particles + 255) / 256) * 256; }
}  // namespace

size_t rad_traj_workspace_bytes(const rad_traj_params *p, int64_t first, int n_particles)
{
    if (!p || n_particles <= 0 || first < 0 || check_params(p) != RAD_OK) return 0;
    int64_t max_steps = 0;
    for (int i = 0; i < n_particles; ++i) {
        Stream r = particle_stream(p->seed, first + i);
        max_steps = std::max<int64_t>(max_steps, draw_steps(*p, r));
    }
    size_t b = desc_bytes(n_particles);
    if (p->ms_on) b += sizeof(double) * 2 * (size_t)max_steps * (size_t)n_particles;
    return b;
}

rad_status rad_traj_generate(const rad_traj_params *p, int64_t first, int n_particles, double *cols,
                             int64_t total_samples, void *ws, size_t ws_bytes, void *stream)
{
    rad_status rs = check_params(p);
    if (rs != RAD_OK) return rs;
    if (n_particles <= 0 || first < 0) return tfail(RAD_EINVAL, "need n_particles > 0 and first >= 0");
    std::vector<TrajDesc> desc(n_particles);
    int64_t off = 0, max_steps = 0;
    for (int i = 0; i < n_particles; ++i) {
        Stream r = particle_stream(p->seed, first + i);
        desc[i].n = draw_steps(*p, r);
        desc[i].off = off;
        off += desc[i].n + 1;
        max_steps = std::max<int64_t>(max_steps, desc[i].n);
    }
    if (off != total_samples)
        return tfail(RAD_EINVAL, "total_samples is %lld, the particles have %lld", (long long)total_samples,
                     (long long)off);
    const size_t need = rad_traj_workspace_bytes(p, first, n_particles);
    if (ws_bytes < need) return tfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if ((rs = trange(ws, need, "workspace")) != RAD_OK) return rs;
    if ((rs = trange(cols, (size_t)RAD_TRAJ_NCOL * (size_t)total_samples * sizeof(double), "cols")) != RAD_OK)
        return rs;
    double *kicks = p->ms_on ? (double *)((char *)ws + desc_bytes(n_particles)) : nullptr;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t copied = nullptr;
    hipError_t e = hipEventCreateWithFlags(&copied, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws, desc.data(), sizeof(TrajDesc) * desc.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(copied, st);
    TrajLaunch L{*p, first, n_particles, total_samples, (const TrajDesc *)ws, cols, kicks, max_steps};
    if (e == hipSuccess && kicks) e = launch_kicks(L, st);
    if (e == hipSuccess) e = launch_traj(L, st);
    // the descriptors are pageable host memory: wait for their copy (not the kernel)
    if (e == hipSuccess) e = hipEventSynchronize(copied);
    if (copied) (void)hipEventDestroy(copied);
    if (e != hipSuccess) return tfail(RAD_EDEVICE, "trajectory generation: %s", hipGetErrorString(e));
    return RAD_OK;
}

size_t rad_traj_sections_workspace_bytes(int n_particles, int n_sections)
{
    if (n_particles <= 0 || n_sections <= 0) return 0;
    return (sizeof(SecDesc) + sizeof(double)) * (size_t)n_particles * (size_t)n_sections;
}

rad_status rad_traj_sections(const rad_traj_params *p, int64_t first, int n_particles, int n_sections,
                             const double *cols, int64_t total_samples, double *sec_cols,
                             int64_t total_section_samples, double *entry_energy, void *ws, size_t ws_bytes,
                             void *stream)
{
    rad_status rs = check_params(p);
    if (rs != RAD_OK) return rs;
    if (n_particles <= 0 || first < 0 || n_sections <= 0 || !entry_energy)
        return tfail(RAD_EINVAL, "need n_particles > 0, first >= 0, n_sections > 0, entry_energy");
    if (p->n_min < n_sections) return tfail(RAD_EINVAL, "n_min (%lld) < n_sections (%d)", (long long)p->n_min, n_sections);
    const int64_t n_sec = (int64_t)n_particles * n_sections;
    if (n_sec > (1 << 30)) return tfail(RAD_EINVAL, "too many sections");
    std::vector<SecDesc> desc((size_t)n_sec);
    int64_t src = 0, dst = 0;
    for (int i = 0; i < n_particles; ++i) {
        Stream r = particle_stream(p->seed, first + i);
        const int64_t n = draw_steps(*p, r);
        for (int s = 0; s < n_sections; ++s) {
            const int64_t k0 = ((int64_t)s * n) / n_sections, k1 = ((int64_t)(s + 1) * n) / n_sections;
            desc[(size_t)i * n_sections + s] = SecDesc{src, k0, k1, dst};
            dst += k1 - k0 + 1;
        }
        src += n + 1;
    }
    if (src != total_samples)
        return tfail(RAD_EINVAL, "total_samples is %lld, the particles have %lld", (long long)total_samples,
                     (long long)src);
    if (dst != total_section_samples)
        return tfail(RAD_EINVAL, "total_section_samples is %lld, the sections have %lld",
                     (long long)total_section_samples, (long long)dst);
    const size_t need = rad_traj_sections_workspace_bytes(n_particles, n_sections);
    if (ws_bytes < need) return tfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if ((rs = trange(ws, need, "workspace")) != RAD_OK) return rs;
    if ((rs = trange(cols, (size_t)RAD_TRAJ_NCOL * (size_t)total_samples * sizeof(double), "cols")) != RAD_OK)
        return rs;
    if ((rs = trange(sec_cols, (size_t)RAD_TRAJ_NCOL * (size_t)total_section_samples * sizeof(double),
                     "sec_cols")) != RAD_OK)
        return rs;
    hipStream_t st = (hipStream_t)stream;
    SecDesc *d_desc = (SecDesc *)ws;
    double *d_energy = (double *)((char *)ws + sizeof(SecDesc) * (size_t)n_sec);
    hipError_t e = hipMemcpyAsync(d_desc, desc.data(), sizeof(SecDesc) * (size_t)n_sec, hipMemcpyHostToDevice, st);
    SecLaunch L{d_desc, (int)n_sec, p->energy_eV / kMe_eV, cols, total_samples, sec_cols, total_section_samples,
                d_energy};
    if (e == hipSuccess) e = launch_sections(L, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(entry_energy, d_energy, sizeof(double) * (size_t)n_sec, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return tfail(RAD_EDEVICE, "trajectory sections: %s", hipGetErrorString(e));
    return RAD_OK;
}

}  // extern "C"

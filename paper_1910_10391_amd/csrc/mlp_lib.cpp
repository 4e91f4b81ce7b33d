// librad: host side of the MLP C ABI (include/rad_mlp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mlp_internal.h"
#include "rad_mlp.h"

using namespace radmlp;

struct rad_mlp {
    MlpLayout L{};
    int device = 0;
    float *p = nullptr, *m1 = nullptr, *m2 = nullptr;
    uint16_t *W1p = nullptr, *W2 = nullptr, *W2T = nullptr, *W3 = nullptr, *W3T = nullptr, *W3P = nullptr,
             *W4 = nullptr;
    int64_t step = 0;
    int n_cu = 256;
};

// Error text shared with the rest of librad.
namespace rad_err {
void set(const char *msg);
}

namespace {

rad_status mfail(rad_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    rad_err::set(buf);
    return st;
}

rad_status mhip(hipError_t e, const char *what)
{
    return mfail(RAD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// batches are padded to whole row blocks of the row products
int64_t round_rows(int64_t b) { return (b + kRowBlock - 1) / kRowBlock * kRowBlock; }
size_t al(size_t x) { return (x + 255) / 256 * 256; }

MlpLayout make_layout(int nf, int np)
{
    MlpLayout L;
    L.n_feat = nf;
    L.n_point = np;
    L.n_in = nf + np;
    int64_t o = 0;
    L.w1 = o; o += (int64_t)kWidth * L.n_in;
    L.b1 = o; o += kWidth;
    L.w2 = o; o += (int64_t)kWidth * kWidth;
    L.b2 = o; o += kWidth;
    L.w3 = o; o += (int64_t)kWidth * kWidth;
    L.b3 = o; o += kWidth;
    L.w4 = o; o += kWidth;
    L.b4 = o; o += 1;
    L.total = o;
    return L;
}

// Workspace carve-up for a padded batch Bp and n_traj trajectories.
struct MWs {
    uint16_t *in1, *in1_k8, *h1, *h2, *h3, *h1_k8, *h2_k8, *dzA, *dzB, *dz_k8;
    uint16_t *ds1, *ds2, *ds3;   // silu' of the layers' pre-activations (BF16)
    float *y, *cb;
    float *part[3];      // split-K partials of the W3, W2, W1 gradients
    float *opart;        // output-layer partials [Bp / 64][514]
    float *colpart[2];   // column partials of dz2, dz1 [Bp / 64][256]
    size_t total;
};

constexpr int kSplits = 64;     // most split-K slices of the weight-gradient products

// Inference needs the folded biases, and unless the fused kernel runs (n_point <= 8)
// also h1..h3 and y (about 1.5 KB per point).
MWs carve_infer(char *base, int64_t Bp, int n_traj, bool fused)
{
    MWs w{};
    size_t o = 0;
    auto take = [&](size_t bytes) { char *p = base ? base + o : nullptr; o = al(o + bytes); return p; };
    const size_t act = fused ? 0 : (size_t)Bp * kWidth;
    if (!fused) {
        w.h1 = (uint16_t *)take(act * 2);
        w.h2 = (uint16_t *)take(act * 2);
        w.h3 = (uint16_t *)take(act * 2);
        w.y = (float *)take((size_t)Bp * 4);
    }
    w.cb = (float *)take((size_t)std::max(n_traj, 1) * kWidth * 4);
    w.total = o;
    return w;
}

bool fused_ok(const rad_mlp *m) { return m && m->L.n_point <= kFusedMaxPointHost; }

MWs carve(char *base, int64_t Bp, int n_traj)
{
    MWs w{};
    size_t o = 0;
    auto take = [&](size_t bytes) { char *p = base ? base + o : nullptr; o = al(o + bytes); return p; };
    const size_t act = (size_t)Bp * kWidth;
    w.in1 = (uint16_t *)take((size_t)Bp * kIn1 * 2);
    w.in1_k8 = (uint16_t *)take((size_t)Bp * kIn1 * 2);
    w.h1 = (uint16_t *)take(act * 2);
    w.h2 = (uint16_t *)take(act * 2);
    w.h3 = (uint16_t *)take(act * 2);
    w.h1_k8 = (uint16_t *)take(act * 2);
    w.h2_k8 = (uint16_t *)take(act * 2);
    w.dzA = (uint16_t *)take(act * 2);
    w.dzB = (uint16_t *)take(act * 2);
    w.dz_k8 = (uint16_t *)take(act * 2);
    w.ds1 = (uint16_t *)take(act * 2);
    w.ds2 = (uint16_t *)take(act * 2);
    w.ds3 = (uint16_t *)take(act * 2);
    w.y = (float *)take((size_t)Bp * 4);
    for (int l = 0; l < 3; ++l) w.part[l] = (float *)take((size_t)kSplits * kWidth * (l == 2 ? kIn1 : kWidth) * 4);
    w.opart = (float *)take((size_t)(Bp / kOutPointsHost) * kOutPartHost * 4);
    for (int l = 0; l < 2; ++l) w.colpart[l] = (float *)take((size_t)(Bp / kRowTile) * kWidth * 4);
    w.cb = (float *)take((size_t)std::max(n_traj, 1) * kWidth * 4);
    w.total = o;
    return w;
}

rad_status check_mlp(const rad_mlp *m)
{
    if (!m) return mfail(RAD_EINVAL, "mlp is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return mfail(RAD_EDEVICE, "no HIP device");
    if (dev != m->device) return mfail(RAD_EINVAL, "mlp lives on device %d, current device is %d", m->device, dev);
    return RAD_OK;
}

rad_status check_range(const void *p, size_t bytes, const char *name)
{
    if (!p) return mfail(RAD_EINVAL, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(RAD_EINVAL, "%s (%p) is not a device allocation", name, p);
    }
    if ((const char *)p + bytes > (const char *)base + size)
        return mfail(RAD_EINVAL, "%s: %zu bytes exceed its device allocation", name, bytes);
    return RAD_OK;
}

rad_status check_batch(const rad_mlp *m, const float *feat, int n_traj, const int *traj, const float *x, int batch,
                       void *ws, size_t ws_bytes, MWs &w, bool training)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if (batch <= 0 || n_traj <= 0) return mfail(RAD_EINVAL, "batch and n_traj must be > 0");
    if (batch > (1 << 26)) return mfail(RAD_EINVAL, "batch too large");
    const int64_t Bp = round_rows(batch);
    w = training ? carve(nullptr, Bp, n_traj) : carve_infer(nullptr, Bp, n_traj, fused_ok(m));
    if (!ws) return mfail(RAD_EINVAL, "workspace is NULL");
    if (ws_bytes < w.total) return mfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, w.total);
    if ((rs = check_range(ws, w.total, "workspace")) != RAD_OK) return rs;
    if (m->L.n_feat > 0 && (rs = check_range(feat, (size_t)n_traj * m->L.n_feat * 4, "feat")) != RAD_OK) return rs;
    if ((rs = check_range(traj, (size_t)batch * 4, "traj")) != RAD_OK) return rs;
    if ((rs = check_range(x, (size_t)batch * m->L.n_point * 4, "x")) != RAD_OK) return rs;
    w = training ? carve((char *)ws, Bp, n_traj) : carve_infer((char *)ws, Bp, n_traj, fused_ok(m));
    return RAD_OK;
}

struct Splitmix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

}  // namespace

extern "C" {

rad_status rad_mlp_create(int n_feat, int n_point, uint64_t seed, void *stream, rad_mlp **out)
{
    if (!out) return mfail(RAD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_feat < 0 || n_point < 1 || n_feat + n_point > kIn1)
        return mfail(RAD_EINVAL, "need n_feat >= 0, n_point >= 1, n_feat + n_point <= %d", kIn1);
    rad_mlp *m = new rad_mlp();
    m->L = make_layout(n_feat, n_point);
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return mfail(RAD_EDEVICE, "no HIP device");
    }
    if (hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
        m->n_cu < 1)
        m->n_cu = 256;
    const size_t P = (size_t)m->L.total;
    const size_t sq = (size_t)kWidth * kWidth;
    struct { void **p; size_t bytes; } allocs[] = {
        {(void **)&m->p, P * 4}, {(void **)&m->m1, P * 4}, {(void **)&m->m2, P * 4},
        {(void **)&m->W1p, (size_t)kWidth * kIn1 * 2}, {(void **)&m->W2, sq * 2}, {(void **)&m->W2T, sq * 2},
        {(void **)&m->W3, sq * 2}, {(void **)&m->W3T, sq * 2}, {(void **)&m->W3P, sq * 2},
        {(void **)&m->W4, (size_t)kWidth * 2}};
    for (auto &a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            rad_mlp_free(m);
            return mfail(RAD_ENOMEM, "hipMalloc of %zu bytes for the MLP", a.bytes);
        }
    }
    // initial parameters
    std::vector<float> h(P, 0.0f);
    Splitmix rng{seed * 0x9E3779B97F4A7C15ull + 0x1234567ull};
    auto fill = [&](int64_t off, int64_t n, int fan_in, double scale) {
        const double a = scale * std::sqrt(6.0 / fan_in);
        for (int64_t i = 0; i < n; ++i) h[off + i] = (float)((2.0 * rng.uniform() - 1.0) * a);
    };
    fill(m->L.w1, (int64_t)kWidth * m->L.n_in, m->L.n_in, 1.0);
    fill(m->L.w2, (int64_t)sq, kWidth, 1.0);
    fill(m->L.w3, (int64_t)sq, kWidth, 1.0);
    fill(m->L.w4, kWidth, kWidth, 0.25);
    rad_status rs = rad_mlp_set_params(m, h.data(), stream);
    if (rs != RAD_OK) {
        rad_mlp_free(m);
        return rs;
    }
    std::vector<float> zero(P, 0.0f);
    rs = rad_mlp_set_adam(m, zero.data(), zero.data(), 0, stream);
    if (rs != RAD_OK) {
        rad_mlp_free(m);
        return rs;
    }
    *out = m;
    return RAD_OK;
}

void rad_mlp_free(rad_mlp *m)
{
    if (!m) return;
    for (void *p : {(void *)m->p, (void *)m->m1, (void *)m->m2, (void *)m->W1p, (void *)m->W2, (void *)m->W2T,
                    (void *)m->W3, (void *)m->W3T, (void *)m->W3P, (void *)m->W4})
        if (p) (void)hipFree(p);
    delete m;
}

int64_t rad_mlp_param_count(const rad_mlp *m) { return m ? m->L.total : 0; }

rad_status rad_mlp_get_params(const rad_mlp *m, float *host, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if (!host) return mfail(RAD_EINVAL, "host buffer is NULL");
    hipError_t e = hipMemcpyAsync(host, m->p, (size_t)m->L.total * 4, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? RAD_OK : mhip(e, "parameter download");
}

rad_status rad_mlp_set_params(rad_mlp *m, const float *host, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if (!host) return mfail(RAD_EINVAL, "host buffer is NULL");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(m->p, host, (size_t)m->L.total * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_refresh(m->p, m->L, m->W1p, m->W2, m->W2T, m->W3, m->W3T, m->W3P, m->W4, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e == hipSuccess ? RAD_OK : mhip(e, "parameter upload");
}

rad_status rad_mlp_get_adam(const rad_mlp *m, float *m1, float *m2, int64_t *step, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    const size_t b = (size_t)m->L.total * 4;
    hipError_t e = hipSuccess;
    if (m1) e = hipMemcpyAsync(m1, m->m1, b, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && m2) e = hipMemcpyAsync(m2, m->m2, b, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (step) *step = m->step;
    return e == hipSuccess ? RAD_OK : mhip(e, "Adam state download");
}

rad_status rad_mlp_set_adam(rad_mlp *m, const float *m1, const float *m2, int64_t step, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if (step < 0) return mfail(RAD_EINVAL, "step must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    const size_t b = (size_t)m->L.total * 4;
    hipError_t e = hipSuccess;
    if (m1) e = hipMemcpyAsync(m->m1, m1, b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && m2) e = hipMemcpyAsync(m->m2, m2, b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    m->step = step;
    return e == hipSuccess ? RAD_OK : mhip(e, "Adam state upload");
}

size_t rad_mlp_workspace_bytes(const rad_mlp *m, int batch, int n_traj, int training)
{
    if (!m || batch <= 0 || n_traj <= 0) return 0;
    return (training ? carve(nullptr, round_rows(batch), n_traj)
                     : carve_infer(nullptr, round_rows(batch), n_traj, fused_ok(m))).total;
}

rad_status rad_mlp_grad(const rad_mlp *m, const float *feat, int n_traj, const int *traj, const float *x,
                        const float *target, int batch, float *grad, float *loss_sum, void *ws, size_t ws_bytes,
                        void *stream)
{
    MWs w;
    rad_status rs = check_batch(m, feat, n_traj, traj, x, batch, ws, ws_bytes, w, true);
    if (rs != RAD_OK) return rs;
    if ((rs = check_range(target, (size_t)batch * 4, "target")) != RAD_OK) return rs;
    if ((rs = check_range(grad, (size_t)m->L.total * 4, "grad")) != RAD_OK) return rs;
    if ((rs = check_range(loss_sum, 4, "loss_sum")) != RAD_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    const MlpLayout &L = m->L;
    const int B = batch;
    const int Bp = (int)round_rows(batch);
    // split-K slices of the weight gradients: a power of two dividing the row blocks
    int splits = 1;
    while (splits < kSplits && (Bp / kRowBlock) % (2 * splits) == 0) splits *= 2;
    hipError_t e;
#define CK(x)                                               \
    do {                                                    \
        e = (x);                                            \
        if (e != hipSuccess) return mhip(e, #x);            \
    } while (0)
    // forward: h = silu(z) row-major for the next layer, and in the k8 layout (batch rows
    // interleaved by 8) for the weight gradients
    CK(launch_assemble_in1(feat, L.n_feat, traj, x, L.n_point, B, Bp, w.in1, w.in1_k8, st));
    RowsArgs g{w.in1, m->W1p, Bp, kIn1, m->p + L.b1, nullptr, w.ds1, w.h1, w.h1_k8, nullptr};
    CK(launch_rows(kEpiFwd, g, st));
    g = RowsArgs{w.h1, m->W2, Bp, kWidth, m->p + L.b2, nullptr, w.ds2, w.h2, w.h2_k8, nullptr};
    CK(launch_rows(kEpiFwd, g, st));
    g = RowsArgs{w.h2, m->W3, Bp, kWidth, m->p + L.b3, nullptr, w.ds3, w.h3, nullptr, nullptr};
    CK(launch_rows(kEpiFwd, g, st));
    // output layer: loss, dz3, and the per-block partials of the b3, W4, b4 gradients and
    // the loss (b3, W4, b4 are contiguous in the parameter vector)
    CK(launch_output_grad(w.h3, m->W4, m->p + L.b4, B, Bp, target, w.ds3, w.dzA, w.dz_k8, w.opart, st));
    static_assert(kOutPartHost == 2 * kWidth + 2, "partials: b3, W4, b4, loss");
    // layers 3, 2, 1: split-K partials of dW = dz^T h_prev from the k8 layouts, then
    // dz_prev = (dz W) silu'(z_prev) with the per-block column sums of dz_prev
    const uint16_t *hprev_k8[3] = {w.h2_k8, w.h1_k8, w.in1_k8};
    const int nprev[3] = {kWidth, kWidth, kIn1};
    const uint16_t *WT[2] = {m->W3T, m->W2T};
    const uint16_t *dsprev[2] = {w.ds2, w.ds1};
    uint16_t *dz_cur = w.dzA, *dz_next = w.dzB;
    for (int l = 0; l < 3; ++l) {
        K8Args k8{w.dz_k8, hprev_k8[l], kWidth, nprev[l], (int64_t)Bp / splits, w.part[l]};
        CK(launch_k8(k8, splits, st));
        if (l < 2) {
            g = RowsArgs{dz_cur, WT[l], Bp, kWidth, nullptr, dsprev[l], nullptr, dz_next, w.dz_k8, w.colpart[l]};
            CK(launch_rows(kEpiBwd, g, st));
            uint16_t *t = dz_cur;
            dz_cur = dz_next;
            dz_next = t;
        }
    }
    // every reduction into the gradient vector, in one launch
    FinishArgs f{};
    const int64_t woff[3] = {L.w3, L.w2, L.w1};
    for (int l = 0; l < 3; ++l) f.w[l] = FinishW{w.part[l], splits, nprev[l], l == 2 ? L.n_in : kWidth, grad + woff[l], 0};
    f.c[0] = FinishC{w.opart, kOutPartHost, Bp / kOutPointsHost, 2 * kWidth + 2, 2 * kWidth + 1, grad + L.b3, loss_sum, 0};
    f.c[1] = FinishC{w.colpart[0], kWidth, Bp / kRowTile, kWidth, kWidth, grad + L.b2, nullptr, 0};
    f.c[2] = FinishC{w.colpart[1], kWidth, Bp / kRowTile, kWidth, kWidth, grad + L.b1, nullptr, 0};
    CK(launch_finish_grad(f, st));
#undef CK
    return RAD_OK;
}

rad_status rad_mlp_adam(rad_mlp *m, const float *grad, float lr, float beta1, float beta2, float eps, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if ((rs = check_range(grad, (size_t)m->L.total * 4, "grad")) != RAD_OK) return rs;
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return mfail(RAD_EINVAL, "invalid Adam hyper-parameters");
    hipStream_t st = (hipStream_t)stream;
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)m->step));
    hipError_t e = launch_adam(m->p, m->m1, m->m2, grad, m->L.total, lr, beta1, beta2, eps, c1, c2, st);
    if (e == hipSuccess) e = launch_refresh(m->p, m->L, m->W1p, m->W2, m->W2T, m->W3, m->W3T, m->W3P, m->W4, st);
    return e == hipSuccess ? RAD_OK : mhip(e, "Adam launch");
}

rad_status rad_mlp_forward(const rad_mlp *m, const float *feat, int n_traj, const int *traj, const float *x,
                           int batch, float *y, void *ws, size_t ws_bytes, void *stream)
{
    MWs w;
    rad_status rs = check_batch(m, feat, n_traj, traj, x, batch, ws, ws_bytes, w, false);
    if (rs != RAD_OK) return rs;
    if ((rs = check_range(y, (size_t)batch * 4, "y")) != RAD_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    const MlpLayout &L = m->L;
    const int Bp = (int)round_rows(batch);
    hipError_t e = launch_fold_bias(m->W1p, m->p + L.b1, feat, L.n_feat, n_traj, w.cb, st);
    if (fused_ok(m)) {
        if (e == hipSuccess)
            e = launch_infer_fused(m->W1p, m->W2, m->W3P, m->W4, w.cb, m->p + L.b2, m->p + L.b3, m->p + L.b4, traj, x,
                                   L.n_feat, L.n_point, batch, 0, y, m->n_cu, st);
        return e == hipSuccess ? RAD_OK : mhip(e, "MLP forward");
    }
    if (e == hipSuccess) e = launch_layer1_points(m->W1p, w.cb, L.n_feat, traj, x, L.n_point, batch, Bp, w.h1, st);
    RowsArgs g{w.h1, m->W2, Bp, kWidth, m->p + L.b2, nullptr, nullptr, w.h2, nullptr, nullptr};
    if (e == hipSuccess) e = launch_rows(kEpiFwd, g, st);
    g = RowsArgs{w.h2, m->W3, Bp, kWidth, m->p + L.b3, nullptr, nullptr, w.h3, nullptr, nullptr};
    if (e == hipSuccess) e = launch_rows(kEpiFwd, g, st);
    if (e == hipSuccess) e = launch_output(w.h3, m->W4, m->p + L.b4, batch, Bp, w.y, st);
    if (e == hipSuccess) e = hipMemcpyAsync(y, w.y, (size_t)batch * 4, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? RAD_OK : mhip(e, "MLP forward");
}

size_t rad_mlp_grid_workspace_bytes(const rad_mlp *m, int n_traj)
{
    if (!m || n_traj < 1) return 0;
    return carve_infer(nullptr, 0, n_traj, true).total;
}

rad_status rad_mlp_forward_grid(const rad_mlp *m, const float *feat, int n_traj, const float *x, int64_t n_pts,
                                float *y, void *ws, size_t ws_bytes, void *stream)
{
    rad_status rs = check_mlp(m);
    if (rs != RAD_OK) return rs;
    if (!fused_ok(m)) return mfail(RAD_EUNSUPPORTED, "the grid form needs n_point <= %d", kFusedMaxPointHost);
    if (n_traj < 1 || n_pts < 1) return mfail(RAD_EINVAL, "need n_traj >= 1 and n_pts >= 1");
    const int64_t B = (int64_t)n_traj * n_pts;
    if (B > ((int64_t)1 << 40)) return mfail(RAD_EINVAL, "too many points");
    const size_t need = rad_mlp_grid_workspace_bytes(m, n_traj);
    if (ws_bytes < need) return mfail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, need);
    if ((rs = check_range(ws, need, "workspace")) != RAD_OK) return rs;
    if (m->L.n_feat > 0 && (rs = check_range(feat, (size_t)n_traj * m->L.n_feat * 4, "feat")) != RAD_OK) return rs;
    if ((rs = check_range(x, (size_t)n_pts * m->L.n_point * 4, "x")) != RAD_OK) return rs;
    if ((rs = check_range(y, (size_t)B * 4, "y")) != RAD_OK) return rs;
    const MWs w = carve_infer((char *)ws, 0, n_traj, true);
    const MlpLayout &L = m->L;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_fold_bias(m->W1p, m->p + L.b1, feat, L.n_feat, n_traj, w.cb, st);
    if (e == hipSuccess)
        e = launch_infer_fused(m->W1p, m->W2, m->W3P, m->W4, w.cb, m->p + L.b2, m->p + L.b3, m->p + L.b4, nullptr,
                               x, L.n_feat, L.n_point, B, n_pts, y, m->n_cu, st);
    return e == hipSuccess ? RAD_OK : mhip(e, "MLP grid forward");
}

}  // extern "C"

// librad: host side of the C ABI declared in include/rad.h.
//
// Validates every argument on the host (including that device buffers lie
// inside a device allocation large enough for what the kernels touch), plans
// the launch (time chunks, block counts, longest-segment-first order), writes
// the segment descriptors into the caller's workspace and launches:
//   amp_kernel (one launch per integral set: kappa = k and/or kappa = k*),
//   fin_kernel (fixed-order reduction and spectrum weights),
//   angle_kernel (rad_angle_integrate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "rad.h"
#include "rad_internal.h"
#include "rad_plan.h"

namespace rad {
hipError_t launch_amp(const AmpLaunch &L, int variant, bool withj, bool mixed, int grid_blocks,
                      hipStream_t st, int *occupancy);
hipError_t launch_reset(unsigned *counters, int n, hipStream_t st);
hipError_t launch_cells_fin(const CellsFin &F, hipStream_t st);
hipError_t launch_cell_compact(const CellCompact &C, hipStream_t st);
hipError_t launch_fin(const FinLaunch &F, hipStream_t st);
hipError_t launch_phase(const double *turns, int64_t n, int mixed, double *c, double *s, hipStream_t st);
hipError_t launch_angle(const double *cube, const double *wx, const double *wy, int n_x, int n_y,
                        int n_w, int n_cubes, double *out, hipStream_t st);
}  // namespace rad

using namespace rad;

struct rad_plan;

struct rad_grid {
    int n_w = 0, n_x = 0, n_y = 0;
    int device = 0;
    double *d_hw = nullptr, *d_k = nullptr, *d_thx = nullptr, *d_thy = nullptr;
    double *d_wx = nullptr, *d_wy = nullptr;
    std::vector<double> hw, thx, thy;
    double dth = 0.0;   // common spacing of uniform thx and thy, or 0
    // pinned staging for descriptor uploads, reused after its last copy completed
    std::mutex mu;
    void *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    bool stage_pending = false;
};

namespace {

thread_local std::string g_err;

rad_status fail(rad_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rad_status hip_fail(hipError_t e, const char *what)
{
    return fail(RAD_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kInitialStage = (size_t)1 << 20;   // pinned descriptor staging per grid

// The int a C caller passed for a precision: read as bits through a reference, since
// loading a C++ enum value outside the enumeration's range is undefined behaviour.
int prec_value(const rad_precision &p)
{
    static_assert(sizeof(rad_precision) == sizeof(int), "rad_precision is an int");
    int v = 0;
    std::memcpy(&v, &p, sizeof v);
    return v;
}
bool valid_prec(const rad_precision &p) { return prec_value(p) == RAD_FP64 || prec_value(p) == RAD_MIXED; }

// ---- profiling
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pending;
double g_prof_ms = 0.0;
int64_t g_prof_launches = 0;

// The device allocation that holds [p, p + bytes) must exist.
rad_status check_dev_range(const void *p, size_t bytes, const char *name)
{
    if (!p) return fail(RAD_EINVAL, "%s is NULL", name);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RAD_EINVAL, "%s (%p) is not a device allocation", name, p);
    }
    const char *b = (const char *)base, *q = (const char *)p;
    if (q < b || q + bytes > b + size)
        return fail(RAD_EINVAL, "%s: %zu bytes at %p exceed its device allocation", name, bytes, p);
    return RAD_OK;
}

// Kernel variant per [persistent][mixed][with J]; the default is the measured best
// on MI355X for the benchmark shapes, the autotuner may change it.
std::mutex g_var_mu;
int g_variant[2][2][2] = {{{kVar44x2, kVar44x2}, {kVar44x2, kVar44x2}},
                          {{kVar44x2, kVar44x2}, {kVar44x2, kVar44x2}}};

int variant_for(bool persistent, bool mixed, bool withj)
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    return g_variant[persistent ? 1 : 0][mixed ? 1 : 0][withj ? 1 : 0];
}

// Launch-shape knobs, also set by the autotuner: waves of a block over photon energies
// per [persistent][mixed] (0: chosen by the grid), and the work-item target of the time
// chunking (0: kTargetBlocks), one for every form so that a workspace size holds for both.
int g_wg[2][2] = {{0, 0}, {0, 0}};
int64_t g_target = 0;

int wg_for(bool persistent, bool mixed)
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    return g_wg[persistent ? 1 : 0][mixed ? 1 : 0];
}

int64_t target_blocks()
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    return g_target > 0 ? g_target : radplan::kTargetBlocks;
}

using radplan::chunk_factor;
using radplan::kMaxChunk;
using radplan::kMinChunk;
using radplan::kTargetBlocks;
using radplan::Layout;
using radplan::plan_chunks;
using radplan::popcount3;
using radplan::Tile;
static_assert(radplan::kWave == kWave && radplan::kWavesPerBlock == kWavesPerBlock, "block shape");
static_assert(radplan::kClassical == RAD_CLASSICAL && radplan::kSpin0 == RAD_SPIN0 &&
              radplan::kSpinHalf == RAD_SPINHALF, "kind bits");
static_assert(sizeof(double2) == 16, "complex FP64 partials");

// Block shape for a grid and kernel variant; both integral sets of a call use
// the same chunking, so the tile counts of the larger direction tile decide it.
Tile plan_tile(const rad_grid *g, int variant, int wg = 0)
{
    return radplan::plan_tile(g->n_w, g->n_x, g->n_y, variant, kVarTX[variant], kVarTY[variant], wg);
}

Layout layout(const rad_grid *g, int n_segs, int n_out, int kinds, int64_t sum_chunks)
{
    return radplan::layout(g->n_w, g->n_x, g->n_y, sizeof(SegDesc), n_segs, n_out, kinds, sum_chunks);
}

rad_status check_grid(const rad_grid *g)
{
    if (!g) return fail(RAD_EINVAL, "grid is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(RAD_EDEVICE, "no HIP device");
    if (dev != g->device)
        return fail(RAD_EINVAL, "grid was built on device %d, current device is %d", g->device, dev);
    return RAD_OK;
}

rad_status check_segment(const rad_segment *s, int idx, bool quantum)
{
    if (!s) return fail(RAD_EINVAL, "segment %d is NULL", idx);
    if (s->n < 2) return fail(RAD_EINVAL, "segment %d: n = %lld < 2", idx, (long long)s->n);
    if (s->n > ((int64_t)1 << 40)) return fail(RAD_EINVAL, "segment %d: n too large", idx);
    if (!(std::isfinite(s->gamma) && s->gamma > 0.0))
        return fail(RAD_EINVAL, "segment %d: gamma must be finite and > 0", idx);
    if (quantum && !(std::isfinite(s->energy_eV) && s->energy_eV > 0.0))
        return fail(RAD_EINVAL, "segment %d: energy_eV must be finite and > 0", idx);
    const double *cols[C_NCOL] = {s->t, s->x, s->y, s->dz, s->vx, s->vy, s->dvz, s->ax, s->ay, s->az};
    static const char *names[C_NCOL] = {"t", "x", "y", "dz", "vx", "vy", "dvz", "ax", "ay", "az"};
    const size_t bytes = (size_t)s->n * sizeof(double);
    for (int c = 0; c < C_NCOL; ++c) {
        rad_status st = check_dev_range(cols[c], bytes, names[c]);
        if (st != RAD_OK) return fail(st, "segment %d: %s", idx, g_err.c_str());
    }
    if (s->w) {
        rad_status st = check_dev_range(s->w, bytes, "w");
        if (st != RAD_OK) return fail(st, "segment %d: %s", idx, g_err.c_str());
    }
    return RAD_OK;
}

void set_grid_tiles(SegDesc &d, const Tile &t)
{
    d.n_tx = t.n_tx;
    d.n_ty = t.n_ty;
    d.n_groups = t.n_groups;
    d.n_wblocks = t.n_wblocks;
}

// A planned call: everything the kernels need, decided on the host.
struct Plan {
    rad_grid *g = nullptr;
    int n_segs = 0, n_out = 0, kinds = 0, n_kinds = 0;
    bool mixed = false, quantum = false, withj = false;
    Layout lay{};
    Tile tile_c{}, tile_q{};
    int64_t blocks_c = 0, blocks_q = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<char> host;      // descriptor region, uploaded to ws[0, lay.desc_bytes)
    bool persistent = false;
    int pgrid_c = 0, pgrid_q = 0;  // persistent grid sizes
    bool one_chunk = false;        // every segment is a single time chunk
};

// fixed_cap > 0: `ws` is the library's own fixed scratch of fixed_cap bytes (no
// device-allocation check); the time chunks are then made coarser, down to one chunk
// per segment, until the workspace fits in it.
rad_status plan_build(rad_grid *g, const rad_segment *segs, int n_segs, const int *out_index,
                      int n_out, int kinds, rad_precision prec, void *ws, size_t ws_bytes,
                      bool persistent, Plan &P, size_t fixed_cap = 0)
{
    rad_status rs = check_grid(g);
    if (rs != RAD_OK) return rs;
    if (kinds <= 0 || kinds > 7) return fail(RAD_EINVAL, "kinds must be a non-empty subset of 1|2|4");
    if (!valid_prec(prec)) return fail(RAD_EINVAL, "unknown precision %d", prec_value(prec));
    if (!segs || n_segs <= 0) return fail(RAD_EINVAL, "no segments");
    if (!out_index) return fail(RAD_EINVAL, "out_index is NULL");
    if (n_out <= 0) return fail(RAD_EINVAL, "n_out must be > 0");
    const bool quantum = (kinds & (RAD_SPIN0 | RAD_SPINHALF)) != 0;
    for (int s = 0; s < n_segs; ++s) {
        if (out_index[s] < 0 || out_index[s] >= n_out)
            return fail(RAD_EINVAL, "out_index[%d] = %d outside [0, %d)", s, out_index[s], n_out);
        rs = check_segment(&segs[s], s, quantum);
        if (rs != RAD_OK) return rs;
    }
    P.g = g;
    P.n_segs = n_segs;
    P.n_out = n_out;
    P.kinds = kinds;
    P.n_kinds = popcount3(kinds);
    P.mixed = prec == RAD_MIXED;
    P.quantum = quantum;
    P.withj = (kinds & RAD_SPINHALF) != 0;
    const int wg = wg_for(persistent, P.mixed);
    P.tile_c = plan_tile(g, variant_for(persistent, P.mixed, false), wg);
    P.tile_q = plan_tile(g, variant_for(persistent, P.mixed, P.withj), wg);
    // chunking independent of the variant and of the energy spread (the 4x4 tile at the
    // grid's own spread), so that a workspace size holds for every form
    int64_t cf = chunk_factor(plan_tile(g, kVar44x2), n_segs, target_blocks());
    std::vector<int32_t> nch(n_segs), clen(n_segs);
    auto chunk_all = [&](int64_t c) {
        int64_t sum = 0;
        for (int s = 0; s < n_segs; ++s) {
            plan_chunks(segs[s].n, c, nch[s], clen[s]);
            sum += nch[s];
        }
        return sum;
    };
    int64_t sum_chunks = chunk_all(cf);
    P.lay = layout(g, n_segs, n_out, kinds, sum_chunks);
    if (fixed_cap > 0 && P.lay.total > fixed_cap) {
        // the largest chunk factor whose workspace fits (the size grows with the factor)
        int64_t lo = 1, hi = cf - 1;
        if (layout(g, n_segs, n_out, kinds, chunk_all(1)).total > fixed_cap)
            return fail(RAD_ENOMEM, "the call needs %zu bytes of scratch even in one time chunk per segment; "
                        "the fixed scratch holds %zu", layout(g, n_segs, n_out, kinds, chunk_all(1)).total, fixed_cap);
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (layout(g, n_segs, n_out, kinds, chunk_all(mid)).total <= fixed_cap) lo = mid; else hi = mid - 1;
        }
        cf = lo;
        sum_chunks = chunk_all(cf);
        P.lay = layout(g, n_segs, n_out, kinds, sum_chunks);
    }
    P.one_chunk = sum_chunks == n_segs;
    if (!ws) return fail(RAD_EINVAL, "workspace is NULL");
    if (ws_bytes < P.lay.total)
        return fail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, P.lay.total);
    if (fixed_cap == 0) {
        rs = check_dev_range(ws, P.lay.total, "workspace");
        if (rs != RAD_OK) return rs;
    }
    P.ws = (char *)ws;
    P.ws_bytes = ws_bytes;
    const size_t cube = (size_t)g->n_w * g->n_x * g->n_y;

    // launch order: longest segment first (dispatch order, and the persistent queue's order)
    std::vector<int> order(n_segs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return segs[a].n > segs[b].n; });

    P.host.assign(P.lay.desc_bytes, 0);
    SegDesc *amp_c = (SegDesc *)(P.host.data() + P.lay.off_amp_c);
    SegDesc *amp_q = (SegDesc *)(P.host.data() + P.lay.off_amp_q);
    SegDesc *id_c = (SegDesc *)(P.host.data() + P.lay.off_id_c);
    SegDesc *id_q = (SegDesc *)(P.host.data() + P.lay.off_id_q);
    int *begin = (int *)(P.host.data() + P.lay.off_begin);
    int *list = (int *)(P.host.data() + P.lay.off_list);

    std::vector<int64_t> part_off_c(n_segs), part_off_q(n_segs);
    {
        int64_t oc = 0, oq = 0;
        for (int s = 0; s < n_segs; ++s) {
            part_off_c[s] = oc;
            part_off_q[s] = oq;
            oc += (int64_t)nch[s] * 2 * (int64_t)cube;
            oq += (int64_t)nch[s] * P.lay.comps_q * (int64_t)cube;
        }
    }
    int64_t blocks_c = 0, blocks_q = 0;
    for (int r = 0; r < n_segs; ++r) {
        const int s = order[r];
        SegDesc d{};
        const rad_segment &sg = segs[s];
        const double *cols[C_NCOL] = {sg.t, sg.x, sg.y, sg.dz, sg.vx, sg.vy, sg.dvz, sg.ax, sg.ay, sg.az};
        for (int c = 0; c < C_NCOL; ++c) d.col[c] = cols[c];
        d.w = sg.w;
        d.n = sg.n;
        d.gamma = sg.gamma;
        d.c0 = 1.0 / (2.0 * sg.gamma * sg.gamma);
        d.energy = sg.energy_eV;
        d.n_chunks = nch[s];
        d.chunk_len = clen[s];
        d.hw = g->d_hw;
        d.k = g->d_k;
        d.thx = g->d_thx;
        d.thy = g->d_thy;
        d.dth = g->dth;
        d.n_w = g->n_w;
        d.n_x = g->n_x;
        d.n_y = g->n_y;
        SegDesc dc = d, dq = d;
        set_grid_tiles(dc, P.tile_c);
        set_grid_tiles(dq, P.tile_q);
        dc.block_begin = blocks_c;
        dq.block_begin = blocks_q;
        blocks_c += (int64_t)nch[s] * P.tile_c.base_blocks;
        blocks_q += (int64_t)nch[s] * P.tile_q.base_blocks;
        dc.part_off = part_off_c[s];
        dq.part_off = part_off_q[s];
        amp_c[r] = dc;
        amp_q[r] = dq;
        id_c[s] = dc;
        id_q[s] = dq;
    }
    if (std::max(blocks_c, blocks_q) >= ((int64_t)1 << 31) - 1)
        return fail(RAD_EUNSUPPORTED, "launch of %lld blocks", (long long)std::max(blocks_c, blocks_q));
    P.blocks_c = blocks_c;
    P.blocks_q = blocks_q;
    // outputs -> segments in segment order
    {
        std::vector<int> cnt(n_out + 1, 0);
        for (int s = 0; s < n_segs; ++s) cnt[out_index[s] + 1]++;
        for (int o = 0; o < n_out; ++o) cnt[o + 1] += cnt[o];
        for (int o = 0; o <= n_out; ++o) begin[o] = cnt[o];
        std::vector<int> fill(cnt.begin(), cnt.end() - 1);
        for (int s = 0; s < n_segs; ++s) list[fill[out_index[s]]++] = s;
    }
    // A one-block-per-item launch holds at most 2^32 - 1 work-items (2^24 - 1 blocks of
    // 256).  Its partial amplitudes take 128 kB per block on a full direction tile, so only
    // a grid of very many energies over few directions gets there within device memory;
    // such a launch runs its items on the persistent kernel with the same tile (the same
    // sums per item, bit for bit).
    const int64_t max_item_blocks = (int64_t)(0xffffffffu / kBlock);
    P.persistent = persistent || std::max(blocks_c, blocks_q) > max_item_blocks;
    if (P.persistent) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            return fail(RAD_EDEVICE, "cannot query the compute-unit count");
        auto grid_for = [&](const Tile &t, bool wj, int64_t items, int &gb) -> rad_status {
            int occ = 0;
            hipError_t e = launch_amp(AmpLaunch{}, t.variant, wj, P.mixed, 0, nullptr, &occ);
            if (e != hipSuccess || occ <= 0) return hip_fail(e, "occupancy query");
            gb = (int)std::min<int64_t>(items, (int64_t)occ * cus);
            return RAD_OK;
        };
        if (kinds & RAD_CLASSICAL) {
            rs = grid_for(P.tile_c, false, blocks_c, P.pgrid_c);
            if (rs != RAD_OK) return rs;
        }
        if (quantum) {
            rs = grid_for(P.tile_q, P.lay.comps_q == 3, blocks_q, P.pgrid_q);
            if (rs != RAD_OK) return rs;
        }
    }
    return RAD_OK;
}

// Upload the descriptor region through the grid's pinned staging buffer (async on st).
rad_status plan_upload_async(Plan &P, hipStream_t st)
{
    rad_grid *g = P.g;
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->stage_pending) {
        hipError_t e = hipEventSynchronize(g->stage_done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        g->stage_pending = false;
    }
    if (g->stage_bytes < P.lay.desc_bytes) {
        if (g->stage) (void)hipHostFree(g->stage);
        g->stage = nullptr;
        g->stage_bytes = 0;
        hipError_t e = hipHostMalloc(&g->stage, P.lay.desc_bytes, hipHostMallocDefault);
        if (e != hipSuccess) return fail(RAD_ENOMEM, "pinned staging of %zu bytes", P.lay.desc_bytes);
        g->stage_bytes = P.lay.desc_bytes;
    }
    if (!g->stage_done) {
        hipError_t e = hipEventCreateWithFlags(&g->stage_done, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    std::memcpy(g->stage, P.host.data(), P.lay.desc_bytes);
    hipError_t e = hipMemcpyAsync(P.ws, g->stage, P.lay.desc_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipEventRecord(g->stage_done, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    g->stage_pending = true;
    return RAD_OK;
}

// Kernels only: no host copy, no allocation (capturable).  `profile` brackets the
// amplitude launches with events.
rad_status check_out(const Plan &P, const double *out)
{
    const size_t cube = (size_t)P.g->n_w * P.g->n_x * P.g->n_y;
    return check_dev_range(out, (size_t)P.n_out * P.n_kinds * cube * sizeof(double), "out");
}

// `out` must have passed check_out.
rad_status plan_launch(const Plan &P, double *out, hipStream_t st, bool profile)
{
    const rad_grid *g = P.g;
    char *wsb = P.ws;
    double2 *part_c = (double2 *)(wsb + P.lay.off_part_c);
    double2 *part_q = (double2 *)(wsb + P.lay.off_part_q);
    const int64_t part_c_len = (int64_t)((P.lay.off_part_q - P.lay.off_part_c) / sizeof(double2));
    const int64_t part_q_len = (int64_t)((P.lay.total - P.lay.off_part_q) / sizeof(double2));
    unsigned *counters = (unsigned *)(wsb + P.lay.off_counters);

    AmpLaunch L{};
    L.n_segs = P.n_segs;
    L.items = nullptr;
    L.rec = g->dth != 0.0 ? 1 : 0;
    auto set_tile = [&](const Tile &t, int64_t nb) {
        L.n_blocks = nb;
        L.wg = t.wg;
        L.nt = t.nt;
    };
    if (P.persistent) {
        hipError_t e = launch_reset(counters, 2, st);
        if (e != hipSuccess) return hip_fail(e, "counter reset launch");
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (profile) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
            return fail(RAD_EDEVICE, "hipEventCreate for profiling");
        (void)hipEventRecord(ev0, st);
    }
    if (P.kinds & RAD_CLASSICAL) {
        set_tile(P.tile_c, P.blocks_c);
        L.segs = (const SegDesc *)(wsb + P.lay.off_amp_c);
        L.quantum = 0;
        L.comps = 2;
        L.part = part_c;
        L.part_len = part_c_len;
        L.counter = counters;
        hipError_t e = launch_amp(L, P.tile_c.variant, false, P.mixed, P.persistent ? P.pgrid_c : 0, st, nullptr);
        if (e != hipSuccess) return hip_fail(e, "amplitude kernel launch");
    }
    if (P.quantum) {
        set_tile(P.tile_q, P.blocks_q);
        L.segs = (const SegDesc *)(wsb + P.lay.off_amp_q);
        L.quantum = 1;
        L.comps = P.lay.comps_q;
        L.part = part_q;
        L.part_len = part_q_len;
        L.counter = counters + 1;
        hipError_t e = launch_amp(L, P.tile_q.variant, P.lay.comps_q == 3, P.mixed,
                                  P.persistent ? P.pgrid_q : 0, st, nullptr);
        if (e != hipSuccess) return hip_fail(e, "amplitude kernel launch");
    }
    if (profile) {
        (void)hipEventRecord(ev1, st);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending.emplace_back(ev0, ev1);
    }

    FinLaunch F{};
    F.out_seg_begin = (const int *)(wsb + P.lay.off_begin);
    F.out_seg_list = (const int *)(wsb + P.lay.off_list);
    F.cls = (const SegDesc *)(wsb + P.lay.off_id_c);
    F.qs = (const SegDesc *)(wsb + P.lay.off_id_q);
    F.part_c = part_c;
    F.part_q = part_q;
    F.part_c_len = part_c_len;
    F.part_q_len = part_q_len;
    F.comps_q = P.lay.comps_q;
    F.hw = g->d_hw;
    F.thx = g->d_thx;
    F.thy = g->d_thy;
    F.n_w = g->n_w;
    F.n_x = g->n_x;
    F.n_y = g->n_y;
    F.n_out = P.n_out;
    F.kinds = P.kinds;
    F.n_kinds = P.n_kinds;
    F.one_chunk = P.one_chunk ? 1 : 0;
    F.out = out;
    hipError_t e = launch_fin(F, st);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
    return RAD_OK;
}

bool profiling_on()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}

// Shared driver of rad_classical, rad_quantum and rad_batch.
rad_status run(rad_grid *g, const rad_segment *segs, int n_segs, const int *out_index, int n_out,
               int kinds, rad_precision prec, double *out, void *ws, size_t ws_bytes,
               hipStream_t st)
{
    Plan P;
    rad_status rs = plan_build(g, segs, n_segs, out_index, n_out, kinds, prec, ws, ws_bytes, false, P);
    if (rs != RAD_OK) return rs;
    rs = check_out(P, out);
    if (rs != RAD_OK) return rs;
    rs = plan_upload_async(P, st);
    if (rs != RAD_OK) return rs;
    return plan_launch(P, out, st, profiling_on());
}

}  // namespace

namespace rad {
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st);

// rad_batch on `cap` bytes of the library's fixed device scratch at `scratch`: the time
// chunks are coarsened until the workspace fits, and the descriptors reach the scratch
// as kernel arguments, so nothing is allocated (no pinned staging, no device memory).
rad_status run_in_scratch(const rad_grid *grid, const rad_segment *segs, int n_segs, const int *out_index,
                          int n_out, int kinds, rad_precision prec, double *out, char *scratch, size_t cap,
                          hipStream_t st)
{
    rad_grid *g = const_cast<rad_grid *>(grid);
    if (!scratch) return fail(RAD_EDEVICE, "no fixed scratch on this device");
    Plan P;
    rad_status rs = plan_build(g, segs, n_segs, out_index, n_out, kinds, prec, scratch, cap, false, P, cap);
    if (rs != RAD_OK) return rs;
    rs = check_out(P, out);
    if (rs != RAD_OK) return rs;
    hipError_t e = launch_upload(P.ws, P.host.data(), P.lay.desc_bytes, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    return plan_launch(P, out, st, false);
}
}  // namespace rad

namespace {

// The chunking (and so the size) must not depend on which form or variant runs:
// it is planned with the 4x4 tile count whatever the variant.
size_t workspace_for(const rad_grid *g, const std::vector<int64_t> &ns, int n_out, int kinds, bool bound)
{
    const Tile tile = plan_tile(g, kVar44x2);
    const int64_t cf = chunk_factor(tile, (int64_t)ns.size(), target_blocks());
    int64_t sum = 0;
    for (int64_t n : ns) {
        if (bound) {
            sum += radplan::max_chunks(n, cf);   // the most any n' <= n gets
        } else {
            int32_t c, l;
            plan_chunks(n, cf, c, l);
            sum += c;
        }
    }
    return layout(g, (int)ns.size(), n_out, kinds, sum).total;
}

// Spacing d of a uniform grid (th[j] = th[0] + j d to within a few units in the last
// place of the largest |th|), or 0; 0 also for fewer than two points.
double uniform_step(const std::vector<double> &th)
{
    const size_t n = th.size();
    if (n < 2) return 0.0;
    const double d = (th[n - 1] - th[0]) / (double)(n - 1);
    if (!(d != 0.0)) return 0.0;
    const double tol = 8.0 * std::numeric_limits<double>::epsilon() * std::max(std::fabs(th[0]), std::fabs(th[n - 1]));
    for (size_t j = 0; j < n; ++j)
        if (std::fabs(th[j] - (th[0] + (double)j * d)) > tol) return 0.0;
    return d;
}

// The spacing the phase recurrence uses: thx and thy uniform with the same spacing
// (one axis of a single direction takes the other's), else 0.
double common_step(const std::vector<double> &thx, const std::vector<double> &thy)
{
    const double dx = uniform_step(thx), dy = uniform_step(thy);
    if (thx.size() < 2) return dy;
    if (thy.size() < 2) return dx;
    if (dx == 0.0 || dy == 0.0) return 0.0;
    return std::fabs(dx - dy) <= 8.0 * std::numeric_limits<double>::epsilon() * std::fabs(dx) ? dx : 0.0;
}

std::vector<double> cell_widths(const std::vector<double> &th)
{
    const size_t n = th.size();
    std::vector<double> w(n, 1.0);
    if (n < 2) return w;
    for (size_t i = 1; i + 1 < n; ++i) w[i] = 0.5 * (th[i + 1] - th[i - 1]);
    w[0] = th[1] - th[0];
    w[n - 1] = th[n - 1] - th[n - 2];
    return w;
}

}  // namespace

extern "C" {

const char *rad_status_string(rad_status s)
{
    // a C caller may pass any int: read the bits, since a C++ enum value outside the
    // enumeration's range is undefined behaviour
    int v = 0;
    static_assert(sizeof(rad_status) == sizeof(int), "rad_status is an int");
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
    case RAD_OK: return "ok";
    case RAD_EINVAL: return "invalid argument";
    case RAD_ENOMEM: return "out of memory / workspace too small";
    case RAD_EDEVICE: return "HIP device error";
    case RAD_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *rad_last_error(void) { return g_err.c_str(); }

rad_status rad_setup_grid(const double *hw_eV, int n_w, const double *thx, int n_x, const double *thy,
                          int n_y, void *stream, rad_grid **out)
{
    if (!out) return fail(RAD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!hw_eV || !thx || !thy) return fail(RAD_EINVAL, "grid arrays must not be NULL");
    if (n_w < 1 || n_x < 1 || n_y < 1) return fail(RAD_EINVAL, "grid sizes must be >= 1");
    if ((int64_t)n_w * n_x * n_y > ((int64_t)1 << 31))
        return fail(RAD_EINVAL, "grid of %lld points is too large", (long long)n_w * n_x * n_y);
    for (int i = 0; i < n_w; ++i)
        if (!(std::isfinite(hw_eV[i]) && hw_eV[i] > 0.0)) return fail(RAD_EINVAL, "hw_eV[%d] must be finite and > 0", i);
    for (int i = 0; i < n_x; ++i)
        if (!std::isfinite(thx[i]) || std::fabs(thx[i]) >= 1.0) return fail(RAD_EINVAL, "thx[%d] invalid", i);
    for (int i = 0; i < n_y; ++i)
        if (!std::isfinite(thy[i]) || std::fabs(thy[i]) >= 1.0) return fail(RAD_EINVAL, "thy[%d] invalid", i);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(RAD_EDEVICE, "no HIP device");
    rad_grid *g = new rad_grid();
    g->n_w = n_w;
    g->n_x = n_x;
    g->n_y = n_y;
    g->device = dev;
    g->hw.assign(hw_eV, hw_eV + n_w);
    g->thx.assign(thx, thx + n_x);
    g->thy.assign(thy, thy + n_y);
    g->dth = common_step(g->thx, g->thy);
    std::vector<double> k(n_w);
    for (int i = 0; i < n_w; ++i) k[i] = hw_eV[i] / kHbarC_eVm;
    const std::vector<double> wx = cell_widths(g->thx), wy = cell_widths(g->thy);
    struct { double **dst; const double *src; size_t n; } arrs[] = {
        {&g->d_hw, hw_eV, (size_t)n_w}, {&g->d_k, k.data(), (size_t)n_w},
        {&g->d_thx, thx, (size_t)n_x},  {&g->d_thy, thy, (size_t)n_y},
        {&g->d_wx, wx.data(), (size_t)n_x}, {&g->d_wy, wy.data(), (size_t)n_y}};
    for (auto &a : arrs) {
        hipError_t e = hipMalloc((void **)a.dst, a.n * sizeof(double));
        if (e != hipSuccess) {
            rad_free_grid(g);
            return fail(RAD_ENOMEM, "hipMalloc for the grid: %s", hipGetErrorString(e));
        }
        e = hipMemcpyAsync(*a.dst, a.src, a.n * sizeof(double), hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e != hipSuccess) {
            rad_free_grid(g);
            return hip_fail(e, "grid upload");
        }
    }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) {
        rad_free_grid(g);
        return hip_fail(e, "grid upload");
    }
    // pinned staging for the descriptor uploads of compute calls, allocated here so that
    // a call whose descriptors fit (about 1000 segments) allocates nothing
    e = hipHostMalloc(&g->stage, kInitialStage, hipHostMallocDefault);
    if (e != hipSuccess) {
        g->stage = nullptr;
        rad_free_grid(g);
        return fail(RAD_ENOMEM, "pinned staging of %zu bytes", kInitialStage);
    }
    g->stage_bytes = kInitialStage;
    *out = g;
    return RAD_OK;
}

void rad_free_grid(rad_grid *g)
{
    if (!g) return;
    if (g->stage_pending && g->stage_done) (void)hipEventSynchronize(g->stage_done);
    if (g->stage_done) (void)hipEventDestroy(g->stage_done);
    if (g->stage) (void)hipHostFree(g->stage);
    for (double *p : {g->d_hw, g->d_k, g->d_thx, g->d_thy, g->d_wx, g->d_wy})
        if (p) (void)hipFree(p);
    delete g;
}

rad_status rad_grid_dims(const rad_grid *g, int *n_w, int *n_x, int *n_y)
{
    if (!g) return fail(RAD_EINVAL, "grid is NULL");
    if (n_w) *n_w = g->n_w;
    if (n_x) *n_x = g->n_x;
    if (n_y) *n_y = g->n_y;
    return RAD_OK;
}

rad_status rad_grid_step(const rad_grid *g, double *dth)
{
    if (!g || !dth) return fail(RAD_EINVAL, "grid or dth is NULL");
    *dth = g->dth;
    return RAD_OK;
}

size_t rad_workspace_bytes(const rad_grid *g, int64_t max_n, int kinds, rad_precision prec)
{
    if (!g || max_n < 2 || kinds <= 0 || kinds > 7) return 0;
    if (!valid_prec(prec)) return 0;
    return workspace_for(g, {max_n}, 1, kinds, true);
}

size_t rad_batch_workspace_bytes(const rad_grid *g, const rad_segment *segs, int n_segs, int n_out,
                                 int kinds, rad_precision prec)
{
    if (!g || !segs || n_segs <= 0 || n_out <= 0 || kinds <= 0 || kinds > 7) return 0;
    if (!valid_prec(prec)) return 0;
    std::vector<int64_t> ns(n_segs);
    for (int s = 0; s < n_segs; ++s) {
        if (segs[s].n < 2) return 0;
        ns[s] = segs[s].n;
    }
    return workspace_for(g, ns, n_out, kinds, false);
}

rad_status rad_classical(const rad_grid *g, const rad_segment *seg, rad_precision prec, double *out,
                         void *ws, size_t ws_bytes, void *stream)
{
    const int zero = 0;
    return run(const_cast<rad_grid *>(g), seg, 1, &zero, 1, RAD_CLASSICAL, prec, out, ws, ws_bytes,
               (hipStream_t)stream);
}

rad_status rad_quantum(const rad_grid *g, const rad_segment *seg, int kinds, rad_precision prec,
                       double *out, void *ws, size_t ws_bytes, void *stream)
{
    if (kinds <= 0 || (kinds & ~(RAD_SPIN0 | RAD_SPINHALF)))
        return fail(RAD_EINVAL, "rad_quantum kinds must be a non-empty subset of RAD_SPIN0|RAD_SPINHALF");
    const int zero = 0;
    return run(const_cast<rad_grid *>(g), seg, 1, &zero, 1, kinds, prec, out, ws, ws_bytes,
               (hipStream_t)stream);
}

rad_status rad_batch(const rad_grid *g, const rad_segment *segs, int n_segs, const int *out_index,
                     int n_out, int kinds, rad_precision prec, double *out, void *ws, size_t ws_bytes,
                     void *stream)
{
    return run(const_cast<rad_grid *>(g), segs, n_segs, out_index, n_out, kinds, prec, out, ws,
               ws_bytes, (hipStream_t)stream);
}

rad_status rad_phase_factors(const double *turns, int64_t n, rad_precision prec, double *c, double *s,
                             void *stream)
{
    if (!valid_prec(prec)) return fail(RAD_EINVAL, "unknown precision %d", prec_value(prec));
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(RAD_EINVAL, "n = %lld outside [0, 2^40]", (long long)n);
    if (n == 0) return RAD_OK;
    const size_t bytes = (size_t)n * sizeof(double);
    rad_status rs = check_dev_range(turns, bytes, "turns");
    if (rs == RAD_OK) rs = check_dev_range(c, bytes, "c");
    if (rs == RAD_OK) rs = check_dev_range(s, bytes, "s");
    if (rs != RAD_OK) return rs;
    hipError_t e = launch_phase(turns, n, prec == RAD_MIXED ? 1 : 0, c, s, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phase kernel launch");
    return RAD_OK;
}

rad_status rad_angle_integrate(const rad_grid *g, const double *cube, int n_cubes, double *dIdw,
                               void *stream)
{
    rad_status rs = check_grid(g);
    if (rs != RAD_OK) return rs;
    if (n_cubes <= 0) return fail(RAD_EINVAL, "n_cubes must be > 0");
    const size_t cb = (size_t)g->n_w * g->n_x * g->n_y * sizeof(double);
    rs = check_dev_range(cube, cb * n_cubes, "cube");
    if (rs != RAD_OK) return rs;
    rs = check_dev_range(dIdw, (size_t)n_cubes * g->n_w * sizeof(double), "dIdw");
    if (rs != RAD_OK) return rs;
    hipError_t e = launch_angle(cube, g->d_wx, g->d_wy, g->n_x, g->n_y, g->n_w, n_cubes, dIdw,
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "angle kernel launch");
    return RAD_OK;
}

}  // extern "C"

namespace rad_err {
void set(const char *msg) { g_err = msg; }
}  // namespace rad_err

bool rad_grid_view(const rad_grid *g, rad::GridView *v)
{
    if (!g || !v) return false;
    *v = rad::GridView{g->d_hw, g->d_k, g->d_thx, g->d_thy, g->d_wx, g->d_wy, g->n_w, g->n_x, g->n_y, g->device};
    return true;
}

extern "C" {

struct rad_plan {
    Plan P;
    hipGraphExec_t gexec = nullptr;
    double *g_out = nullptr;
};

rad_status rad_plan_create(const rad_grid *g, const rad_segment *segs, int n_segs, const int *out_index,
                           int n_out, int kinds, rad_precision prec, void *ws, size_t ws_bytes,
                           void *stream, rad_plan **out)
{
    if (!out) return fail(RAD_EINVAL, "out is NULL");
    *out = nullptr;
    rad_plan *p = new rad_plan();
    rad_status rs = plan_build(const_cast<rad_grid *>(g), segs, n_segs, out_index, n_out, kinds, prec,
                               ws, ws_bytes, true, p->P);
    if (rs != RAD_OK) {
        delete p;
        return rs;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(p->P.ws, p->P.host.data(), p->P.lay.desc_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "plan upload");
    }
    *out = p;
    return RAD_OK;
}

rad_status rad_plan_launch(rad_plan *p, double *out, void *stream)
{
    if (!p) return fail(RAD_EINVAL, "plan is NULL");
    rad_status rs = check_grid(p->P.g);
    if (rs != RAD_OK) return rs;
    rs = check_out(p->P, out);
    if (rs != RAD_OK) return rs;
    return plan_launch(p->P, out, (hipStream_t)stream, profiling_on());
}

rad_status rad_plan_launch_graph(rad_plan *p, double *out, void *stream)
{
    if (!p) return fail(RAD_EINVAL, "plan is NULL");
    if (!stream) return fail(RAD_EINVAL, "graph capture needs a created stream, not the default stream");
    rad_status rs = check_grid(p->P.g);
    if (rs != RAD_OK) return rs;
    rs = check_out(p->P, out);
    if (rs != RAD_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    if (!p->gexec || p->g_out != out) {
        if (p->gexec) {
            (void)hipGraphExecDestroy(p->gexec);
            p->gexec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        rs = plan_launch(p->P, out, st, false);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(st, &graph);
        if (rs != RAD_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rs;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            p->gexec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        p->g_out = out;
    }
    const bool prof = profiling_on();
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof) {
        if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
            return fail(RAD_EDEVICE, "hipEventCreate for profiling");
        (void)hipEventRecord(ev0, st);
    }
    hipError_t e = hipGraphLaunch(p->gexec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (prof) {
        (void)hipEventRecord(ev1, st);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_pending.emplace_back(ev0, ev1);
    }
    return RAD_OK;
}

void rad_plan_free(rad_plan *p)
{
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    delete p;
}

}  // extern "C"

// ---------------------------------------------------------------- cell refinement
namespace {

struct CellsPlan {
    int n_segs = 0, ncx = 0, ncy = 0, n_cells = 0, n_wb = 0;
    int n_ps = 0;                 // active (segment, cell) pseudo-segments
    int64_t n_items = 0;
    bool dense = false;           // device mask: every (segment, cell) pair, p = s * n_cells + c
    // waves over photon energies (the launch's wg; 0: grouped, each item carries its own)
    // and direction-tile groups per cell
    int wg = 1, n_groups = 1;
    bool grouped = false;
    size_t off_ps, off_items, off_psof, off_mask, off_part, desc_bytes, total;
    size_t off_flags = 0, off_live = 0, off_nlive = 0;   // device-mask compaction (dense plans)
    size_t off_grouped = 0;                               // its regrouped items (grouped form)
    std::vector<char> host;
};

// Cell items: a block spreads its 4 waves over wg groups of 64 photon energies and
// 4 / wg of the cell's four 4 x 4 direction tiles (wg = 1: the whole 8 x 8 cell for 64
// energies).  0, the default, groups: the selected 64-energy blocks of a (segment, cell,
// time chunk) are taken by four (wg = 4, one tile per item), then two, then one, so that a
// staged direction serves up to 256 energies while a cell is still evaluated only for the
// blocks that have a selected energy.
int g_cell_wg = 0;

int cell_wg()
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    return g_cell_wg;
}

// The work of rad_cells for a host mask (only the selected (segment, cell, photon-energy
// block) items), or, with mask == nullptr and dense set, for a device mask read by the
// kernels themselves: every (segment, cell) pair and every block, items of unselected
// blocks leaving at once.
rad_status cells_plan(const rad_grid *g, const rad_segment *segs, int n_segs, int kind, int cx, int cy,
                      const uint8_t *mask, bool fill, CellsPlan &C, int comps, bool dense = false)
{
    if (!g) return fail(RAD_EINVAL, "grid is NULL");
    if (!segs || n_segs <= 0) return fail(RAD_EINVAL, "no segments");
    if (!mask && !dense) return fail(RAD_EINVAL, "mask is NULL");
    C.dense = dense;
    if (kind != RAD_CLASSICAL && kind != RAD_SPIN0 && kind != RAD_SPINHALF)
        return fail(RAD_EINVAL, "kind must be exactly one of RAD_CLASSICAL, RAD_SPIN0, RAD_SPINHALF");
    if (cx != 8 || cy != 8) return fail(RAD_EUNSUPPORTED, "cells of %d x %d directions (8 x 8 supported)", cx, cy);
    if (g->n_x % cx || g->n_y % cy) return fail(RAD_EINVAL, "the grid (%d x %d) is not a whole number of cells", g->n_x, g->n_y);
    C.n_segs = n_segs;
    C.ncx = g->n_x / cx;
    C.ncy = g->n_y / cy;
    C.n_cells = C.ncx * C.ncy;
    C.wg = cell_wg();
    // the grouped form plans as wg = 1 (one item per selected block and tile group of the
    // whole cell); its block indices travel as bytes, so past 256 blocks it is wg = 1
    C.grouped = C.wg == 0 && (g->n_w + kWave - 1) / kWave <= 256;
    if (C.wg == 0 && !C.grouped) C.wg = 1;
    const int wgp = C.grouped ? 1 : C.wg;
    C.n_groups = ((cx / 4) * (cy / 4)) / (kWavesPerBlock / wgp);
    C.n_wb = (g->n_w + kWave * wgp - 1) / (kWave * wgp);
    const int n_w = g->n_w;
    // active (segment, cell) pairs and their photon-energy blocks
    std::vector<int> psof((size_t)n_segs * C.n_cells, -1);
    std::vector<std::vector<int>> wbs;
    std::vector<std::pair<int, int>> ps;   // (segment, cell)
    for (int s = 0; s < n_segs; ++s)
        for (int c = 0; c < C.n_cells; ++c) {
            std::vector<int> blocks;
            for (int b = 0; b < C.n_wb; ++b) {
                bool any = dense;
                for (int w = b * kWave * wgp; w < std::min(n_w, (b + 1) * kWave * wgp) && !any; ++w)
                    any = mask[((size_t)s * n_w + w) * C.n_cells + c] != 0;
                if (any) blocks.push_back(b);
            }
            if (!blocks.empty()) {
                psof[(size_t)s * C.n_cells + c] = (int)ps.size();
                ps.emplace_back(s, c);
                wbs.push_back(blocks);
            }
        }
    C.n_ps = (int)ps.size();
    int64_t items = 0;
    for (auto &v : wbs) items += (int64_t)v.size() * C.n_groups;
    // time chunks: enough items to fill the GPU
    const int64_t cf = items >= kTargetBlocks ? 1 : (kTargetBlocks + std::max<int64_t>(items, 1) - 1) / std::max<int64_t>(items, 1);
    std::vector<int32_t> nch(std::max(C.n_ps, 1)), clen(std::max(C.n_ps, 1));
    int64_t sum_chunks = 0;
    for (int p = 0; p < C.n_ps; ++p) {
        plan_chunks(segs[ps[p].first].n, cf, nch[p], clen[p]);
        sum_chunks += nch[p];
        items += (int64_t)(nch[p] - 1) * (int64_t)wbs[p].size() * C.n_groups;
    }
    C.n_items = items;
    const size_t cell_dirs = (size_t)cx * cy;
    size_t o = 0;
    C.off_ps = o; o = align_up(o + sizeof(SegDesc) * (size_t)std::max(C.n_ps, 1));
    C.off_items = o; o = align_up(o + sizeof(int4) * (size_t)std::max<int64_t>(items, 1));
    C.off_psof = o; o = align_up(o + sizeof(int) * psof.size());
    C.off_mask = o; o = align_up(o + (dense ? 0 : (size_t)n_segs * n_w * C.n_cells));
    C.desc_bytes = o;
    if (dense) {   // written by the compaction kernels, not uploaded
        C.off_flags = o; o = align_up(o + sizeof(int) * (size_t)std::max<int64_t>(items, 1));
        C.off_live = o; o = align_up(o + sizeof(int4) * (size_t)std::max<int64_t>(items, 1));
        C.off_nlive = o; o = align_up(o + sizeof(int));
        if (C.grouped) {
            C.off_grouped = o;
            o = align_up(o + sizeof(int4) * (size_t)std::max<int64_t>(items, 1));
        }
    }
    C.off_part = o;
    o = align_up(o + (size_t)sum_chunks * comps * cell_dirs * n_w * sizeof(double2));
    C.total = o;
    if (!fill) return RAD_OK;
    // descriptors
    C.host.assign(C.desc_bytes, 0);
    SegDesc *D = (SegDesc *)(C.host.data() + C.off_ps);
    int4 *I = (int4 *)(C.host.data() + C.off_items);
    std::memcpy(C.host.data() + C.off_psof, psof.data(), sizeof(int) * psof.size());
    if (!dense) std::memcpy(C.host.data() + C.off_mask, mask, (size_t)n_segs * n_w * C.n_cells);
    // launch order: longest segment first
    std::vector<int> order(C.n_ps);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return segs[ps[a].first].n > segs[ps[b].first].n; });
    int64_t part = 0, it = 0;
    for (int p = 0; p < C.n_ps; ++p) {
        const rad_segment &sg = segs[ps[p].first];
        const int c = ps[p].second, ci = c % C.ncx, cj = c / C.ncx;
        SegDesc d{};
        const double *cols[C_NCOL] = {sg.t, sg.x, sg.y, sg.dz, sg.vx, sg.vy, sg.dvz, sg.ax, sg.ay, sg.az};
        for (int k = 0; k < C_NCOL; ++k) d.col[k] = cols[k];
        d.w = sg.w;
        d.n = sg.n;
        d.gamma = sg.gamma;
        d.c0 = 1.0 / (2.0 * sg.gamma * sg.gamma);
        d.energy = sg.energy_eV;
        d.n_chunks = nch[p];
        d.chunk_len = clen[p];
        d.part_off = part;
        part += (int64_t)nch[p] * comps * (int64_t)cell_dirs * n_w;
        d.block_begin = 0;
        d.hw = g->d_hw;
        d.k = g->d_k;
        d.thx = g->d_thx + (size_t)ci * cx;
        d.thy = g->d_thy + (size_t)cj * cy;
        d.dth = g->dth;
        d.n_w = n_w;
        d.n_x = cx;
        d.n_y = cy;
        d.n_tx = cx / 4;
        d.n_ty = cy / 4;
        d.n_groups = C.n_groups;
        d.n_wblocks = C.n_wb;
        D[p] = d;
    }
    for (int r = 0; r < C.n_ps; ++r) {
        const int p = order[r];
        const std::vector<int> &v = wbs[p];
        for (int ch = 0; ch < nch[p]; ++ch) {
            if (C.grouped && !dense) {
                // k blocks -> k items: tile group g in bits 0..7, k in bits 8..15, the
                // blocks one byte each (the device mask's compaction groups the same way)
                size_t q = 0;
                auto put = [&](int k) {
                    uint32_t packed = 0;
                    for (int u = 0; u < k; ++u) packed |= (uint32_t)v[q + u] << (8 * u);
                    for (int g = 0; g < k; ++g) I[it++] = make_int4(p, ch, g | (k << 8), (int)packed);
                    q += k;
                };
                while (v.size() - q >= 4) put(4);
                if (v.size() - q >= 2) put(2);
                if (v.size() - q == 1) put(1);
            } else {
                for (int grp = 0; grp < C.n_groups; ++grp)
                    for (int b : v) I[it++] = make_int4(p, ch, grp, b);
            }
        }
    }
    return RAD_OK;
}

// rad_cells (host mask) and rad_cells_device (device mask, dense plan).
rad_status cells_run(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind, rad_precision prec,
                     int cx, int cy, const uint8_t *mask, bool dev_mask, double *cell_out, void *ws,
                     size_t ws_bytes, void *stream)
{
    rad_grid *g = const_cast<rad_grid *>(grid);
    rad_status rs = check_grid(g);
    if (rs != RAD_OK) return rs;
    if (!valid_prec(prec)) return fail(RAD_EINVAL, "unknown precision %d", prec_value(prec));
    const bool quantum = kind != RAD_CLASSICAL;
    for (int s = 0; s < n_segs && segs; ++s) {
        rs = check_segment(&segs[s], s, quantum);
        if (rs != RAD_OK) return rs;
    }
    const int comps = kind == RAD_SPINHALF ? 3 : 2;
    CellsPlan C;
    if (dev_mask && !mask) return fail(RAD_EINVAL, "mask is NULL");
    rs = cells_plan(g, segs, n_segs, kind, cx, cy, dev_mask ? nullptr : mask, true, C, comps, dev_mask);
    if (rs != RAD_OK) return rs;
    // one block per item, at most 2^32 - 1 work-items (the partial amplitudes of that many
    // items, 128 kB each, would not fit in device memory anyway)
    if (C.n_items > (int64_t)(0xffffffffu / kBlock))
        return fail(RAD_EUNSUPPORTED, "cell launch of %lld blocks", (long long)C.n_items);
    if (dev_mask) {
        rs = check_dev_range(mask, (size_t)n_segs * g->n_w * C.n_cells, "mask");
        if (rs != RAD_OK) return rs;
    }
    if (!ws) return fail(RAD_EINVAL, "workspace is NULL");
    if (ws_bytes < C.total) return fail(RAD_ENOMEM, "workspace of %zu bytes, need %zu", ws_bytes, C.total);
    rs = check_dev_range(ws, C.total, "workspace");
    if (rs != RAD_OK) return rs;
    rs = check_dev_range(cell_out, (size_t)n_segs * g->n_w * C.n_cells * sizeof(double), "cell_out");
    if (rs != RAD_OK) return rs;
    hipStream_t st = (hipStream_t)stream;
    Plan P;      // only for the staging upload
    P.g = g;
    P.ws = (char *)ws;
    P.lay.desc_bytes = C.desc_bytes;
    P.host.swap(C.host);
    rs = plan_upload_async(P, st);
    if (rs != RAD_OK) return rs;
    char *wsb = (char *)ws;
    double2 *part = (double2 *)(wsb + C.off_part);
    if (C.n_items > 0) {
        AmpLaunch L{};
        L.segs = (const SegDesc *)(wsb + C.off_ps);
        L.items = (const int4 *)(wsb + C.off_items);
        L.n_segs = C.n_ps;
        L.n_blocks = C.n_items;
        L.wg = C.grouped ? 0 : C.wg;
        L.nt = C.grouped ? kWavesPerBlock : kWavesPerBlock / C.wg;
        L.quantum = quantum ? 1 : 0;
        L.rec = g->dth != 0.0 ? 1 : 0;
        L.comps = comps;
        L.part = part;
        L.part_len = (int64_t)((C.total - C.off_part) / sizeof(double2));
        L.counter = nullptr;
        if (dev_mask) {
            // the items whose block has a mask bit set, compacted to the front in launch
            // order; the launch keeps every item's block and the rest return at once
            CellCompact K{};
            K.items = L.items;
            K.n_items = C.n_items;
            K.mask = mask;
            K.n_cells = C.n_cells;
            K.n_w = g->n_w;
            K.wg = C.grouped ? 0 : C.wg;
            K.n_wb = C.n_wb;
            K.grouped = C.grouped ? (int4 *)(wsb + C.off_grouped) : nullptr;
            K.flags = (int *)(wsb + C.off_flags);
            K.live = (int4 *)(wsb + C.off_live);
            K.n_live = (int *)(wsb + C.off_nlive);
            hipError_t ec = launch_cell_compact(K, st);
            if (ec != hipSuccess) return hip_fail(ec, "cell compaction launch");
            L.items = K.live;
            L.n_live = K.n_live;
        }
        const bool mixed = prec == RAD_MIXED;
        const bool prof = profiling_on();
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (prof) {
            if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess)
                return fail(RAD_EDEVICE, "hipEventCreate for profiling");
            (void)hipEventRecord(ev0, st);
        }
        hipError_t e = launch_amp(L, kVar44x2, comps == 3, mixed, 0, st, nullptr);
        if (e != hipSuccess) return hip_fail(e, "amplitude kernel launch");
        if (prof) {
            (void)hipEventRecord(ev1, st);
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof_pending.emplace_back(ev0, ev1);
        }
    }
    CellsFin F{};
    F.segs = (const SegDesc *)(wsb + C.off_ps);
    F.psof = (const int *)(wsb + C.off_psof);
    F.mask = dev_mask ? mask : (const uint8_t *)(wsb + C.off_mask);
    F.part = part;
    F.part_len = (int64_t)((C.total - C.off_part) / sizeof(double2));
    F.comps = comps;
    F.kind = kind;
    F.wx = g->d_wx;
    F.wy = g->d_wy;
    F.hw = g->d_hw;
    F.n_segs = n_segs;
    F.n_w = g->n_w;
    F.n_x = g->n_x;
    F.ncx = C.ncx;
    F.n_cells = C.n_cells;
    F.cx = cx;
    F.cy = cy;
    F.out = cell_out;
    hipError_t e = launch_cells_fin(F, st);
    if (e != hipSuccess) return hip_fail(e, "cell finalize launch");
    return RAD_OK;
}

}  // namespace

extern "C" {

size_t rad_cells_workspace_bytes(const rad_grid *g, const rad_segment *segs, int n_segs, int kind,
                                 rad_precision prec, int cx, int cy, const uint8_t *mask)
{
    if (!valid_prec(prec)) return 0;
    CellsPlan C;
    if (cells_plan(g, segs, n_segs, kind, cx, cy, mask, false, C, kind == RAD_SPINHALF ? 3 : 2) != RAD_OK)
        return 0;
    return C.total;
}

rad_status rad_cells(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                     rad_precision prec, int cx, int cy, const uint8_t *mask, double *cell_out,
                     void *ws, size_t ws_bytes, void *stream)
{
    return cells_run(grid, segs, n_segs, kind, prec, cx, cy, mask, false, cell_out, ws, ws_bytes, stream);
}

size_t rad_cells_device_workspace_bytes(const rad_grid *g, const rad_segment *segs, int n_segs, int kind,
                                        rad_precision prec, int cx, int cy)
{
    if (!valid_prec(prec)) return 0;
    CellsPlan C;
    if (cells_plan(g, segs, n_segs, kind, cx, cy, nullptr, false, C, kind == RAD_SPINHALF ? 3 : 2, true) != RAD_OK)
        return 0;
    return C.total;
}

rad_status rad_cells_device(const rad_grid *grid, const rad_segment *segs, int n_segs, int kind,
                            rad_precision prec, int cx, int cy, const uint8_t *mask, double *cell_out,
                            void *ws, size_t ws_bytes, void *stream)
{
    return cells_run(grid, segs, n_segs, kind, prec, cx, cy, mask, true, cell_out, ws, ws_bytes, stream);
}

}  // extern "C"

extern "C" {
rad_status rad_tune_set_variant(int persistent, int mixed, int with_j, int variant)
{
    if (variant < 0 || variant >= kNumVariants) return fail(RAD_EINVAL, "variant %d unknown", variant);
    if (with_j && !kVarJ[variant])
        return fail(RAD_EUNSUPPORTED, "variant %d (%dx%d tile) serves only integral sets without J", variant,
                    kVarTX[variant], kVarTY[variant]);
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_variant[persistent ? 1 : 0][mixed ? 1 : 0][with_j ? 1 : 0] = variant;
    return RAD_OK;
}

rad_status rad_tune_get_variant(int persistent, int mixed, int with_j, int *variant)
{
    if (!variant) return fail(RAD_EINVAL, "variant is NULL");
    *variant = variant_for(persistent != 0, mixed != 0, with_j != 0);
    return RAD_OK;
}

int rad_tune_num_variants(void) { return kNumVariants; }

rad_status rad_tune_set_shape(int persistent, int mixed, int wg)
{
    if (wg != 0 && wg != 1 && wg != 2 && wg != 4) return fail(RAD_EINVAL, "wg %d: 0 (by the grid), 1, 2 or 4", wg);
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_wg[persistent ? 1 : 0][mixed ? 1 : 0] = wg;
    return RAD_OK;
}

rad_status rad_tune_get_shape(int persistent, int mixed, int *wg)
{
    if (!wg) return fail(RAD_EINVAL, "wg is NULL");
    *wg = wg_for(persistent != 0, mixed != 0);
    return RAD_OK;
}

rad_status rad_tune_set_chunk_target(int64_t target_blocks)
{
    if (target_blocks < 0 || target_blocks > radplan::kMaxTargetBlocks)
        return fail(RAD_EINVAL, "chunk target %lld outside [0, 2^24]", (long long)target_blocks);
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_target = target_blocks;
    return RAD_OK;
}

int64_t rad_tune_get_chunk_target(void) { return target_blocks(); }

rad_status rad_tune_set_cell_spread(int wg)
{
    if (wg != 0 && wg != 1 && wg != 2 && wg != 4) return fail(RAD_EINVAL, "wg %d: 0 (default), 1, 2 or 4", wg);
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_cell_wg = wg;
    return RAD_OK;
}

int rad_tune_get_cell_spread(void) { return cell_wg(); }

rad_status rad_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return RAD_OK;
}

rad_status rad_profile_read(double *kernel_ms, int64_t *launches, int reset)
{
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending);
    }
    double ms = 0.0;
    for (auto &pr : pend) {
        float m = 0.0f;
        hipError_t e = hipEventSynchronize(pr.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&m, pr.first, pr.second);
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
        if (e != hipSuccess) return hip_fail(e, "profiling events");
        ms += m;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_ms += ms;
    g_prof_launches += (int64_t)pend.size();
    if (kernel_ms) *kernel_ms = g_prof_ms;
    if (launches) *launches = g_prof_launches;
    if (reset) {
        g_prof_ms = 0.0;
        g_prof_launches = 0;
    }
    return RAD_OK;
}

}  // extern "C"

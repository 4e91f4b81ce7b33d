// Radiation-integral kernels for gfx950 (CDNA4).
//
// amp_kernel   : complex amplitudes A_x, A_y (and J) of one time chunk of a
//                segment for 64*wg photon energies x nt direction tiles.
// fin_kernel   : fixed-order sum over chunks and segments, |A|^2, the
//                classical / spin-0 / spin-1/2 weights, written to the cube.
// angle_kernel : dI/d hw, the weighted sum of each cube row over directions.
//
// Method (Nielsen, arXiv:1910.10391, Sec. II): for every photon energy and
// direction n = (thx, thy), sum over time samples
//     A += w f(t, n) exp(i kappa psi(t, n)),   J += w Q(t, n) exp(i kappa psi(t, n)),
// with the small-angle expansion of Sec. II:
//     D   = 1/(2g^2) + th^2/2 - dvz - thx vx - thy vy,   G = w / D^2,
//     C   = 1/(2g^2) - th^2/2 - dvz,
//     f_x = [(az + thy ay)(thx - vx) - (thy (thy - vy) + C) ax] G,
//     f_y = [(az + thx ax)(thy - vy) - (thx (thx - vx) + C) ay] G,
//     Q   = (thx ax + thy ay + az) G,
//     psi = (1/(2g^2) + th^2/2) t - dz - thx x - thy y.
// f_z is not accumulated: thx f_x + thy f_y + f_z = 0 identically, so
// A_z = -(thx A_x + thy A_y) is formed in fin_kernel.
//
// Work decomposition (one block = 4 waves = 256 lanes):
//   * a lane owns one photon energy (kappa in a register) and a TX x TY tile of
//     directions, with TX*TY complex accumulators per component in VGPRs;
//   * the integrand f, Q (shared by every photon energy) and the two parts of
//     the phase are computed once per (time step, direction) by the whole
//     block into LDS, then read by each wave as a broadcast (one address);
//   * the phase separates, psi = Px(t, thx) + Py(t, thy) with
//     Px = 1/(2g^2) t - dz + thx (thx t/2 - x), Py = thy (thy t/2 - y).  The
//     tile's first row is folded into the x part: with X_jx = exp(i kappa (Px_jx
//     + Py_0)) and Y_jy = exp(i kappa (Py_jy - Py_0)), exp(i kappa psi) = X_jx Y_jy
//     and Y_0 = 1, so a lane evaluates TX + TY - 1 phase factors per time step and
//     forms the other factors with (TY - 1) TX complex products; on a uniform grid
//     (REC) Px and Py are quadratic in the direction index and the FP64 form gets
//     a tile's factors from 4 evaluated ones by recurrence;
//   * a long segment is cut into time chunks whose FP64 partial amplitudes are
//     summed in a fixed order by fin_kernel.
#include <hip/hip_runtime.h>

#include "rad_internal.h"
#include "rad_math.h"

namespace rad {

// Index checks of the debug build (-DRAD_DEBUG=1): descriptor, chunk and partial-amplitude
// indices are checked against the launch's bounds; a violation is counted (read with
// rad_debug_violations) and the access skipped.  The release build compiles them away.
#ifndef RAD_DEBUG
#define RAD_DEBUG 0
#endif
#if RAD_DEBUG
__device__ unsigned long long g_debug_violations = 0;
__device__ __forceinline__ bool debug_ok(bool cond)
{
    if (!cond) atomicAdd(&g_debug_violations, 1ull);
    return cond;
}
#define RAD_DEBUG_OK(cond) debug_ok(cond)
#else
#define RAD_DEBUG_OK(cond) true
#endif

// A wave-uniform 64-bit value taken into scalar registers (readfirstlane of both halves).
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Phase factor of a lane: FP64 polynomial on half turns, or FP32 hardware
// sin/cos on revolutions (mixed precision).  `kh` is kappa/pi (FP64 form) or
// kappa/(2 pi) (mixed form).
template <bool MIXED>
__device__ __forceinline__ void lane_cis(double kh, double part, double &c, double &s)
{
    if constexpr (MIXED) {
        float cf, sf;
        cis_revolutions_f32(kh * part, cf, sf);
        c = (double)cf;
        s = (double)sf;
    } else {
        cis_halfturns(kh * part, c, s);
    }
}

// LDS of one work item: the staged integrand and phase parts of kSlots (time
// step, direction tile) pairs, the angles of the item's direction tiles and, in the
// mixed form, the trajectory columns of the pass's time steps (the ten columns and the
// weight).
constexpr int kRowCols = C_NCOL + 1;   // + the quadrature weight
// One staged (time step, direction tile) slot: the integrand of the tile's directions and the
// phase parts.  Kept together, so that a time step's reads in the hot loop all sit at fixed
// offsets from one address, which advances once per step.
template <int TX, int TY, bool WITHJ>
struct AmpSlot {
    double2 fxy[TX * TY];
    double fq[WITHJ ? TX * TY : 1];
    double px[TX];
    double py[TY];
};
template <int TX, int TY, bool WITHJ, bool ROWS>
struct AmpSmem {
    double row[ROWS ? kRowCols : 1][ROWS ? kSlots : 1];
    // the block's direction tiles, thx then thy (0 outside), and which exist
    double th[kWavesPerBlock][TX + TY];
    unsigned char thok[kWavesPerBlock][TX + TY];
    AmpSlot<TX, TY, WITHJ> slot[kSlots];
    int seg;
};

// One work item b = (segment, time chunk, direction-tile group, photon-energy
// block) of an amplitude launch, computed by the whole block.
// CELLS: the one-block-per-item launches, which serve the cell refinement's device
// mask; the persistent form never does, and leaves the check out of its code.
template <int TX, int TY, bool WITHJ, bool MIXED, bool REC, bool CELLS = true>
__device__ __forceinline__ void amp_item(const AmpLaunch &L, int64_t b, AmpSmem<TX, TY, WITHJ, MIXED> &sm)
{
    constexpr int NP = TX * TY;
    AmpSlot<TX, TY, WITHJ> *const s_slot = sm.slot;

    // cell refinement with a device mask: the live items were compacted to the front
    // of the list, and the blocks past them leave at once
    if (CELLS && L.n_live && b >= (int64_t)__builtin_amdgcn_readfirstlane(*L.n_live)) return;
    // segment and coordinates of this item: from the explicit list, or the
    // last segment s with block_begin <= b
    int chunk = 0, grp = 0, wb = 0;
    if (threadIdx.x == 0) {
        int lo;
        if (L.items) {
            lo = L.items[b].x;
        } else {
            lo = 0;
            int hi = L.n_segs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.segs[mid].block_begin <= b) lo = mid; else hi = mid - 1;
            }
        }
        sm.seg = lo;
    }
    __syncthreads();
    // wave-uniform: descriptor fields then live in SGPRs (scalar loads), not VGPRs
    int s_seg = __builtin_amdgcn_readfirstlane(sm.seg);
    if (!RAD_DEBUG_OK(s_seg >= 0 && s_seg < L.n_segs)) s_seg = 0;
    const SegDesc &S = L.segs[s_seg];
    const int64_t n = S.n;
    const double c0 = S.c0;
    const double energy = S.energy;
    const double *__restrict__ ct = S.col[C_T];
    const double *__restrict__ cw = S.w;
    const double *__restrict__ g_hw = S.hw;
    const double *__restrict__ g_k = S.k;
    const double *__restrict__ g_thx = S.thx;
    const double *__restrict__ g_thy = S.thy;
    const int n_w = S.n_w, n_x = S.n_x, n_y = S.n_y, n_tx = S.n_tx;

    if (L.items) {
        const int4 it = L.items[b];
        chunk = __builtin_amdgcn_readfirstlane(it.y);
        grp = __builtin_amdgcn_readfirstlane(it.z);
        wb = __builtin_amdgcn_readfirstlane(it.w);
    } else {
        // 64-bit divisions expand into vector instructions: their results are taken back
        // into scalar registers, so that the time loop's bounds and counter stay scalar
        // (in vector registers they took four of them and were spilled in every pass)
        int64_t local = b - S.block_begin;
        wb = __builtin_amdgcn_readfirstlane((int)(local % S.n_wblocks));
        local /= S.n_wblocks;
        grp = __builtin_amdgcn_readfirstlane((int)(local % S.n_groups));
        chunk = __builtin_amdgcn_readfirstlane((int)(local / S.n_groups));
    }
    const int64_t k_begin = uniform64((int64_t)chunk * S.chunk_len);
    int64_t k_end = uniform64(min(n, k_begin + (int64_t)S.chunk_len));
    if (!RAD_DEBUG_OK(chunk >= 0 && chunk < S.n_chunks && k_begin < n)) k_end = k_begin;

    int nt = L.nt, wg = L.wg;
    // grouped cell items (a launch with wg = 0) carry their own shape: the item's waves
    // over photon energies in bits 8..15 of its tile-group field, and its wg 64-energy
    // blocks (not necessarily adjacent) one byte per wave in the block field
    const bool grouped = CELLS && wg == 0;
    if (grouped) {
        wg = grp >> 8;
        grp &= 0xff;
        if (!(wg == 1 || wg == 2 || wg == 4)) {   // leaves before any barrier of the item
            (void)RAD_DEBUG_OK(false);
            return;
        }
        nt = kWavesPerBlock / wg;
    }
    const int lnt = nt == 4 ? 2 : (nt == 2 ? 1 : 0);   // nt is 1, 2 or 4 (checked at launch)
    const int T = kSlots / nt;
    const int n_tiles = n_tx * S.n_ty;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int tl = wave / wg;
    const int wblock = grouped ? (int)(((unsigned)wb >> (8 * (wave % wg))) & 0xffu) : wb * wg + wave % wg;
    const int iw = wblock * kWave + lane;
    const int gtile = grp * nt + tl;

    double kappa = 0.0;
    if (iw < n_w) {
        const double k = g_k[iw];
        if (!L.quantum) {
            kappa = k;
        } else {
            const double hw = g_hw[iw];
            kappa = hw < energy ? k * energy / (energy - hw) : 0.0;
        }
    }
    const double kh = MIXED ? kappa * (0.5 / kPi) : kappa * (1.0 / kPi);

    // the angles of the block's nt direction tiles, once per item: the staging loops then
    // read them instead of dividing by the grid's tile count for every staged value (in
    // the FP64 form that index arithmetic had been about half of a staged value's
    // instructions); the first barrier of the time loop orders these writes before any read
    for (int i = threadIdx.x; i < nt * (TX + TY); i += kBlock) {
        const int tile = i / (TX + TY), j = i % (TX + TY);
        const int gt = grp * nt + tile;
        double th = 0.0;
        bool ok = false;
        if (gt < n_tiles) {
            if (j < TX) {
                const int jx = (gt % n_tx) * TX + j;
                ok = jx < n_x;
                if (ok) th = g_thx[jx];
            } else {
                const int jy = (gt / n_tx) * TY + (j - TX);
                ok = jy < n_y;
                if (ok) th = g_thy[jy];
            }
        }
        sm.th[tile][j] = th;
        sm.thok[tile][j] = ok ? 1 : 0;
    }
    // direction j (thx for j < TX, else thy) of tile `tile`: its angle (0 outside the
    // grid) and whether it exists
    auto direction = [&](int tile, int j, double &th) -> bool {
        th = sm.th[tile][j];
        return sm.thok[tile][j] != 0;
    };

    double axr[NP], axi[NP], ayr[NP], ayi[NP], jr[WITHJ ? NP : 1], ji[WITHJ ? NP : 1];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        axr[p] = axi[p] = ayr[p] = ayi[p] = 0.0;
        if constexpr (WITHJ) jr[p] = ji[p] = 0.0;
    }

    for (int64_t k0 = k_begin; k0 < k_end; k0 += T) {
        __syncthreads();
        // the weight of sample k: given, or the trapezoid rule on t
        auto weight = [&](int64_t k) {
            return cw ? cw[k] : 0.5 * (ct[k + 1 < n ? k + 1 : n - 1] - ct[k > 0 ? k - 1 : 0]);
        };
        if constexpr (MIXED) {
            // ---- stage: the pass's trajectory rows, read once per time step (coalesced)
            // instead of once per (time step, direction).  The FP64 form measured
            // faster reading the columns directly, so only the mixed form does this.
            for (int i = threadIdx.x; i < kRowCols * T; i += kBlock) {
                const int c = i >> (kLogSlots - lnt), tloc = i & (T - 1);   // T = kSlots / nt
                const int64_t k = k0 + tloc;
                double v = 0.0;
                if (k < k_end) v = c < C_NCOL ? S.col[c][k] : weight(k);
                sm.row[c][tloc] = v;
            }
            __syncthreads();
        }
        // column c at time step k (pass position tloc)
        auto col = [&](int c, int tloc, int64_t k) {
            if constexpr (MIXED) return sm.row[c][tloc];
            else return S.col[c][k];
        };
        // ---- stage: integrand and phase parts for kSlots (t, tile) pairs
        for (int i = threadIdx.x; i < kSlots * NP; i += kBlock) {
            const int slot = i / NP, p = i % NP;
            const int tloc = slot >> lnt, tile = slot & (nt - 1);
            const int64_t k = k0 + tloc;
            double fx = 0.0, fy = 0.0, fq = 0.0, thx, thy;
            const bool okx = direction(tile, p % TX, thx), oky = direction(tile, TX + p / TX, thy);
            if (k < k_end && okx && oky) {
                const double vx = col(C_VX, tloc, k), vy = col(C_VY, tloc, k), dvz = col(C_DVZ, tloc, k);
                const double ax = col(C_AX, tloc, k), ay = col(C_AY, tloc, k), az = col(C_AZ, tloc, k);
                double w;
                if constexpr (MIXED) w = sm.row[C_NCOL][tloc];
                else w = weight(k);
                const double th2h = 0.5 * (thx * thx + thy * thy);
                const double D = ((c0 + th2h) - dvz) - thx * vx - thy * vy;
                const double C = (c0 - th2h) - dvz;
                if constexpr (MIXED) {
                    // FP32 integrand; D and C are formed in FP64 (they are
                    // small differences) and rounded once.
                    const float Df = (float)D, Cf = (float)C;
                    const float G = (float)w * __builtin_amdgcn_rcpf(Df * Df);   // 1 ulp
                    const float tx = (float)thx, ty = (float)thy;
                    const float vxf = (float)vx, vyf = (float)vy;
                    const float axf = (float)ax, ayf = (float)ay, azf = (float)az;
                    fx = (double)(((azf + ty * ayf) * (tx - vxf) - (ty * (ty - vyf) + Cf) * axf) * G);
                    fy = (double)(((azf + tx * axf) * (ty - vyf) - (tx * (tx - vxf) + Cf) * ayf) * G);
                    fq = (double)((tx * axf + ty * ayf + azf) * G);
                } else {
                    const double G = w / (D * D);
                    fx = ((az + thy * ay) * (thx - vx) - (thy * (thy - vy) + C) * ax) * G;
                    fy = ((az + thx * ax) * (thy - vy) - (thx * (thx - vx) + C) * ay) * G;
                    fq = (thx * ax + thy * ay + az) * G;
                }
            }
            s_slot[slot].fxy[p] = make_double2(fx, fy);
            if constexpr (WITHJ) s_slot[slot].fq[p] = fq;
        }
        if constexpr (REC) {
            // uniform grids: per (time step, tile) the phase of the tile's first
            // direction and the multipliers of the recurrence along x and y (below)
            const double dth = S.dth;
            for (int i = threadIdx.x; i < kSlots * 4; i += kBlock) {
                const int slot = i >> 2, j = i & 3;
                const int tloc = slot >> lnt, tile = slot & (nt - 1);
                const int64_t k = k0 + tloc;
                double v = 0.0;
                if (k < k_end && grp * nt + tile < n_tiles) {
                    const double t = col(C_T, tloc, k);
                    double thx0, thy0;
                    (void)direction(tile, 0, thx0);
                    (void)direction(tile, TX, thy0);
                    if (j == 0)
                        v = ((c0 * t - col(C_DZ, tloc, k)) + thx0 * (0.5 * thx0 * t - col(C_X, tloc, k))) +
                            thy0 * (0.5 * thy0 * t - col(C_Y, tloc, k));
                    else if (j == 1)
                        v = dth * ((thx0 + 0.5 * dth) * t - col(C_X, tloc, k));
                    else if (j == 2)
                        v = dth * dth * t;
                    else
                        v = dth * ((thy0 + 0.5 * dth) * t - col(C_Y, tloc, k));
                }
                if (j < 3) s_slot[slot].px[j] = v; else s_slot[slot].py[0] = v;
            }
        } else {
            for (int i = threadIdx.x; i < kSlots * (TX + TY); i += kBlock) {
                const int slot = i / (TX + TY), j = i % (TX + TY);
                const int tloc = slot >> lnt, tile = slot & (nt - 1);
                const int64_t k = k0 + tloc;
                double v = 0.0;
                if (k < k_end && grp * nt + tile < n_tiles) {
                    const double t = col(C_T, tloc, k), y = col(C_Y, tloc, k);
                    double th, thy0;
                    (void)direction(tile, j, th);
                    (void)direction(tile, TX, thy0);
                    // Px_jx + Py_0, and Py_jy - Py_0 written as a product (0 for jy = 0)
                    if (j < TX)
                        v = ((c0 * t - col(C_DZ, tloc, k)) + th * (0.5 * th * t - col(C_X, tloc, k))) +
                            thy0 * (0.5 * thy0 * t - y);
                    else
                        v = (th - thy0) * (0.5 * (th + thy0) * t - y);
                }
                if (j < TX) s_slot[slot].px[j] = v; else s_slot[slot].py[j - TX] = v;
            }
        }
        __syncthreads();
        // ---- accumulate: every lane, its photon energy, its direction tile
        const int tn = (int)min<int64_t>((int64_t)T, k_end - k0);
        for (int tloc = 0; tloc < tn; ++tloc) {
            const int slot = tloc * nt + tl;
            double xr[TX], xi[TX];
            // the direct forms read row 0's integrand values (and the mixed form row 1's
            // phase part) before the X phase factors, so that their latency is hidden
            double2 fn[TX];
            double qn[TX];
            const AmpSlot<TX, TY, WITHJ> &S_ = s_slot[slot];
            double pyn = (MIXED && TY > 1) ? S_.py[1] : 0.0;
            if constexpr (!REC) {
#pragma unroll
                for (int jx = 0; jx < TX; ++jx) {
                    fn[jx] = S_.fxy[jx];
                    if constexpr (WITHJ) qn[jx] = S_.fq[jx];
                }
            }
            // uniform grids: the phase along x and along y is quadratic in the direction
            // index, so from the tile's first factor X_0 and R_0 = exp(i kappa a),
            // B = exp(i kappa dth^2 t), X_{j+1} = X_j R_j with R_{j+1} = R_j B (and
            // along y Y_1 = S_0, Y_{j+1} = Y_j S_j, S_{j+1} = S_j B): 4 phase factors per
            // time step instead of TX + TY - 1
            double br = 0.0, bi = 0.0, sr = 0.0, si = 0.0;
            if constexpr (REC) {
                double rr, ri;
                lane_cis<false>(kh, S_.px[0], xr[0], xi[0]);
                lane_cis<false>(kh, S_.px[1], rr, ri);
                lane_cis<false>(kh, S_.px[2], br, bi);
#pragma unroll
                for (int jx = 1; jx < TX; ++jx) {
                    xr[jx] = xr[jx - 1] * rr - xi[jx - 1] * ri;
                    xi[jx] = xr[jx - 1] * ri + xi[jx - 1] * rr;
                    if (jx + 1 < TX) {
                        const double t_ = rr * br - ri * bi;
                        ri = rr * bi + ri * br;
                        rr = t_;
                    }
                }
                lane_cis<false>(kh, S_.py[0], sr, si);
            } else {
#pragma unroll
                for (int jx = 0; jx < TX; ++jx) lane_cis<MIXED>(kh, S_.px[jx], xr[jx], xi[jx]);
            }
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int jy = 0; jy < TY; ++jy) {
                // with J at 16 directions per lane the kernel sits at the VGPR limit: each
                // row is its own scheduling region, so that only two rows of integrand
                // values are ever live; the next row's values are read at the end of this
                // row's region (software pipelining across the barrier).
                if constexpr (WITHJ && TX * TY >= 16) __builtin_amdgcn_sched_barrier(0);
                double2 f[TX];
                double q[TX];
#pragma unroll
                for (int jx = 0; jx < TX; ++jx) {
                    // the recurrence form keeps its y state in the registers the next
                    // row's prefetched integrand values would take, so it reads them here
                    if constexpr (REC) {
                        f[jx] = S_.fxy[jy * TX + jx];
                        if constexpr (WITHJ) q[jx] = S_.fq[jy * TX + jx];
                    } else {
                        f[jx] = fn[jx];
                        if constexpr (WITHJ) q[jx] = qn[jx];
                    }
                }
                // row 0: Y_0 = 1
                if constexpr (REC) {
                    if (jy == 1) {
                        yr = sr;
                        yi = si;
                    } else if (jy > 1) {
                        // Y_jy = Y_{jy-1} S_{jy-1}
                        const double t_ = yr * sr - yi * si;
                        yi = yr * si + yi * sr;
                        yr = t_;
                    }
                    if (jy > 0 && jy + 1 < TY) {
                        // S_jy = S_{jy-1} B
                        const double u_ = sr * br - si * bi;
                        si = sr * bi + si * br;
                        sr = u_;
                    }
                } else if (jy > 0) {
                    // this row's phase part: the mixed form reads the next row's one region
                    // ahead; the FP64 direct form reads it here (with that prefetch the
                    // allocator spilled two accumulators in this loop)
                    const double py = MIXED ? pyn : S_.py[jy];
                    if (MIXED && jy + 1 < TY) pyn = S_.py[jy + 1];
                    lane_cis<MIXED>(kh, py, yr, yi);
                }
#pragma unroll
                for (int jx = 0; jx < TX; ++jx) {
                    const int p = jy * TX + jx;
                    const double er = jy == 0 ? xr[jx] : xr[jx] * yr - xi[jx] * yi;
                    const double ei = jy == 0 ? xi[jx] : xr[jx] * yi + xi[jx] * yr;
                    axr[p] = __builtin_fma(f[jx].x, er, axr[p]);
                    axi[p] = __builtin_fma(f[jx].x, ei, axi[p]);
                    ayr[p] = __builtin_fma(f[jx].y, er, ayr[p]);
                    ayi[p] = __builtin_fma(f[jx].y, ei, ayi[p]);
                    if constexpr (WITHJ) {
                        jr[p] = __builtin_fma(q[jx], er, jr[p]);
                        ji[p] = __builtin_fma(q[jx], ei, ji[p]);
                    }
                }
                if (!REC && jy + 1 < TY) {
#pragma unroll
                    for (int jx = 0; jx < TX; ++jx) {
                        fn[jx] = S_.fxy[(jy + 1) * TX + jx];
                        if constexpr (WITHJ) qn[jx] = S_.fq[(jy + 1) * TX + jx];
                    }
                }
            }
        }
    }

    // ---- partial amplitudes of this chunk: part[seg][chunk][comp][n][w]
    if (iw >= n_w || gtile >= n_tiles) return;   // no barrier follows in this item
    const int64_t n_n = (int64_t)n_x * n_y;
    const int64_t base = S.part_off + (int64_t)chunk * L.comps * n_n * n_w;
    const int tx0 = (gtile % n_tx) * TX, ty0 = (gtile / n_tx) * TY;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int jx = tx0 + p % TX, jy = ty0 + p / TX;
        if (jx >= n_x || jy >= n_y) continue;
        const int64_t nn = (int64_t)jy * n_x + jx;
        if (!RAD_DEBUG_OK(base + ((int64_t)(L.comps - 1) * n_n + nn) * n_w + iw < L.part_len)) continue;
        L.part[base + (0 * n_n + nn) * n_w + iw] = make_double2(axr[p], axi[p]);
        L.part[base + (1 * n_n + nn) * n_w + iw] = make_double2(ayr[p], ayi[p]);
        if constexpr (WITHJ) L.part[base + (2 * n_n + nn) * n_w + iw] = make_double2(jr[p], ji[p]);
    }
}

// One block per work item.
template <int TX, int TY, bool WITHJ, bool MIXED, int MINB, bool REC>
__global__ __launch_bounds__(kBlock, MINB) void amp_kernel(AmpLaunch L)
{
    __shared__ AmpSmem<TX, TY, WITHJ, MIXED> sm;
    // launched with one block per item, so this runs once; written as a loop because
    // the register allocation of the hot loop comes out tighter in this form
    // (measured in the gfx950 assembly: no copies or scratch in the recurrence form)
    if constexpr (TY == 6) {
        // the 4x6 tile (no J) allocates its hot loop without spills only in this loop form
        for (int64_t b = blockIdx.x; b < L.n_blocks; b += gridDim.x) {
            amp_item<TX, TY, WITHJ, MIXED, REC>(L, b, sm);
            __syncthreads();
        }
    } else {
        amp_item<TX, TY, WITHJ, MIXED, REC>(L, (int64_t)blockIdx.x, sm);
    }
}

// Persistent form: a fixed grid of resident blocks pulls work items in launch
// order (longest segment first) from an atomic ticket until the list is
// exhausted; every block leaves the loop once a ticket is past the end.  The
// ticket only schedules: every item writes its own partial slot, so results do
// not depend on which block ran it.
template <int TX, int TY, bool WITHJ, bool MIXED, int MINB, bool REC>
__global__ __launch_bounds__(kBlock, MINB) void amp_persistent(AmpLaunch L)
{
    __shared__ AmpSmem<TX, TY, WITHJ, MIXED> sm;
    __shared__ int s_item;
    auto ticket = [&]() -> int64_t {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(L.counter, 1u);
        __syncthreads();
        const int64_t t = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();   // all lanes hold the ticket before thread 0 may take the next
        return t;
    };
    for (int64_t b = ticket(); b < L.n_blocks; b = ticket()) amp_item<TX, TY, WITHJ, MIXED, REC, false>(L, b, sm);
}

// Tickets start at zero for every launch (a kernel, so graphs hold no memset node).
__global__ void reset_counters_kernel(unsigned *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}

// Sum of the n chunk partials p[0], p[stride], ..., p[(n-1) stride] in a fixed order:
// partial c goes to running sum c % 16 and the sixteen sums are added pairwise, so that
// sixteen loads are in flight instead of one (a small problem cut into many short chunks
// would otherwise wait on one load latency per chunk).
__device__ __forceinline__ double2 chunk_sum(const double2 *__restrict__ p, int64_t stride, int n)
{
    constexpr int K = 16;
    double2 s[K];
#pragma unroll
    for (int j = 0; j < K; ++j) s[j] = make_double2(0.0, 0.0);
    int c = 0;
    for (; c + K <= n; c += K) {
        double2 v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = p[(int64_t)(c + j) * stride];
        // all K loads are issued before the first add waits (the scheduler would
        // otherwise reuse one register and wait after every load)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            s[j].x += v[j].x;
            s[j].y += v[j].y;
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (c + j < n) {
            const double2 v = p[(int64_t)(c + j) * stride];
            s[j].x += v.x;
            s[j].y += v.y;
        }
    // pairwise: 16 -> 8 -> 4 -> 2 -> 1
#pragma unroll
    for (int h = K / 2; h >= 1; h /= 2)
#pragma unroll
        for (int j = 0; j < h; ++j) {
            s[j].x += s[j + h].x;
            s[j].y += s[j + h].y;
        }
    return s[0];
}

// ONE: every segment of the launch is a single chunk, and its partial is the sum (the
// same value chunk_sum returns for n = 1, without the sixteen running sums' registers)
template <bool ONE>
__device__ __forceinline__ void sum_chunks(const double2 *__restrict__ part, int64_t part_len, const SegDesc &d,
                                           int comps, int comp, int64_t n_n, int n_w, int64_t nn,
                                           int iw, double &re, double &im)
{
    const int64_t stride = (int64_t)comps * n_n * n_w;
    const int64_t first = d.part_off + ((int64_t)comp * n_n + nn) * n_w + iw;
    if (!RAD_DEBUG_OK(first >= 0 && first + (int64_t)(d.n_chunks - 1) * stride < part_len)) {
        re = im = 0.0;
        return;
    }
    (void)part_len;
    const double2 *p = part + first;
    const double2 v = ONE ? *p : chunk_sum(p, stride, d.n_chunks);
    re = v.x;
    im = v.y;
}

template <bool ONE>
__global__ __launch_bounds__(256) void fin_kernel(FinLaunch F)
{
    const int64_t n_n = (int64_t)F.n_x * F.n_y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int o = blockIdx.y;
    if (i >= n_n * F.n_w) return;
    const int iw = (int)(i % F.n_w);
    const int64_t nn = i / F.n_w;
    const int jx = (int)(nn % F.n_x), jy = (int)(nn / F.n_x);
    const double thx = F.thx[jx], thy = F.thy[jy], hw = F.hw[iw];
    const double pref = kAlpha / (4.0 * kPi * kPi);
    double sc = 0.0, s0 = 0.0, sh = 0.0;
    for (int e = F.out_seg_begin[o]; e < F.out_seg_begin[o + 1]; ++e) {
        const int s = F.out_seg_list[e];
        if (F.kinds & 1) {
            const SegDesc &d = F.cls[s];
            double xr, xi, yr, yi;
            sum_chunks<ONE>(F.part_c, F.part_c_len, d, 2, 0, n_n, F.n_w, nn, iw, xr, xi);
            sum_chunks<ONE>(F.part_c, F.part_c_len, d, 2, 1, n_n, F.n_w, nn, iw, yr, yi);
            const double zr = -(thx * xr + thy * yr), zi = -(thx * xi + thy * yi);
            sc += pref * (xr * xr + xi * xi + yr * yr + yi * yi + zr * zr + zi * zi);
        }
        if (F.kinds & 6) {
            const SegDesc &d = F.qs[s];
            const double E = d.energy;
            if (hw < E) {
                double xr, xi, yr, yi;
                sum_chunks<ONE>(F.part_q, F.part_q_len, d, F.comps_q, 0, n_n, F.n_w, nn, iw, xr, xi);
                sum_chunks<ONE>(F.part_q, F.part_q_len, d, F.comps_q, 1, n_n, F.n_w, nn, iw, yr, yi);
                const double zr = -(thx * xr + thy * yr), zi = -(thx * xi + thy * yi);
                const double S = xr * xr + xi * xi + yr * yr + yi * yi + zr * zr + zi * zi;
                const double Es = E - hw;
                if (F.kinds & 2) s0 += pref * (Es / E) * S;
                if (F.kinds & 4) {
                    double jr_, ji_;
                    sum_chunks<ONE>(F.part_q, F.part_q_len, d, F.comps_q, 2, n_n, F.n_w, nn, iw, jr_, ji_);
                    const double SJ = jr_ * jr_ + ji_ * ji_;
                    sh += pref * ((Es * Es + E * E) / (2.0 * E * E) * S +
                                  hw * hw / (2.0 * E * E * d.gamma * d.gamma) * SJ);
                }
            }
        }
    }
    const int64_t cube = n_n * F.n_w;
    const int64_t dst = (int64_t)iw * n_n + nn;
    double *out = F.out + (int64_t)o * F.n_kinds * cube;
    int kk = 0;
    if (F.kinds & 1) out[(kk++) * cube + dst] = sc;
    if (F.kinds & 2) out[(kk++) * cube + dst] = s0;
    if (F.kinds & 4) out[(kk++) * cube + dst] = sh;
}

// Cell integrals of the refinement.  Thread per (segment, cell, photon energy),
// photon energy fastest (contiguous partial reads).  Directions and chunks are
// summed in a fixed order.
__global__ __launch_bounds__(256) void cells_fin_kernel(CellsFin F)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)F.n_segs * F.n_cells * F.n_w;
    if (i >= total) return;
    const int w = (int)(i % F.n_w);
    const int c = (int)((i / F.n_w) % F.n_cells);
    const int s = (int)(i / ((int64_t)F.n_w * F.n_cells));
    const int64_t dst = ((int64_t)s * F.n_w + w) * F.n_cells + c;
    const int p = F.psof[(int64_t)s * F.n_cells + c];
    if (p < 0 || !F.mask[dst]) {
        F.out[dst] = 0.0;
        return;
    }
    const SegDesc &d = F.segs[p];
    const double hw = F.hw[w], E = d.energy;
    if (F.kind != 1 && !(hw < E)) {
        F.out[dst] = 0.0;
        return;
    }
    const int ci = c % F.ncx, cj = c / F.ncx;
    const int n_dir = F.cx * F.cy;
    const int64_t stride = (int64_t)F.comps * n_dir * F.n_w;
    const double pref = kAlpha / (4.0 * kPi * kPi);
    double acc = 0.0;
    for (int nn = 0; nn < n_dir; ++nn) {
        const int jx = nn % F.cx, jy = nn / F.cx;
        const double thx = d.thx[jx], thy = d.thy[jy];
        double re[3] = {0.0, 0.0, 0.0}, im[3] = {0.0, 0.0, 0.0};
        for (int comp = 0; comp < F.comps; ++comp) {
            const int64_t first = d.part_off + ((int64_t)comp * n_dir + nn) * F.n_w + w;
            if (!RAD_DEBUG_OK(first >= 0 && first + (int64_t)(d.n_chunks - 1) * stride < F.part_len)) continue;
            const double2 v = chunk_sum(F.part + first, stride, d.n_chunks);
            re[comp] = v.x;
            im[comp] = v.y;
        }
        const double zr = -(thx * re[0] + thy * re[1]), zi = -(thx * im[0] + thy * im[1]);
        const double S = re[0] * re[0] + im[0] * im[0] + re[1] * re[1] + im[1] * im[1] + zr * zr + zi * zi;
        double spec;
        if (F.kind == 1) {
            spec = pref * S;
        } else {
            const double Es = E - hw;
            if (F.kind == 2)
                spec = pref * (Es / E) * S;
            else
                spec = pref * ((Es * Es + E * E) / (2.0 * E * E) * S +
                               hw * hw / (2.0 * E * E * d.gamma * d.gamma) * (re[2] * re[2] + im[2] * im[2]));
        }
        acc += spec * F.wx[ci * F.cx + jx] * F.wy[cj * F.cy + jy];
    }
    F.out[dst] = acc;
}

// dIdw[c][i] = sum_{jy, jx} cube[c][i][jy][jx] wx[jx] wy[jy]; one block per (i, c),
// a fixed strided partial sum per thread and a fixed tree: deterministic.
__global__ __launch_bounds__(256) void angle_kernel(const double *__restrict__ cube,
                                                    const double *__restrict__ wx,
                                                    const double *__restrict__ wy, int n_x,
                                                    int n_y, int n_w, double *__restrict__ out)
{
    __shared__ double red[256];
    const int i = blockIdx.x, c = blockIdx.y;
    const int64_t n_n = (int64_t)n_x * n_y;
    const double *row = cube + ((int64_t)c * n_w + i) * n_n;
    double acc = 0.0;
    for (int64_t p = threadIdx.x; p < n_n; p += blockDim.x) {
        const int jx = (int)(p % n_x), jy = (int)(p / n_x);
        acc += row[p] * wx[jx] * wy[jy];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)c * n_w + i] = red[0];
}

// The phase-factor routines of the two forms on given arguments: half turns u
// (cos(pi u), sin(pi u), FP64 polynomial) or revolutions r (cos(2 pi r), sin(2 pi r),
// hardware FP32 sin/cos after the exact FP64 reduction), for measuring their accuracy.
__global__ __launch_bounds__(256) void phase_kernel(const double *__restrict__ turns, int64_t n, int mixed,
                                                    double *__restrict__ c, double *__restrict__ s)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double cc, ss;
        if (mixed) {
            float cf, sf;
            cis_revolutions_f32(turns[i], cf, sf);
            cc = cf;
            ss = sf;
        } else {
            cis_halfturns(turns[i], cc, ss);
        }
        c[i] = cc;
        s[i] = ss;
    }
}

// ---------------------------------------------------------------- launchers
// grid_blocks > 0: persistent launch with that many blocks; 0: one block per item.
// occupancy != nullptr: only report resident blocks per CU of the persistent kernel.
template <int TX, int TY, bool WITHJ, bool MIXED, int MINB, bool REC>
static hipError_t launch_amp_r(const AmpLaunch &L, int grid_blocks, hipStream_t st, int *occupancy)
{
    if (occupancy)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occupancy, reinterpret_cast<const void *>(amp_persistent<TX, TY, WITHJ, MIXED, MINB, REC>), kBlock, 0);
    if (grid_blocks > 0)
        hipLaunchKernelGGL((amp_persistent<TX, TY, WITHJ, MIXED, MINB, REC>), dim3((unsigned)grid_blocks),
                           dim3(kBlock), 0, st, L);
    else
        hipLaunchKernelGGL((amp_kernel<TX, TY, WITHJ, MIXED, MINB, REC>), dim3((unsigned)L.n_blocks),
                           dim3(kBlock), 0, st, L);
    return hipGetLastError();
}

// The recurrence form exists for FP64 only: in the mixed form a hardware phase
// factor costs about as much as the complex products that would replace it.
template <int TX, int TY, bool WITHJ, bool MIXED, int MINB>
static hipError_t launch_amp_t(const AmpLaunch &L, int grid_blocks, hipStream_t st, int *occupancy)
{
    if constexpr (!MIXED)
        if (L.rec) return launch_amp_r<TX, TY, WITHJ, false, MINB, true>(L, grid_blocks, st, occupancy);
    return launch_amp_r<TX, TY, WITHJ, MIXED, MINB, false>(L, grid_blocks, st, occupancy);
}

template <bool WITHJ, bool MIXED>
static hipError_t launch_amp_v(const AmpLaunch &L, int variant, int grid_blocks, hipStream_t st,
                               int *occupancy)
{
    switch (variant) {
    case kVar44x2: return launch_amp_t<4, 4, WITHJ, MIXED, 2>(L, grid_blocks, st, occupancy);
    case kVar43x2: return launch_amp_t<4, 3, WITHJ, MIXED, 2>(L, grid_blocks, st, occupancy);
    case kVar44x1: return launch_amp_t<4, 4, WITHJ, MIXED, 1>(L, grid_blocks, st, occupancy);
    case kVar42x2: return launch_amp_t<4, 2, WITHJ, MIXED, 2>(L, grid_blocks, st, occupancy);
    case kVar46x2:
        if constexpr (WITHJ) return hipErrorInvalidValue;   // rejected on the host first
        else return launch_amp_t<4, 6, false, MIXED, 2>(L, grid_blocks, st, occupancy);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_amp(const AmpLaunch &L, int variant, bool withj, bool mixed, int grid_blocks,
                      hipStream_t st, int *occupancy)
{
    // the kernel shifts by log2(nt) (an occupancy query passes no launch)
    if (!occupancy && L.nt != 1 && L.nt != 2 && L.nt != 4) return hipErrorInvalidValue;
    // compacted cell items need the item list and the one-block-per-item form
    if (L.n_live && (grid_blocks > 0 || !L.items)) return hipErrorInvalidValue;
    // so do grouped cell items (wg = 0: each item carries its shape); else wg is 1, 2 or 4
    if (!occupancy && L.wg == 0 && (grid_blocks > 0 || !L.items)) return hipErrorInvalidValue;
    if (!occupancy && L.wg != 0 && L.wg != 1 && L.wg != 2 && L.wg != 4) return hipErrorInvalidValue;
    if (withj)
        return mixed ? launch_amp_v<true, true>(L, variant, grid_blocks, st, occupancy)
                     : launch_amp_v<true, false>(L, variant, grid_blocks, st, occupancy);
    return mixed ? launch_amp_v<false, true>(L, variant, grid_blocks, st, occupancy)
                 : launch_amp_v<false, false>(L, variant, grid_blocks, st, occupancy);
}

hipError_t launch_cells_fin(const CellsFin &F, hipStream_t st)
{
    const int64_t total = (int64_t)F.n_segs * F.n_cells * F.n_w;
    hipLaunchKernelGGL(cells_fin_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, F);
    return hipGetLastError();
}

// Cell compaction, pass 1: one wave per item, flags[i] = 1 if any photon energy of the
// item's block has its mask bit set for the item's (segment, cell).
__global__ __launch_bounds__(256) void cell_flags_kernel(CellCompact C)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (i >= C.n_items) return;
    const int4 it = C.items[i];
    const int s = it.x / C.n_cells, c = it.x % C.n_cells;
    int any = 0;
    for (int k = lane; k < C.wg * kWave; k += kWave) {
        const int w = it.w * C.wg * kWave + k;
        if (w < C.n_w) any |= C.mask[((int64_t)s * C.n_w + w) * C.n_cells + c] != 0;
    }
    any = __any(any);
    if (lane == 0) C.flags[i] = any;
}

// Pass 2: one block of 1024 threads scans the flags tile by tile in order and writes the
// flagged items to live[0 .. n), n to *n_live (order kept: the launch order of the plan).
__global__ __launch_bounds__(1024) void cell_compact_kernel(CellCompact C)
{
    __shared__ int wsum[16];
    __shared__ int base;
    const int t = threadIdx.x, lane = t % kWave, wave = t / kWave;
    if (t == 0) base = 0;
    __syncthreads();
    for (int64_t t0 = 0; t0 < C.n_items; t0 += 1024) {
        const int64_t i = t0 + t;
        const int f = i < C.n_items ? C.flags[i] : 0;
        const uint64_t bal = __ballot(f);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));   // flagged lanes below this one
        if (lane == 0) wsum[wave] = __popcll(bal);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        if (f) C.live[off + before] = C.items[i];
        __syncthreads();
        if (t == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wsum[w];
            base += tot;
        }
        __syncthreads();
    }
    if (t == 0) *C.n_live = base;
}

// Pass 1 of the grouped form: one wave per row of n_wb dense items (p, chunk, 0, b).  The
// row's blocks with a mask bit set are taken in order by four, then by two, then one by one
// (the remainder of 3 as 2 + 1); a group of k blocks becomes k items, tile group
// g = 0 .. k - 1 with k in bits 8..15 and the k block indices one byte each, written in
// order to the row's first slots of `grouped` and flagged; the row's other slots are left
// unflagged.  The items are as many as the selected blocks, as in the one-block form.
__global__ __launch_bounds__(256) void cell_group_kernel(CellCompact C)
{
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (r >= C.n_items / C.n_wb) return;
    const int64_t i0 = r * C.n_wb;
    const int4 it = C.items[i0];
    const int s = it.x / C.n_cells, c = it.x % C.n_cells;
    int j = 0;                      // items written so far (wave-uniform)
    auto emit = [&](int k, uint32_t blocks) {
        if (lane < k) {
            C.grouped[i0 + j + lane] = make_int4(it.x, it.y, lane | (k << 8), (int)blocks);
            C.flags[i0 + j + lane] = 1;
        }
        j += k;
    };
    uint32_t pend = 0;              // pending block indices, one byte each
    int np = 0;
    for (int b = 0; b < C.n_wb; ++b) {
        const int w = b * kWave + lane;
        if (__any(w < C.n_w && C.mask[((int64_t)s * C.n_w + w) * C.n_cells + c] != 0)) {
            pend |= (uint32_t)b << (8 * np);
            if (++np == 4) {
                emit(4, pend);
                pend = 0;
                np = 0;
            }
        }
    }
    if (np >= 2) {
        emit(2, pend & 0xffffu);
        pend >>= 16;
        np -= 2;
    }
    if (np == 1) emit(1, pend);
    for (int k = j + lane; k < C.n_wb; k += kWave) C.flags[i0 + k] = 0;
}

hipError_t launch_cell_compact(const CellCompact &C, hipStream_t st)
{
    // the live count and offsets are 32-bit
    if (C.n_items < 1 || C.n_items > 0x7fffffff || C.n_cells < 1 || C.wg < 0) return hipErrorInvalidValue;
    CellCompact P = C;
    if (C.wg == 0) {
        // block indices are packed in bytes; rows are whole
        if (C.n_wb < 1 || C.n_wb > 256 || C.n_items % C.n_wb || !C.grouped) return hipErrorInvalidValue;
        const int64_t threads = C.n_items / C.n_wb * kWave;
        hipLaunchKernelGGL(cell_group_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, C);
        P.items = C.grouped;
    } else {
        const int64_t threads = C.n_items * kWave;
        hipLaunchKernelGGL(cell_flags_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, C);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cell_compact_kernel, dim3(1), dim3(1024), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_reset(unsigned *counters, int n, hipStream_t st)
{
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, st, counters, n);
    return hipGetLastError();
}

hipError_t launch_fin(const FinLaunch &F, hipStream_t st)
{
    const int64_t items = (int64_t)F.n_x * F.n_y * F.n_w;
    const unsigned gx = (unsigned)((items + 255) / 256);
    if (F.one_chunk)
        hipLaunchKernelGGL(fin_kernel<true>, dim3(gx, (unsigned)F.n_out), dim3(256), 0, st, F);
    else
        hipLaunchKernelGGL(fin_kernel<false>, dim3(gx, (unsigned)F.n_out), dim3(256), 0, st, F);
    return hipGetLastError();
}

// ---------------------------------------------------------------- descriptor upload
// Copies `n` bytes carried in the kernel argument to device memory: descriptors reach
// device memory without host staging buffers or a memcpy node.
constexpr unsigned kUploadChunk = 3072;
struct UploadChunk {
    unsigned char b[kUploadChunk];
};

__global__ __launch_bounds__(256) void upload_kernel(unsigned char *__restrict__ dst, UploadChunk c, unsigned n)
{
    for (unsigned i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.b[i];
}

hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const unsigned char *s = (const unsigned char *)src;
    for (size_t off = 0; off < bytes; off += kUploadChunk) {
        const unsigned n = (unsigned)(bytes - off < kUploadChunk ? bytes - off : kUploadChunk);
        UploadChunk c;
        __builtin_memcpy(c.b, s + off, n);
        hipLaunchKernelGGL(upload_kernel, dim3(1), dim3(256), 0, st, (unsigned char *)dst + off, c, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}


hipError_t launch_phase(const double *turns, int64_t n, int mixed, double *c, double *s, hipStream_t st)
{
    const int64_t want = (n + 255) / 256, blocks = want < 8192 ? want : 8192;
    hipLaunchKernelGGL(phase_kernel, dim3((unsigned)blocks), dim3(256), 0, st, turns, n, mixed, c, s);
    return hipGetLastError();
}

hipError_t launch_angle(const double *cube, const double *wx, const double *wy, int n_x, int n_y,
                        int n_w, int n_cubes, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(angle_kernel, dim3((unsigned)n_w, (unsigned)n_cubes), dim3(256), 0, st, cube,
                       wx, wy, n_x, n_y, n_w, out);
    return hipGetLastError();
}

}  // namespace rad

extern "C" int64_t rad_debug_violations(int reset)
{
#if RAD_DEBUG
    unsigned long long v = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(rad::g_debug_violations), sizeof v, 0, hipMemcpyDeviceToHost) != hipSuccess)
        return -2;
    if (reset) {
        const unsigned long long z = 0;
        if (hipMemcpyToSymbol(HIP_SYMBOL(rad::g_debug_violations), &z, sizeof z, 0, hipMemcpyHostToDevice) != hipSuccess)
            return -2;
    }
    return (int64_t)v;
#else
    (void)reset;
    return -1;
#endif
}

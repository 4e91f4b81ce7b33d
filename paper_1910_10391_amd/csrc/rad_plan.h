// Launch planning of the amplitude kernels: block shape, time chunks and the
// workspace layout of a call, as plain integer arithmetic on the grid sizes (no HIP
// calls), shared by the library and its CPU checks (built there with the host
// sanitizers).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>

namespace radplan {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Tile {
    int variant, wg, nt, n_tx, n_ty, n_groups, n_wblocks;
    int64_t base_blocks;
};

// Block shape for a grid of n_w photon energies and n_x x n_y directions, with a
// direction tile of tx x ty per lane: wg waves of a block spread over photon energies,
// nt = 4 / wg direction tiles per block.
// wg_pref: 1, 2 or 4 waves over photon energies; anything else chooses by n_w.
inline Tile plan_tile(int n_w, int n_x, int n_y, int variant, int tx, int ty, int wg_pref = 0)
{
    Tile t;
    t.variant = variant;
    t.wg = (wg_pref == 1 || wg_pref == 2 || wg_pref == 4) ? wg_pref : (n_w > 128 ? 4 : (n_w > 64 ? 2 : 1));
    t.nt = kWavesPerBlock / t.wg;
    t.n_tx = (n_x + tx - 1) / tx;
    t.n_ty = (n_y + ty - 1) / ty;
    const int tiles = t.n_tx * t.n_ty;
    t.n_groups = (tiles + t.nt - 1) / t.nt;
    t.n_wblocks = (n_w + kWave * t.wg - 1) / (kWave * t.wg);
    t.base_blocks = (int64_t)t.n_groups * t.n_wblocks;
    return t;
}

constexpr int64_t kTargetBlocks = 2048;  // 256 CUs x 2 resident blocks x 4 rounds
// Chunk lengths are multiples of kMinChunk samples.  A small problem (few direction
// tiles and photon energies) is cut this fine so that its blocks, each a single
// latency-bound wave per SIMD, stay short; the finalize sums the many partials with
// sixteen loads in flight.
constexpr int64_t kMinChunk = 16;
// Longest chunk: chunk lengths are 32-bit in the descriptors, while a segment may have
// up to 2^40 samples.
constexpr int64_t kMaxChunk = (int64_t)1 << 30;

// Largest work-item target the tuning accepts.
constexpr int64_t kMaxTargetBlocks = (int64_t)1 << 24;

// chunks per segment when the launch has `n_segs` segments: enough for `target` work
// items (kTargetBlocks unless tuned)
inline int64_t chunk_factor(const Tile &t, int64_t n_segs, int64_t target = kTargetBlocks)
{
    const int64_t have = n_segs * t.base_blocks;
    if (have >= target) return 1;
    return (target + have - 1) / have;
}

// A segment of n samples cut for chunk factor c: chunk_len a multiple of kMinChunk (or
// n itself), at most kMaxChunk, n_chunks = ceil(n / chunk_len).
inline void plan_chunks(int64_t n, int64_t c, int32_t &n_chunks, int32_t &chunk_len)
{
    int64_t len = (n + c - 1) / c;
    len = (len + kMinChunk - 1) / kMinChunk * kMinChunk;
    len = std::min(std::min(len, n), kMaxChunk);
    chunk_len = (int32_t)len;
    n_chunks = (int32_t)((n + len - 1) / len);
}

// The most chunks plan_chunks gives any segment of at most n samples: min(cf,
// ceil(n / kMinChunk)) while the chunk-length cap does not decide, else
// ceil(n / kMaxChunk); both grow with n.
inline int64_t max_chunks(int64_t n, int64_t cf)
{
    return std::max<int64_t>(std::min<int64_t>(cf, (n + kMinChunk - 1) / kMinChunk), (n + kMaxChunk - 1) / kMaxChunk);
}

inline int popcount3(int k) { return (k & 1) + ((k >> 1) & 1) + ((k >> 2) & 1); }

// kinds bits, as rad_kind
constexpr int kClassical = 1, kSpin0 = 2, kSpinHalf = 4;

// Workspace of a call: the descriptor region (two tickets, segment descriptors of both
// integral sets in launch order and by segment, the output -> segment lists), then the
// chunk partial amplitudes of each set, [seg][chunk][comp][n][w] complex FP64.
struct Layout {
    size_t off_counters, off_amp_c, off_amp_q, off_id_c, off_id_q, off_begin, off_list, off_part_c,
        off_part_q;
    size_t desc_bytes;  // bytes of the descriptor region (uploaded)
    size_t total;
    int comps_q;
};

inline Layout layout(int n_w, int n_x, int n_y, size_t seg_desc_bytes, int n_segs, int n_out, int kinds,
                     int64_t sum_chunks)
{
    Layout L{};
    const size_t sd = seg_desc_bytes * (size_t)n_segs;
    size_t o = 0;
    L.off_counters = o; o = align_up(o + 2 * sizeof(unsigned));
    L.off_amp_c = o; o = align_up(o + sd);
    L.off_amp_q = o; o = align_up(o + sd);
    L.off_id_c = o; o = align_up(o + sd);
    L.off_id_q = o; o = align_up(o + sd);
    L.off_begin = o; o = align_up(o + sizeof(int) * (size_t)(n_out + 1));
    L.off_list = o; o = align_up(o + sizeof(int) * (size_t)n_segs);
    L.desc_bytes = o;
    const size_t cube2 = (size_t)n_w * n_x * n_y * 16;   // complex FP64
    L.comps_q = (kinds & kSpinHalf) ? 3 : 2;
    L.off_part_c = o;
    if (kinds & kClassical) o = align_up(o + (size_t)sum_chunks * 2 * cube2);
    L.off_part_q = o;
    if (kinds & (kSpin0 | kSpinHalf)) o = align_up(o + (size_t)sum_chunks * L.comps_q * cube2);
    L.total = o;
    return L;
}

}  // namespace radplan

// CPU checks of the launch-planning arithmetic (csrc/rad_plan.h), built with the host
// address and undefined-behaviour sanitizers by tests/test_host_sanitizers.py.
// Prints "ok" and exits 0, or names the first failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rad_plan.h"

using namespace radplan;

static int fails = 0;
#define CHECK(c, ...)                                                 \
    do {                                                              \
        if (!(c)) {                                                   \
            std::printf("FAILED %s:%d: %s: ", __FILE__, __LINE__, #c); \
            std::printf(__VA_ARGS__);                                 \
            std::printf("\n");                                        \
            if (++fails > 20) std::exit(1);                           \
        }                                                             \
    } while (0)

int main()
{
    // segment lengths: small, around the chunk multiples, and past the 2^30 chunk cap
    std::vector<int64_t> ns = {2, 3, 15, 16, 17, 31, 33, 100, 3000, 40000, 120000, 300000, 1 << 20};
    for (int64_t k = 1; k <= 4; ++k)
        for (int64_t d : {-17, -1, 0, 1, 5}) ns.push_back(k * kMaxChunk + d);
    ns.push_back(((int64_t)1 << 40) - 3);
    ns.push_back((int64_t)1 << 40);
    const int64_t cfs[] = {1, 2, 3, 7, 16, 171, 1024, 2048};
    for (int64_t n : ns)
        for (int64_t cf : cfs) {
            int32_t nc = 0, len = 0;
            plan_chunks(n, cf, nc, len);
            CHECK(len >= 1 && len <= kMaxChunk, "n %lld cf %lld len %d", (long long)n, (long long)cf, len);
            CHECK(len == n || len % kMinChunk == 0, "n %lld cf %lld len %d", (long long)n, (long long)cf, len);
            CHECK((int64_t)nc * len >= n && (int64_t)(nc - 1) * len < n, "n %lld cf %lld: %d x %d",
                  (long long)n, (long long)cf, nc, len);
            // the workspace bound of a call with segments of at most n samples covers this
            // segment and every shorter one
            for (int64_t m : ns) {
                if (m > n) continue;
                int32_t mc = 0, ml = 0;
                plan_chunks(m, cf, mc, ml);
                CHECK(max_chunks(n, cf) >= mc, "bound n %lld cf %lld < chunks of %lld (%d)", (long long)n,
                      (long long)cf, (long long)m, mc);
            }
        }
    // the case the 2^30 cap decides: one chunk factor, three and a bit chunk lengths
    {
        const int64_t n = 3 * kMaxChunk + 5;
        int32_t nc = 0, len = 0;
        plan_chunks(n, 1, nc, len);
        CHECK(nc == 4 && len == kMaxChunk, "%d x %d", nc, len);
        CHECK(max_chunks(n, 1) == 4, "%lld", (long long)max_chunks(n, 1));
    }
    // block shapes and chunk factors
    for (int n_w : {1, 37, 64, 65, 128, 129, 512}) {
        const Tile t = plan_tile(n_w, 32, 32, 0, 4, 4);
        CHECK(t.wg * t.nt == kWavesPerBlock, "n_w %d", n_w);
        CHECK((int64_t)t.n_wblocks * kWave * t.wg >= n_w && (int64_t)(t.n_wblocks - 1) * kWave * t.wg < n_w,
              "n_w %d", n_w);
        CHECK(t.n_groups * t.nt >= t.n_tx * t.n_ty, "n_w %d", n_w);
        for (int64_t segs : {1, 3, 256, 4096}) {
            const int64_t cf = chunk_factor(t, segs);
            CHECK(cf >= 1 && (cf == 1 || segs * t.base_blocks * cf >= kTargetBlocks), "segs %lld", (long long)segs);
        }
    }
    // workspace layout: aligned, ordered, regions large enough
    for (int kinds = 1; kinds <= 7; ++kinds)
        for (int n_segs : {1, 5, 2048}) {
            const int64_t sum_chunks = 3 * (int64_t)n_segs;
            const Layout L = layout(256, 16, 16, 200, n_segs, n_segs, kinds, sum_chunks);
            const size_t offs[] = {L.off_counters, L.off_amp_c, L.off_amp_q, L.off_id_c, L.off_id_q,
                                   L.off_begin, L.off_list, L.desc_bytes, L.off_part_c, L.off_part_q, L.total};
            for (size_t i = 0; i < sizeof offs / sizeof offs[0]; ++i) {
                CHECK(offs[i] % kAlign == 0, "kinds %d segs %d offset %zu", kinds, n_segs, i);
                if (i) CHECK(offs[i] >= offs[i - 1], "kinds %d segs %d offset %zu", kinds, n_segs, i);
            }
            CHECK(L.off_amp_q - L.off_amp_c >= 200 * (size_t)n_segs, "descriptors");
            CHECK(L.off_list - L.off_begin >= sizeof(int) * (size_t)(n_segs + 1), "output lists");
            const size_t cube2 = (size_t)256 * 16 * 16 * 16;
            const size_t need_c = (kinds & kClassical) ? (size_t)sum_chunks * 2 * cube2 : 0;
            const size_t need_q = (kinds & (kSpin0 | kSpinHalf)) ? (size_t)sum_chunks * L.comps_q * cube2 : 0;
            CHECK(L.off_part_q - L.off_part_c >= need_c, "classical partials");
            CHECK(L.total - L.off_part_q >= need_q, "quantum partials");
            CHECK(L.comps_q == ((kinds & kSpinHalf) ? 3 : 2), "components");
        }
    CHECK(popcount3(7) == 3 && popcount3(4) == 1 && popcount3(0) == 0, "popcount");
    if (fails) return 1;
    std::printf("ok\n");
    return 0;
}

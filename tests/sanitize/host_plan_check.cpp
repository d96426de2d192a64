// Host-only exercise of the C ABI's plan logic (validation, work list, band
// schedule, queries, twiddle tables) for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer.  VBW_HOST_ONLY plans never touch the device, so
// the GPU launchers are stubs here.  Exit code 0 = every check passed.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "vbw.h"
#include "vbw_internal.h"

namespace vbw {
int ols_fft_wg_per_cu(int, Storage, bool) { return 1; }
hipError_t launch_ols_fft(const LaunchArgs &, int, Storage, bool, hipStream_t, hipEvent_t, hipEvent_t) {
    return hipErrorInvalidValue;
}
int ols_gemm_wg_per_cu(Storage, bool) { return 1; }
hipError_t launch_ols_gemm(const LaunchArgs &, Storage, bool, hipStream_t, hipEvent_t, hipEvent_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_stream_update(const LaunchArgs &, int, Storage, void *, int64_t *, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_stream_reset(void *, int64_t, int64_t *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_copy(const void *, void *, int64_t, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t scratch_of_device(int, unsigned char **, hipError_t (*)(unsigned char *)) { return hipErrorInvalidValue; }
}  // namespace vbw

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

int main() {
    std::mt19937 rng(7);
    std::vector<double> pool(256);
    for (auto &v : pool) v = std::uniform_real_distribution<double>(0, 1)(rng);
    // random plans: mixed N, hops, lengths (incl. 0), dtypes, flags
    for (int trial = 0; trial < 300; ++trial) {
        const int nch = 1 + int(rng() % 9);
        std::vector<vbw_channel> ch(nch);
        int64_t want_blocks = 0;
        for (auto &c : ch) {
            c.n = 1 << (4 + int(rng() % 9));
            c.hop = c.n - 2 * (1 + int(rng() % (c.n / 2 - 1)));
            if (c.hop < 1) c.hop = c.n - 2;
            c.lv = int(rng() % 6);
            c.v_offset = int(rng() % 200);
            c.k1 = c.lv == 0 ? 1 + int(rng() % (c.n / 2 - 1)) : 1 + int(rng() % (c.n / 2 - c.lv));
            c.reserved = 0;
            c.len = (rng() % 5 == 0) ? 0 : int64_t(rng() % 200000);
            want_blocks += c.len ? (c.len + c.hop - 1) / c.hop : 0;
        }
        vbw_plan_desc d{nch, int(pool.size()), ch.data(), pool.data(), int(rng() % 4), 0,
                        VBW_HOST_ONLY | ((rng() & 1) ? VBW_NO_PRUNE : 0u), 0};
        vbw_plan_t p = nullptr;
        const vbw_status st = vbw_plan(&d, &p);
        CHECK(st == VBW_OK);
        if (st != VBW_OK) continue;
        CHECK(vbw_plan_query(p, VBW_Q_TOTAL_BLOCKS) == want_blocks);
        CHECK(vbw_plan_query(p, VBW_Q_N_CHANNELS) == nch);
        // random band changes against a reference map
        std::vector<std::map<int64_t, int>> ref(nch);
        for (int c = 0; c < nch; ++c) ref[c][0] = ch[c].k1;
        for (int e = 0; e < 40; ++e) {
            const int c = int(rng() % nch);
            const int64_t from = int64_t(rng() % 500);
            const int k1 = ch[c].lv == 0 ? 1 + int(rng() % (ch[c].n / 2 - 1)) : 1 + int(rng() % (ch[c].n / 2 - ch[c].lv));
            CHECK(vbw_set_bandwidth(p, c, k1, from) == VBW_OK);
            ref[c][from] = k1;
        }
        for (int q = 0; q < 50; ++q) {
            const int c = int(rng() % nch);
            const int64_t m = int64_t(rng() % 600);
            const int want = std::prev(ref[c].upper_bound(m))->second;
            CHECK(vbw_block_k1(p, c, m) == want);
        }
        CHECK(vbw_set_bandwidth(p, nch, 1, 0) == VBW_EINVAL);
        CHECK(vbw_set_bandwidth(p, 0, 0, 0) == VBW_ERANGE);
        CHECK(vbw_filter(p, nullptr, nullptr, nullptr) == VBW_EINVAL);
        CHECK(vbw_filter_timed(p, nullptr, nullptr, nullptr, nullptr, nullptr) == VBW_EINVAL);
        vbw_destroy(p);
    }
    // every validation error path
    vbw_channel good{256, 192, 8, 0, 24, 0, 1000};
    auto expect = [&](vbw_channel c, int dtype, int engine, uint32_t flags, vbw_status want) {
        vbw_plan_desc d{1, int(pool.size()), &c, pool.data(), dtype, engine, flags | VBW_HOST_ONLY, 0};
        vbw_plan_t p = nullptr;
        const vbw_status st = vbw_plan(&d, &p);
        CHECK(st == want);
        CHECK((st == VBW_OK) == (p != nullptr));
        vbw_destroy(p);
    };
    expect(good, 0, 0, 0, VBW_OK);
    vbw_channel c = good;
    c.n = 100; expect(c, 0, 0, 0, VBW_EINVAL);
    c = good; c.hop = 191; expect(c, 0, 0, 0, VBW_EINVAL);
    c = good; c.k1 = 0; expect(c, 0, 0, 0, VBW_ERANGE);
    c = good; c.k1 = 125; expect(c, 0, 0, 0, VBW_ERANGE);
    c = good; c.v_offset = 250; expect(c, 0, 0, 0, VBW_EINVAL);
    c = good; c.len = -1; expect(c, 0, 0, 0, VBW_EINVAL);
    c = good; c.reserved = 1; expect(c, 0, 0, 0, VBW_EINVAL);
    expect(good, 7, 0, 0, VBW_EINVAL);
    expect(good, 0, 1, 0, VBW_EUNSUPPORTED);
    expect(good, 3, 1, 0, VBW_EUNSUPPORTED);
    expect(good, 0, 0, 1u << 20, VBW_EINVAL);
    c = good; c.len = 1000; expect(c, 0, 0, VBW_STREAM, VBW_EINVAL);
    c = good; c.len = 192 * 5; expect(c, 0, 0, VBW_STREAM, VBW_OK);
    CHECK(vbw_plan(nullptr, nullptr) == VBW_EINVAL);
    // twiddle tables: every size, symmetric and within half an ulp
    std::vector<float> tw(2 * 4096);
    for (int n = 2; n <= 4096; n *= 2) {
        CHECK(vbw_twiddle_table(n, tw.data()) == VBW_OK);
        for (int r = 0; r < n; ++r) {
            const double a = 2.0 * M_PI * r / n;
            CHECK(std::fabs(tw[2 * r] - std::cos(a)) <= 6e-8 && std::fabs(tw[2 * r + 1] + std::sin(a)) <= 6e-8);
        }
    }
    CHECK(vbw_twiddle_table(3, tw.data()) == VBW_EINVAL);
    for (int s = -6; s <= 0; ++s) CHECK(vbw_strerror(vbw_status(s)) != nullptr);
    std::printf("host plan checks: %d failures\n", failures);
    return failures ? 1 : 0;
}

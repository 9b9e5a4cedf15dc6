// Host logic of librsos.so (rsos_host.hpp: validation of initial heights,
// the overflow bound, W^2 of Eq. (2) from the exact sums, the serving
// engine's pool allocator) exercised under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Built with g++ by tests/test_sanitizers.py;
// any sanitizer report aborts the run, and every check prints its failure.
#include "rsos_host.hpp"

#include <cstdio>
#include <random>
#include <vector>

static int g_failed = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::printf("check failed at line %d: %s\n", __LINE__, #c);          \
            ++g_failed;                                                           \
        }                                                                         \
    } while (0)

int main()
{
    using namespace rsosh;
    // validate_h0: flat, a valid ramp, a restriction violation across the
    // periodic seam, out-of-range heights
    for (int L : {2, 3, 16, 64}) {
        std::vector<int32_t> h((size_t)L * L, 0);
        long long mx = -1, s1 = -1, s2 = -1;
        CHECK(validate_h0(h.data(), L, 1, &mx, &s1, &s2) == RSOS_OK);
        CHECK(mx == 0 && s1 == 0 && s2 == 0);
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) h[(size_t)y * L + x] = std::min(x, L - x) + std::min(y, L - y);
        long long e1 = 0, e2 = 0, em = 0;
        for (int32_t v : h) { e1 += v; e2 += (long long)v * v; em = std::max<long long>(em, v); }
        CHECK(validate_h0(h.data(), L, 1, &mx, &s1, &s2) == RSOS_OK);
        CHECK(mx == em && s1 == e1 && s2 == e2);
        h[(size_t)(L - 1) * L + L - 1] += 3;  // breaks bonds across both seams
        CHECK(validate_h0(h.data(), L, 1, &mx, &s1, &s2) == RSOS_E_RSOS);
        CHECK(validate_h0(h.data(), L, 4, &mx, &s1, &s2) == RSOS_OK);
        h[0] = -1;
        CHECK(validate_h0(h.data(), L, 1 << 30, &mx, &s1, &s2) == RSOS_E_INVAL);
        h[0] = 1 << 30;
        CHECK(validate_h0(h.data(), L, 1 << 30, &mx, &s1, &s2) == RSOS_E_INVAL);
    }
    // check_overflow: H = max_h0 + min(dt + N L, D^2 dt) against 2^31 and
    // L^2 H^2 against 2^63, with no intermediate overflow for extreme inputs
    rsos_params p = {16384, 1, 8, 0, 1};
    CHECK(check_overflow(p, 0, 2000) == RSOS_OK);
    CHECK(check_overflow(p, (1ll << 30) - 1, 1ll << 31) == RSOS_E_OVERFLOW);
    rsos_params q = {8192, 1, 8, 0, 1};
    CHECK(check_overflow(q, 0, 300000) == RSOS_OK);        // L H = 2^13 * 3.1e5 < 2^31.5
    CHECK(check_overflow(q, 0, 400000) == RSOS_E_OVERFLOW); // L^2 H^2 >= 2^63
    rsos_params r = {65536, 0x7FFFFFFF, 32, 0, 1};
    CHECK(check_overflow(r, (1ll << 30) - 1, 1ll << 32) == RSOS_E_OVERFLOW);
    CHECK(check_overflow(r, 0, 0) == RSOS_OK);
    // w2_of: exact int128 numerator, one rounding
    CHECK(w2_of(4, 0, 0) == 0.0);
    CHECK(w2_of(2, 2, 2) == 0.25);  // heights 1,1,0,0: mean 1/2, W^2 = 1/4
    CHECK(w2_of(65536, 1ll << 47, 1ll << 62) == 0.0);     // every height 2^15 on the largest lattice
    CHECK(w2_of(65536, (1ll << 47) - 1, (1ll << 62) - (1ll << 16) + 1) > 0.0);  // one site one lower
    // PoolAlloc: first fit, 256-byte rounding, coalescing on release
    PoolAlloc a;
    a.init(1 << 20);
    std::mt19937_64 rng(7);
    std::vector<std::pair<size_t, size_t>> live;
    for (int it = 0; it < 20000; ++it) {
        if (!live.empty() && (rng() % 3 == 0 || live.size() > 60)) {
            const size_t k = rng() % live.size();
            a.release(live[k].first, live[k].second);
            live.erase(live.begin() + (long)k);
        } else {
            const size_t n = 1 + rng() % 40000;
            size_t off = 0;
            if (a.alloc(n, &off)) {
                CHECK(off % kPoolAlign == 0 && off + n <= a.total);
                for (auto &pr : live) CHECK(off + n <= pr.first || pr.first + pr.second <= off);
                live.push_back({off, n});
            }
        }
    }
    for (auto &pr : live) a.release(pr.first, pr.second);
    CHECK(a.used == 0 && a.free_.size() == 1 && a.free_.begin()->second == a.total);
    std::printf("host checks done, %d failed\n", g_failed);
    return g_failed ? 1 : 0;
}

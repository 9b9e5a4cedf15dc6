/* The CPU oracle (oracle/rsos_ref.c) run under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every entry point on small lattices (several
 * tile sizes, restrictions, rough starts, all three schedules, the
 * random-sequential reference, injected choices, power sums), with the
 * invariants of the sweep checked along the way (restriction holds, the
 * accepted count equals the growth of sum h, the logged sums equal the
 * sums of the heights).  Built with gcc by tests/test_sanitizers.py; any
 * sanitizer report aborts the run. */
#include "rsos_ref.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int failed = 0;
#define CHECK(c)                                                       \
    do {                                                               \
        if (!(c)) {                                                    \
            printf("check failed at line %d: %s\n", __LINE__, #c);    \
            ++failed;                                                  \
        }                                                              \
    } while (0)

static void rough(int32_t *h, int L, int N, unsigned seed)
{
    /* a restricted start: a sum of two periodic ramps scaled by N */
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const int dx = (x + (int)seed) % L, dy = (y + 3 * (int)seed) % L;
            const int a = dx < L - dx ? dx : L - dx, b = dy < L - dy ? dy : L - dy;
            h[y * L + x] = 1000 + N * (a + b) / 2;
        }
}

static void check_run(const int32_t *h0, int L, int N, int D, int64_t n, int sched)
{
    int32_t *h = malloc(sizeof(int32_t) * L * L);
    int64_t *log = malloc(sizeof(int64_t) * 4 * n);
    memcpy(h, h0, sizeof(int32_t) * L * L);
    int64_t s10, s20;
    ref_sums(h, L, &s10, &s20);
    int rc = sched == 0 ? ref_run(h, L, N, D, 77, 5, n, log) : ref_run_dt(h, L, N, D, 77, 5, n, log);
    CHECK(rc == 0);
    int64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) acc += log[4 * i + 3];
    int64_t s1, s2;
    ref_sums(h, L, &s1, &s2);
    CHECK(ref_rsos_holds(h, L, N));
    CHECK(s1 == s10 + acc);
    CHECK(log[4 * (n - 1) + 1] == s1 && log[4 * (n - 1) + 2] == s2 && log[4 * (n - 1)] == 5 + n);
    free(h);
    free(log);
}

int main(void)
{
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    ref_philox4x32_10(ctr, key, out);
    int32_t f[16];
    for (int D = 2; D <= 32; D *= 2) CHECK(ref_word_fields(D, 0x12345678u, f) > 0);
    int32_t u[1024], v[1024];
    for (int D = 2; D <= 32; D *= 2) CHECK(ref_tile_sites(D, 99, 7, 1, 5, u, v) == 0);
    const int Ls[] = {4, 8, 16, 32, 64};
    for (int li = 0; li < 5; ++li) {
        const int L = Ls[li];
        int32_t *h0 = malloc(sizeof(int32_t) * L * L);
        for (int D = 2; D <= 32 && 2 * D <= L; D *= 2)
            for (int N = 1; N <= 3; ++N) {
                rough(h0, L, N, (unsigned)(L + D + N));
                CHECK(ref_rsos_holds(h0, L, N));
                check_run(h0, L, N, D, 6, 0);
                if (D == 8 || D == 16) check_run(h0, L, N, D, 4, 1);
            }
        free(h0);
    }
    /* threads and tile order do not change results */
    {
        const int L = 32, N = 2, D = 4;
        int32_t a[32 * 32], b[32 * 32];
        rough(a, L, N, 3);
        memcpy(b, a, sizeof a);
        ref_set_threads(0);
        ref_run(a, L, N, D, 11, 0, 5, NULL);
        ref_set_threads(4);
        ref_set_tile_order_seed(12345);
        ref_run(b, L, N, D, 11, 0, 5, NULL);
        ref_set_threads(0);
        ref_set_tile_order_seed(0);
        CHECK(memcmp(a, b, sizeof a) == 0);
    }
    /* injected choices, random-sequential, multisurface, power sums */
    {
        const int L = 8, N = 1, D = 2, n = 3, T = L / D;
        int32_t h[64] = {0}, origins[2 * 3], sites[3 * 2 * 8 * 4];
        for (int i = 0; i < 2 * n; ++i) origins[i] = i % (2 * D);
        for (int i = 0; i < n * 2 * (T * T / 2) * D * D; ++i) sites[i] = (i * 7) % (D * D);
        int64_t log[4 * 3];
        CHECK(ref_run_injected(h, L, N, D, n, origins, sites, log) == 0);
        CHECK(ref_rsos_holds(h, L, N));
        int32_t hr[64] = {0}, rs[2 * 200];
        for (int i = 0; i < 200; ++i) { rs[2 * i] = (i * 5) % L; rs[2 * i + 1] = (i * 3) % L; }
        CHECK(ref_rs_injected(hr, L, 2, 200, rs) > 0);
        int64_t rlog[4 * 4];
        CHECK(ref_rs_run(hr, L, 2, 9, 0, 4, rlog) == 0);
        CHECK(ref_rsos_holds(hr, L, 2));
        int64_t ps[8];
        ref_power_sums(hr, L, 3, ps);
        const int R = 4;
        int32_t *hm = calloc((size_t)R * 16 * 16, sizeof(int32_t));
        int64_t *mlog = malloc(sizeof(int64_t) * R * 3 * 4);
        CHECK(ref_run_ms(hm, R, 16, 1, 8, 5, 0, 3, mlog) == 0);
        for (int r = 0; r < R; ++r) CHECK(ref_rsos_holds(hm + r * 256, 16, 1));
        free(hm);
        free(mlog);
    }
    /* argument errors return codes, never touch memory */
    {
        int32_t h[16] = {0};
        CHECK(ref_run(h, 4, 1, 3, 1, 0, 1, NULL) != 0);
        CHECK(ref_run(h, 6, 1, 2, 1, 0, 1, NULL) != 0);
        h[0] = 5;
        CHECK(ref_run(h, 4, 1, 2, 1, 0, 1, NULL) != 0);
    }
    printf("oracle checks done, %d failed\n", failed);
    return failed ? 1 : 0;
}

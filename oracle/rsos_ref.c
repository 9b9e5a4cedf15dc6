/*
 * rsos_ref.c -- CPU oracle for the (2+1)-dimensional RSOS deposition sweep.
 *
 * TEST INFRASTRUCTURE ONLY (see rsos_ref.h).  Written for obviousness, not
 * speed: plain arrays, scalar loops, periodic indices by modulo, int64
 * arithmetic wherever a sum or difference is formed.  Optional OpenMP runs
 * the independent tiles of one phase on several threads; the result does
 * not depend on it (tiles of one colour touch only at corners).
 */
#include "rsos_ref.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;
static uint64_t g_order_seed = 0;

void ref_set_threads(int n) { g_threads = n < 0 ? 0 : n; }
void ref_set_tile_order_seed(uint64_t seed) { g_order_seed = seed; }

/* ---------------------------------------------------------------------------
 * Philox4x32-10, as published by Salmon, Moraes, Dror and Shaw (SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of the
 * Philox S-box on a 4-word counter under a 2-word key.  Each round takes
 * the two 64-bit products M0*x0 and M1*x2, and forms
 *   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0));
 * between rounds the key is bumped by the Weyl constants (W0, W1).
 * ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void seed_to_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(seed >> 32);
}

static int log2_exact(int D)
{
    int b = 0;
    while ((1 << b) < D) ++b;
    return ((1 << b) == D) ? b : -1;
}

static int valid_D(int D) { return D == 2 || D == 4 || D == 8 || D == 16 || D == 32; }

/* Sec. II: "after each lattice sweep the origin of the DD was moved
 * randomly"; read as a uniform shift over one period of the colouring. */
void ref_origin(int D, uint64_t seed, uint32_t s, int32_t *ox, int32_t *oy)
{
    uint32_t key[2], ctr[4] = {0u, 0u, s, 2u}, r[4];
    seed_to_key(seed, key);
    ref_philox4x32_10(ctr, key, r);
    *ox = (int32_t)(r[0] % (uint32_t)(2 * D));
    *oy = (int32_t)(r[1] % (uint32_t)(2 * D));
}

int ref_word_fields(int D, uint32_t word, int32_t *fields)
{
    if (!valid_D(D)) return -1;
    int b = 2 * log2_exact(D);
    int f = 32 / b;
    uint32_t mask = (uint32_t)(D * D - 1);
    for (int k = 0; k < f; ++k) fields[k] = (int32_t)((word >> (k * b)) & mask);
    return f;
}

/* The in-tile sites of one tile-phase: uniform with replacement over the D*D
 * sites of the domain (random-sequential inside a domain). */
int ref_tile_sites(int D, uint64_t seed, uint32_t s, uint32_t p, uint32_t tile_id,
                   int32_t *u, int32_t *v)
{
    if (!valid_D(D)) return -1;
    uint32_t key[2];
    seed_to_key(seed, key);
    int b = 2 * log2_exact(D);
    int f = 32 / b;
    int per_call = 4 * f;
    uint32_t r[4] = {0, 0, 0, 0};
    int32_t fields[16];
    for (int a = 0; a < D * D; ++a) {
        if (a % per_call == 0) {
            uint32_t ctr[4] = {(uint32_t)(a / per_call), tile_id, s, p};
            ref_philox4x32_10(ctr, key, r);
        }
        int w = (a % per_call) / f;
        int k = a % f;
        if (k == 0) ref_word_fields(D, r[w], fields);
        u[a] = fields[k] % D;
        v[a] = fields[k] / D;
    }
    return 0;
}

static int wrap(int64_t a, int L)
{
    int64_t m = a % L;
    return (int)(m < 0 ? m + L : m);
}

static int64_t absd(int64_t a) { return a < 0 ? -a : a; }

/* The RSOS rule: deposit at (x, y) only if afterwards the height difference
 * to every nearest neighbour is at most N in magnitude. */
int ref_attempt(int32_t *h, int L, int N, int x, int y)
{
    int64_t after = (int64_t)h[(int64_t)y * L + x] + 1;
    const int nx[4] = {wrap(x + 1, L), wrap(x - 1, L), x, x};
    const int ny[4] = {y, y, wrap(y + 1, L), wrap(y - 1, L)};
    for (int j = 0; j < 4; ++j) {
        int64_t nb = h[(int64_t)ny[j] * L + nx[j]];
        if (absd(after - nb) > (int64_t)N) return 0;
    }
    h[(int64_t)y * L + x] = (int32_t)after;
    return 1;
}

int ref_rsos_holds(const int32_t *h, int L, int N)
{
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            int64_t c = h[(int64_t)y * L + x];
            if (absd(c - h[(int64_t)y * L + wrap(x + 1, L)]) > N) return 0;
            if (absd(c - h[(int64_t)wrap(y + 1, L) * L + x]) > N) return 0;
        }
    return 1;
}

/* Eq. (2) needs sum h and sum h^2 over the L^2 sites. */
void ref_sums(const int32_t *h, int L, int64_t *s1, int64_t *s2)
{
    int64_t a = 0, b = 0;
    for (int64_t i = 0; i < (int64_t)L * L; ++i) {
        a += h[i];
        b += (int64_t)h[i] * h[i];
    }
    *s1 = a;
    *s2 = b;
}

void ref_power_sums(const int32_t *h, int L, int64_t R, int64_t out[8])
{
    __int128 c[4] = {0, 0, 0, 0};
    for (int64_t i = 0; i < (int64_t)L * L; ++i) {
        const __int128 x = (__int128)h[i] - R;
        __int128 p = x;
        for (int k = 0; k < 4; ++k) {
            c[k] += p;
            p *= x;
        }
    }
    for (int k = 0; k < 4; ++k) {
        const unsigned __int128 u = (unsigned __int128)c[k];
        out[2 * k] = (int64_t)(uint64_t)u;
        out[2 * k + 1] = (int64_t)(uint64_t)(u >> 64);
    }
}

static int check_args(int L, int N, int D)
{
    if (!valid_D(D) || L <= 0 || N < 1) return -1;
    if (L % (2 * D) != 0) return -1;
    return 0;
}

/* One tile of colour p: D*D attempts at the given in-tile sites. */
static int64_t tile_update(int32_t *h, int L, int N, int D, int ox, int oy, int tx, int ty,
                           const int32_t *u, const int32_t *v)
{
    int64_t acc = 0;
    for (int a = 0; a < D * D; ++a) {
        int x = wrap((int64_t)ox + (int64_t)tx * D + u[a], L);
        int y = wrap((int64_t)oy + (int64_t)ty * D + v[a], L);
        acc += ref_attempt(h, L, N, x, y);
    }
    return acc;
}

static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Tiles of colour p, listed in increasing tile_id, optionally permuted. */
static int32_t *phase_tiles(int T, int p, uint64_t order_seed, uint32_t s, int64_t *count)
{
    int64_t n = (int64_t)T * T / 2, k = 0;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int ty = 0; ty < T; ++ty)
        for (int tx = 0; tx < T; ++tx)
            if (((tx + ty) & 1) == p) ids[k++] = ty * T + tx;
    if (order_seed != 0) {
        uint64_t st = order_seed ^ ((uint64_t)s << 1) ^ (uint64_t)p;
        for (int64_t i = k - 1; i > 0; --i) {
            int64_t j = (int64_t)(splitmix64(&st) % (uint64_t)(i + 1));
            int32_t t = ids[i]; ids[i] = ids[j]; ids[j] = t;
        }
    }
    *count = k;
    return ids;
}

/* One sweep of the tile-checkerboard schedule.  Returns accepted count. */
static int64_t sweep_once(int32_t *h, int L, int N, int D, uint64_t seed, uint32_t s,
                          const int32_t *inj_origin, const int32_t *inj_sites)
{
    int T = L / D;
    int32_t ox, oy;
    if (inj_origin) { ox = inj_origin[0]; oy = inj_origin[1]; }
    else ref_origin(D, seed, s, &ox, &oy);
    int64_t accepted = 0;
    for (int p = 0; p < 2; ++p) {
        int64_t n;
        int32_t *ids = phase_tiles(T, p, inj_sites ? 0 : g_order_seed, s, &n);
        int nthreads = g_threads;
#ifdef _OPENMP
        if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : accepted) num_threads(nthreads)
#endif
        for (int64_t i = 0; i < n; ++i) {
            int32_t u[1024], v[1024];
            int tid = ids[i];
            int tx = tid % T, ty = tid / T;
            if (inj_sites) {
                /* injected choices are listed in increasing tile_id order,
                 * which is the (unpermuted) order of ids[] */
                const int32_t *r = inj_sites + ((int64_t)p * n + i) * D * D;
                for (int a = 0; a < D * D; ++a) { u[a] = r[a] % D; v[a] = r[a] / D; }
            } else {
                ref_tile_sites(D, seed, s, (uint32_t)p, (uint32_t)tid, u, v);
            }
            accepted += tile_update(h, L, N, D, ox, oy, tx, ty, u, v);
        }
        (void)nthreads;
        free(ids);
    }
    return accepted;
}

int ref_run(int32_t *h, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n,
            int64_t *log)
{
    if (check_args(L, N, D) != 0 || t0 < 0 || n < 0) return -1;
    if (t0 + n > (int64_t)UINT32_MAX + 1) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t s = (uint32_t)(t0 + i);
        int64_t a = sweep_once(h, L, N, D, seed, s, NULL, NULL);
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = (int64_t)s + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

int ref_run_injected(int32_t *h, int L, int N, int D, int64_t n,
                     const int32_t *origins, const int32_t *sites, int64_t *log)
{
    if (check_args(L, N, D) != 0 || n < 0) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    int64_t per_sweep = (int64_t)L * L; /* both phases: T*T tiles of D*D sites */
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = sweep_once(h, L, N, D, 0, (uint32_t)i, origins + 2 * i,
                               sites + i * per_sweep);
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = i + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Double tiling (Sec. II): tiles of 2D x 2D split into 2 x 2 sub-tiles of
 * D x D; the sub-tiles fall into 4 sets by their position in the tile,
 * set k = (sx mod 2) + 2 (sy mod 2) for sub-tile (sx, sy) of the shifted
 * frame, updated set 0, 1, 2, 3 in turn.  Sub-tiles of one set are separated
 * by one sub-tile in each direction, so they are independent.  Sub-tile
 * sub_id = sy*(L/D) + sx of set k takes its D*D sites from Philox counters
 * (j, sub_id, s, 4 + k) (phase codes 4..7 stay clear of the origin's tag 2).
 * The origin is drawn as in the checkerboard schedule, mod 2D.
 * --------------------------------------------------------------------- */
static int32_t *set_subtiles(int T, int k, int64_t *count)
{
    int64_t n = (int64_t)T * T / 4, c = 0;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int sy = 0; sy < T; ++sy)
        for (int sx = 0; sx < T; ++sx)
            if ((sx & 1) + 2 * (sy & 1) == k) ids[c++] = sy * T + sx;
    *count = c;
    return ids;
}

static int64_t sweep_once_dt(int32_t *h, int L, int N, int D, uint64_t seed, uint32_t s,
                             const int32_t *inj_origin, const int32_t *inj_sites)
{
    int T = L / D;
    int32_t ox, oy;
    if (inj_origin) { ox = inj_origin[0]; oy = inj_origin[1]; }
    else ref_origin(D, seed, s, &ox, &oy);
    int64_t accepted = 0;
    for (int k = 0; k < 4; ++k) {
        int64_t n;
        int32_t *ids = set_subtiles(T, k, &n);
        int nthreads = g_threads;
#ifdef _OPENMP
        if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : accepted) num_threads(nthreads)
#endif
        for (int64_t i = 0; i < n; ++i) {
            int32_t u[1024], v[1024];
            int sid = ids[i];
            int sx = sid % T, sy = sid / T;
            if (inj_sites) {
                const int32_t *r = inj_sites + ((int64_t)k * n + i) * D * D;
                for (int a = 0; a < D * D; ++a) { u[a] = r[a] % D; v[a] = r[a] / D; }
            } else {
                ref_tile_sites(D, seed, s, (uint32_t)(4 + k), (uint32_t)sid, u, v);
            }
            accepted += tile_update(h, L, N, D, ox, oy, sx, sy, u, v);
        }
        (void)nthreads;
        free(ids);
    }
    return accepted;
}

int ref_run_dt(int32_t *h, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n, int64_t *log)
{
    if (check_args(L, N, D) != 0 || t0 < 0 || n < 0) return -1;
    if (t0 + n > (int64_t)UINT32_MAX + 1) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t s = (uint32_t)(t0 + i);
        int64_t a = sweep_once_dt(h, L, N, D, seed, s, NULL, NULL);
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = (int64_t)s + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

int ref_run_dt_injected(int32_t *h, int L, int N, int D, int64_t n, const int32_t *origins,
                        const int32_t *sites, int64_t *log)
{
    if (check_args(L, N, D) != 0 || n < 0) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    int64_t per_sweep = (int64_t)L * L;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = sweep_once_dt(h, L, N, D, 0, (uint32_t)i, origins + 2 * i, sites + i * per_sweep);
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = i + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Multisurface lock-step (Sec. II): R realizations share one sequence of
 * selected sites, and each realization applies each selection only with
 * probability 1/2 (its own coin), which breaks the correlation between
 * them.  A sweep makes 2 D^2 selections per tile and phase, so every
 * realization receives L^2 attempts per sweep on average.  Selection a of
 * tile tile_id in phase p of sweep s takes its site field from Philox
 * (j, tile_id, s, p) with the checkerboard layout, a in [0, 2 D^2);
 * realization r's coin is bit (a mod 32) of word (a div 32) mod 4 of Philox
 * (a div 128, tile_id, s, 8 + 2r + p).  Origin and colours as for the
 * checkerboard.
 * --------------------------------------------------------------------- */
static void tile_fields(int D, uint64_t seed, uint32_t s, uint32_t p, uint32_t tile_id, int count,
                        int32_t *u, int32_t *v)
{
    uint32_t key[2];
    seed_to_key(seed, key);
    int b = 2 * log2_exact(D);
    int f = 32 / b;
    int per_call = 4 * f;
    uint32_t r[4] = {0, 0, 0, 0};
    int32_t fields[16];
    for (int a = 0; a < count; ++a) {
        if (a % per_call == 0) {
            uint32_t ctr[4] = {(uint32_t)(a / per_call), tile_id, s, p};
            ref_philox4x32_10(ctr, key, r);
        }
        int w = (a % per_call) / f;
        int k = a % f;
        if (k == 0) ref_word_fields(D, r[w], fields);
        u[a] = fields[k] % D;
        v[a] = fields[k] / D;
    }
}

static int ms_coin(uint64_t seed, uint32_t s, uint32_t p, uint32_t tile_id, int r, int a)
{
    uint32_t key[2], out[4];
    seed_to_key(seed, key);
    uint32_t ctr[4] = {(uint32_t)(a / 128), tile_id, s, 8u + 2u * (uint32_t)r + p};
    ref_philox4x32_10(ctr, key, out);
    return (int)((out[(a / 32) % 4] >> (a % 32)) & 1u);
}

/* One sweep of one realization; choices from the seed, or injected
 * (inj_sites: per phase, tiles of that colour in increasing tile_id, 2 D^2
 * in-tile indices each; inj_coins: the same positions, 0 or 1). */
static int64_t sweep_once_ms(int32_t *h, int L, int N, int D, uint64_t seed, uint32_t s, int r,
                             const int32_t *inj_origin, const int32_t *inj_sites,
                             const int32_t *inj_coins)
{
    int T = L / D;
    int32_t ox, oy;
    if (inj_origin) { ox = inj_origin[0]; oy = inj_origin[1]; }
    else ref_origin(D, seed, s, &ox, &oy);
    int64_t accepted = 0;
    const int sel = 2 * D * D;
    for (int p = 0; p < 2; ++p) {
        int64_t n;
        int32_t *ids = phase_tiles(T, p, 0, s, &n);
        for (int64_t i = 0; i < n; ++i) {
            int32_t u[2048], v[2048];
            int tid = ids[i];
            int tx = tid % T, ty = tid / T;
            if (inj_sites) {
                const int32_t *q = inj_sites + ((int64_t)p * n + i) * sel;
                for (int a = 0; a < sel; ++a) { u[a] = q[a] % D; v[a] = q[a] / D; }
            } else {
                tile_fields(D, seed, s, (uint32_t)p, (uint32_t)tid, sel, u, v);
            }
            for (int a = 0; a < sel; ++a) {
                int coin = inj_coins ? inj_coins[((int64_t)p * n + i) * sel + a]
                                     : ms_coin(seed, s, (uint32_t)p, (uint32_t)tid, r, a);
                if (!coin) continue;
                int x = wrap((int64_t)ox + (int64_t)tx * D + u[a], L);
                int y = wrap((int64_t)oy + (int64_t)ty * D + v[a], L);
                accepted += ref_attempt(h, L, N, x, y);
            }
        }
        free(ids);
    }
    return accepted;
}

int ref_run_ms(int32_t *h, int R, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n,
               int64_t *log)
{
    if (check_args(L, N, D) != 0 || R < 1 || t0 < 0 || n < 0) return -1;
    if (t0 + n > (int64_t)UINT32_MAX + 1) return -1;
    for (int r = 0; r < R; ++r)
        if (!ref_rsos_holds(h + (int64_t)r * L * L, L, N)) return -2;
    int nthreads = g_threads;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int r = 0; r < R; ++r) {
        int32_t *hr = h + (int64_t)r * L * L;
        for (int64_t i = 0; i < n; ++i) {
            uint32_t s = (uint32_t)(t0 + i);
            int64_t a = sweep_once_ms(hr, L, N, D, seed, s, r, NULL, NULL, NULL);
            if (log) {
                int64_t s1, s2;
                ref_sums(hr, L, &s1, &s2);
                int64_t *e = log + 4 * ((int64_t)r * n + i);
                e[0] = (int64_t)s + 1;
                e[1] = s1;
                e[2] = s2;
                e[3] = a;
            }
        }
    }
    (void)nthreads;
    return 0;
}

int ref_run_ms_injected(int32_t *h, int L, int N, int D, int64_t n, const int32_t *origins,
                        const int32_t *sites, const int32_t *coins, int64_t *log)
{
    if (check_args(L, N, D) != 0 || n < 0) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    int64_t per_sweep = 2 * (int64_t)L * L;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = sweep_once_ms(h, L, N, D, 0, (uint32_t)i, 0, origins + 2 * i, sites + i * per_sweep,
                                  coins + i * per_sweep);
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = i + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

/* Uniform integer in [0, n) from SplitMix64 by rejection (exactly uniform). */
static uint32_t uniform_below(uint64_t *st, uint32_t n)
{
    uint64_t limit = UINT64_MAX - (UINT64_MAX % n);
    uint64_t z;
    do { z = splitmix64(st); } while (z >= limit);
    return (uint32_t)(z % n);
}

int ref_rs_run(int32_t *h, int L, int N, uint64_t rs_seed, int64_t t0, int64_t n,
               int64_t *log)
{
    if (L <= 0 || N < 1 || n < 0) return -1;
    if (!ref_rsos_holds(h, L, N)) return -2;
    uint64_t st = rs_seed;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = 0;
        for (int64_t k = 0; k < (int64_t)L * L; ++k) {
            int x = (int)uniform_below(&st, (uint32_t)L);
            int y = (int)uniform_below(&st, (uint32_t)L);
            a += ref_attempt(h, L, N, x, y);
        }
        if (log) {
            int64_t s1, s2;
            ref_sums(h, L, &s1, &s2);
            log[4 * i + 0] = t0 + i + 1;
            log[4 * i + 1] = s1;
            log[4 * i + 2] = s2;
            log[4 * i + 3] = a;
        }
    }
    return 0;
}

int64_t ref_rs_injected(int32_t *h, int L, int N, int64_t n_attempts, const int32_t *sites)
{
    int64_t a = 0;
    for (int64_t k = 0; k < n_attempts; ++k) a += ref_attempt(h, L, N, sites[2 * k], sites[2 * k + 1]);
    return a;
}

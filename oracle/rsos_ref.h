/*
 * rsos_ref.h -- CPU oracle for the (2+1)-dimensional RSOS deposition sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plainly written CPU
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * library never links, includes or calls anything here, and nothing here is
 * shared with the product (no common headers, kernels, tables or helpers).
 *
 * Model (Kelling, Odor & Gemming, "Universality of (2+1)-dimensional
 * restricted solid-on-solid models", Sec. I and Sec. II):
 *   - an L x L periodic square lattice of integer heights h, flat start;
 *   - deposition h_i -> h_i + 1 at a randomly chosen site, accepted only if
 *     afterwards |h_i - h_j| <= N for each of the 4 nearest neighbours j
 *     (the RSOS restriction, Sec. I, the equation after the KPZ discussion);
 *   - time in Monte-Carlo steps: one sweep = L*L attempts (Sec. II);
 *   - squared width W^2(L,t), Eq. (2).
 *
 * Parallel schedule (the "tile checkerboard" reading of the paper's domain
 * decomposition, Sec. II: domains of D x D sites, origin moved randomly
 * after each sweep, independent sets of domains updated by independent
 * workers).  One sweep s (0-based; t = s+1 afterwards):
 *   1. key  = (seed mod 2^32, seed >> 32);
 *   2. origin: Philox4x32-10 at counter (0, 0, s, 2); ox = r0 mod 2D,
 *      oy = r1 mod 2D;
 *   3. shifted frame x' = (x - ox) mod L, y' = (y - oy) mod L; tile
 *      (tx, ty) = (x'/D, y'/D), tile_id = ty*(L/D) + tx, colour (tx+ty) mod 2;
 *   4. phase p = 0 then 1: every tile of colour p makes D*D attempts in
 *      order; attempt a uses Philox call j = a / (4f) at counter
 *      (j, tile_id, s, p), word w = (a mod 4f) / f, field k = a mod f of
 *      b = 2 log2(D) bits (f = floor(32/b) fields per word); the field value
 *      r gives the in-tile site (u, v) = (r mod D, r / D), real site
 *      ((ox + tx D + u) mod L, (oy + ty D + v) mod L);
 *   5. after the sweep: S1 = sum h, S2 = sum h^2 (int64), A = accepted.
 *
 * Conventions: all arrays are host memory, row-major, index y*L + x.
 * Functions return 0 on success and a negative code on invalid arguments
 * (-1 invalid size/parameter, -2 RSOS violation in the input heights).
 */
#ifndef RSOS_REF_H
#define RSOS_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block function (Salmon et al., SC'11): out = f_key(ctr). */
void ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Sweep origin (ox, oy) in [0, 2D)^2 for sweep s. */
void ref_origin(int D, uint64_t seed, uint32_t s, int32_t *ox, int32_t *oy);

/* The D*D in-tile sites (u[a], v[a]) of tile tile_id in phase p of sweep s. */
int ref_tile_sites(int D, uint64_t seed, uint32_t s, uint32_t p, uint32_t tile_id,
                   int32_t *u, int32_t *v);

/* Split one 32-bit word into its f fields of b = 2 log2(D) bits, low first. */
int ref_word_fields(int D, uint32_t word, int32_t *fields);

/* One deposition attempt at (x, y) under restriction N; returns 1 if accepted. */
int ref_attempt(int32_t *h, int L, int N, int x, int y);

/* Checks |h_i - h_j| <= N on every nearest-neighbour bond; 1 if it holds. */
int ref_rsos_holds(const int32_t *h, int L, int N);

/* Sum h and sum h^2 over the lattice, in int64. */
void ref_sums(const int32_t *h, int L, int64_t *s1, int64_t *s2);

/* Power sums about an integer reference R for the height-distribution
 * moments of Eqs. (13)-(15): C_k = sum over sites of (h - R)^k, k = 1..4,
 * accumulated exactly in 128-bit integers.  out[2k-2], out[2k-1] receive the
 * low and high 64-bit halves of C_k (two's complement). */
void ref_power_sums(const int32_t *h, int L, int64_t R, int64_t out[8]);

/* Tile-checkerboard sweeps s = t0 .. t0+n-1 in place.  log (may be NULL)
 * receives 4 int64 per sweep: (t = s+1, S1, S2, A). */
int ref_run(int32_t *h, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n,
            int64_t *log);

/* Same, from injected choices instead of Philox: origins[2*i..] gives the
 * origin of sweep i, sites[] gives, for sweep i, phase p, the tiles of
 * colour p in increasing tile_id order, D*D in-tile indices r = v*D + u each. */
int ref_run_injected(int32_t *h, int L, int N, int D, int64_t n,
                     const int32_t *origins, const int32_t *sites, int64_t *log);

/* Plain random-sequential RSOS (the model's own definition), n sweeps of L*L
 * attempts at uniformly drawn sites, driven by a SplitMix64 stream seeded
 * with rs_seed.  log as in ref_run (t counts sweeps from t0). */
int ref_rs_run(int32_t *h, int L, int N, uint64_t rs_seed, int64_t t0, int64_t n,
               int64_t *log);

/* Random-sequential attempts at injected sites (x = sites[2a], y = sites[2a+1]). */
int64_t ref_rs_injected(int32_t *h, int L, int N, int64_t n_attempts, const int32_t *sites);

/* Schedule knobs that must not change results: OpenMP threads (0 = serial)
 * and a seed for a random permutation of the tile order inside a phase
 * (0 = increasing tile_id). */
/* The double-tiling schedule (Sec. II: 2 x 2 sub-tiles per tile, 4 sets
 * updated in turn; see rsos_ref.c).  Same arguments, log and return codes
 * as ref_run / ref_run_injected; injected sites list, per sweep and set,
 * the sub-tiles of that set in increasing sub_id, D*D in-tile indices each. */
int ref_run_dt(int32_t *h, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n, int64_t *log);
int ref_run_dt_injected(int32_t *h, int L, int N, int D, int64_t n, const int32_t *origins,
                        const int32_t *sites, int64_t *log);

/* Multisurface lock-step (Sec. II; see rsos_ref.c): R realizations sharing
 * one site sequence, each applying each selection with probability 1/2;
 * 2 D^2 selections per tile and phase.  h holds the R lattices one after
 * another (realization-major); log is int64[R][n][4] (t, S1, S2, A).  The
 * injected variant runs one realization along given origins, sites (per
 * sweep and phase, tiles of that colour in increasing tile_id, 2 D^2
 * in-tile indices each) and coins (0/1 at the same positions). */
int ref_run_ms(int32_t *h, int R, int L, int N, int D, uint64_t seed, int64_t t0, int64_t n,
               int64_t *log);
int ref_run_ms_injected(int32_t *h, int L, int N, int D, int64_t n, const int32_t *origins,
                        const int32_t *sites, const int32_t *coins, int64_t *log);

void ref_set_threads(int n);
void ref_set_tile_order_seed(uint64_t seed);

#ifdef __cplusplus
}
#endif
#endif

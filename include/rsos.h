/*
 * rsos.h -- C ABI of librsos.so, the gfx950 RSOS deposition sweep.
 *
 * The library simulates restricted solid-on-solid (RSOS) growth on an
 * L x L periodic square lattice of int32 heights (Kelling, Odor & Gemming,
 * "Universality of (2+1)-dimensional restricted solid-on-solid models"):
 *
 *   - deposition h_i -> h_i + 1 at a randomly chosen site is accepted only
 *     if afterwards |h_i - h_j| <= N for all 4 nearest neighbours j
 *     (the RSOS restriction, Sec. I);
 *   - time is counted in Monte-Carlo steps, one sweep = L*L attempts,
 *     starting from a flat surface (Sec. II);
 *   - the attempts are scheduled by a domain decomposition into D x D tiles
 *     whose origin moves randomly after each sweep (Sec. II): tiles are
 *     coloured like a checkerboard, colour 0 is updated, then colour 1, and
 *     each tile makes D*D sequential uniform attempts inside itself;
 *   - after every sweep the library records S1 = sum h, S2 = sum h^2 and
 *     the accepted count A (exact int64), from which the squared width
 *     W^2(L, t) of Eq. (2) follows.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed
 * (key = (seed mod 2^32, seed >> 32)); sweep s (0-based) draws its origin
 * from counter (0, 0, s, 2), ox = r0 mod 2D, oy = r1 mod 2D; tile tile_id =
 * ty*(L/D) + tx of the shifted frame in phase p draws its D*D in-tile sites
 * from counters (j, tile_id, s, p), j = 0, 1, ..., splitting each output
 * word into floor(32/b) fields of b = 2 log2(D) bits, lowest field first;
 * field r is the site (r mod D, r / D) of the tile.  A trajectory is a
 * function of (L, N, D, seed, initial heights, t0, number of sweeps) only:
 * never of launch shapes, batching, streams or timing.
 *
 * Memory: heights are int32, row-major (index y*L + x), in device memory
 * owned by the caller.  Each surface needs two such buffers (the sweep reads
 * one and writes the other); after t sweeps the current state is in the
 * buffer of parity t (bufs[t & 1] with bufs = {d_h, d_work}).  The library
 * owns only small device buffers of its own (per-sweep log, partial sums).
 *
 * Errors: every function returns an rsos_status; nothing aborts and no C++
 * exception crosses this boundary.  rsos_last_error() gives a thread-local
 * message for the last failure.  After a HIP runtime error a handle is
 * failed for good and later calls return RSOS_E_STATE.  Handles are not
 * thread-safe; distinct handles on distinct streams are independent.
 */
#ifndef RSOS_H
#define RSOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSOS_OK = 0,
    RSOS_E_INVAL = -1,    /* invalid argument (size, pointer, range)          */
    RSOS_E_RSOS = -2,     /* initial heights violate |h_i - h_j| <= N          */
    RSOS_E_OVERFLOW = -3, /* heights or sum h^2 could leave int32 / int64     */
    RSOS_E_DEVICE = -4,   /* HIP runtime error (handle becomes failed)        */
    RSOS_E_NOMEM = -5,    /* library-owned device or host allocation failed   */
    RSOS_E_STATE = -6,    /* handle failed earlier, or call out of sequence   */
    RSOS_E_BUSY = -7      /* serving engine: no room for this job right now   */
} rsos_status;

/* Parameters of one surface.
 *   L     lattice side, a multiple of 2*D, 2*D <= L <= 65536;
 *   N     step restriction of Sec. I, N >= 1 (INT32_MAX: no restriction);
 *   D     tile side of the domain decomposition, one of 2, 4, 8, 16, 32
 *         (the paper uses 8 x 8 domains, Sec. II, and tests 16 x 16,
 *         Sec. III.C); part of the result;
 *   flags 0, RSOS_FLAG_PACKED16 (storage only: results are identical) or
 *         RSOS_FLAG_DT4 (the double-tiling schedule), optionally or-ed with
 *         RSOS_FLAG_TUNE (launch choices from the autotuner; results are
 *         identical);
 *   seed  64-bit Philox key. */
typedef struct {
    int32_t L;
    int32_t N;
    int32_t D;
    int32_t flags;
    uint64_t seed;
} rsos_params;

/* Heights kept in device memory as 16-bit residues mod 2^16 (half the HBM
 * bytes of a sweep).  Exact: on the torus the restriction keeps every height
 * within N*L of every other, and the mean moves by at most one per sweep, so
 * the residue and floor(S1 / L^2) determine each height.  Requires
 * N*L <= 32766, N*D <= 96, L^2 * 4 > 64 KiB (the tile-block path) and a
 * tile-block shape for L (RSOS_E_INVAL otherwise).  Single surfaces and
 * batches; the serving engine keeps int32.  Buffer roles change: d_h (or a
 * batch surface's slice of d_pool) holds both residue buffers, and d_work
 * (or d_work_pool) is the int32 scratch that rsos_heights converts into
 * before a host copy (and that receives h0_host at init).  rsos_time's
 * d_current is NULL in this mode. */
#define RSOS_FLAG_PACKED16 1

/* The paper's double-tiling schedule (Sec. II) instead of the tile
 * checkerboard: tiles of 2D x 2D split into 2 x 2 sub-tiles of D x D, the 4
 * sets of sub-tiles (by position in the tile, set = (sx mod 2) + 2 (sy mod
 * 2)) updated in turn; sub-tile sub_id of set k draws its sites from Philox
 * counters (j, sub_id, s, 4 + k); origin as for the checkerboard.  A
 * different (equally valid) dynamics: results differ from the checkerboard
 * schedule.  D must be 8 or 16; int32 storage only (not combined with
 * RSOS_FLAG_PACKED16); single surfaces and batches. */
#define RSOS_FLAG_DT4 2

/* Launch choices from the autotuner (see rsos_tune below) instead of the
 * first tile-block variant that fits.  Changes speed only, never results.
 * The environment variable RSOS_TUNE=1 sets it for every handle. */
#define RSOS_FLAG_TUNE 4

/* One record of the per-sweep log: the state after t sweeps.
 *   s1 = sum h, s2 = sum h^2 (exact), accepted = accepted attempts of sweep
 *   t (0 for the initial state), w2 = W^2(L, t) of Eq. (2) evaluated as
 *   (L^2 s2 - s1^2) / L^4 from the exact int128 numerator (one rounding to
 *   double when L is a power of two). */
typedef struct {
    int64_t t;
    int64_t s1;
    int64_t s2;
    int64_t accepted;
    double w2;
} rsos_width_t;

/* Moments of the height distribution of one state (the moments of Eqs.
 * (13)-(15) whose averages over samples give the skewness S_h and kurtosis
 * Q_h of the heights).  Exact power sums about the integer reference
 * ref = floor(S1 / L^2):
 *   c1 = sum (h - ref), c2 = sum (h - ref)^2,
 *   c3 = sum (h - ref)^3, c4 = sum (h - ref)^4 as 128-bit two's complement
 *   integers, [0] the low 64 bits, [1] the high 64 bits;
 * and the central moments per site (about the mean S1 / L^2)
 *   phi2 = W^2, phi3, phi4, evaluated from the exact sums in long double. */
typedef struct {
    int64_t t;
    int64_t ref;
    int64_t c1;
    int64_t c2;
    uint64_t c3[2];
    uint64_t c4[2];
    double phi2;
    double phi3;
    double phi4;
} rsos_moments_t;

typedef struct rsos_surface rsos_surface;
typedef struct rsos_batch rsos_batch;
typedef struct rsos_engine rsos_engine;

/* --------------------------------------------------------------------- */
/* Single surface (the plain one-surface path).                            */
/* --------------------------------------------------------------------- */

/* Creates a surface handle.
 *   out       receives the handle;
 *   p         parameters (validated here: RSOS_E_INVAL);
 *   d_h       caller-owned device int32[L*L]; must outlive the handle;
 *   d_work    caller-owned device int32[L*L], the second buffer; NULL makes
 *             the library allocate (and later free) its own;
 *   h0_host   host int32[L*L] initial heights, 0 <= h < 2^30, checked for
 *             the restriction (RSOS_E_RSOS); NULL means flat h = 0 (Sec. II);
 *   t0        sweeps already done (resume from a checkpoint), 0 <= t0 < 2^32;
 *   log_cap   sweeps kept in the device log ring (0 = 65536);
 *   stream    hipStream_t the surface works on (NULL = default stream).
 * The initial state is copied into the buffer of parity t0. */
rsos_status rsos_init(rsos_surface **out, const rsos_params *p, int32_t *d_h, int32_t *d_work,
                      const int32_t *h0_host, int64_t t0, int64_t log_cap, void *stream);

/* Enqueues n_mcs Monte-Carlo sweeps (Sec. II: one sweep = L*L attempted
 * depositions, here D*D per tile of each checkerboard colour) asynchronously
 * on the surface's stream; t += n_mcs.  n_mcs = 0 does nothing; n_mcs < 0
 * or t + n_mcs > 2^32 gives RSOS_E_INVAL.  Checks the overflow bound
 * H = max(h0) + min(t + N L, D^2 t) < 2^31 and L^2 H^2 < 2^63 before
 * enqueuing anything (RSOS_E_OVERFLOW: no device work, t unchanged).  Each
 * sweep is one kernel launch (runs of them replayed as hipGraphs when the
 * surface has a stream; the graph is captured by rsos_init, never inside
 * rsos_sweep); the exact sums of the sweep are part of it. */
rsos_status rsos_sweep(rsos_surface *s, int64_t n_mcs);

/* Synchronises the stream and returns the record of the current time t:
 * S1, S2, the accepted count and W^2(L, t) of Eq. (2). */
rsos_status rsos_width(rsos_surface *s, rsos_width_t *out);

/* Synchronises and returns records t_from .. t_from+n-1 (t_from >= t0).
 * Records older than log_cap sweeps before the current time are gone
 * (RSOS_E_INVAL). */
rsos_status rsos_log(rsos_surface *s, int64_t t_from, int64_t n, rsos_width_t *out);

/* Synchronises and copies the current heights (int32[L*L]) to dst, host or
 * device memory as dst_is_device says. */
rsos_status rsos_heights(rsos_surface *s, int32_t *dst, int dst_is_device);

/* Synchronises and computes the height-distribution moments of the current
 * state on the device (one read of the lattice: two kernels on the
 * surface's stream).  Exact for every state the library accepts. */
rsos_status rsos_moments(rsos_surface *s, rsos_moments_t *out);

/* Current time t and the device buffer that holds the current int32 state
 * (NULL with RSOS_FLAG_PACKED16). */
rsos_status rsos_time(rsos_surface *s, int64_t *t, int32_t **d_current);

/* Kernel timing.  While enabled, every sweep's tile-block kernels are
 * launched with HIP events on the surface's stream that the runtime records
 * when the first kernel starts and the last one ends (hipExtLaunchKernel;
 * sweeps are then issued one by one, not as hipGraph replays).  rsos_timing_read
 * synchronises and returns the number of timed launches and their mean and
 * total duration in milliseconds; it also clears the record. */
rsos_status rsos_timing(rsos_surface *s, int enable);
rsos_status rsos_timing_read(rsos_surface *s, int64_t *launches, double *mean_ms, double *total_ms);

/* Name of the tile-block kernel instance that sweeps this surface, in the
 * form rocprofv3 shows its template arguments: e.g.
 * "block_sweep<8,32,8,256,int8,int16,0>" (D, tiles per block in x and y,
 * threads, LDS element type, the wider type of blocks that do not fit it,
 * schedule), "block_sweep16<8,32,8,256,0>" with 16-bit storage, or
 * "lds_run<8,256,0>" for an LDS-resident surface; written NUL-terminated
 * into buf (at most len bytes).  With several kernel instances (a tuned
 * batch) the first one. */
rsos_status rsos_kernel_name(rsos_surface *s, char *buf, int32_t len);

/* Frees the handle and library-owned memory (never d_h, never a
 * caller-provided d_work).  Synchronises the stream first. */
rsos_status rsos_free(rsos_surface *s);

/* --------------------------------------------------------------------- */
/* For callers that cannot allocate device memory: code under hipGraph    */
/* capture, tight serving loops, harnesses that forbid allocation.         */
/* --------------------------------------------------------------------- */

#define RSOS_STATIC_MAX_SWEEPS 4096

/* rsos_init + rsos_sweep + rsos_log in one call that allocates nothing:
 * no handle, no hipMalloc or hipFree, no pinned host memory, no memset
 * nodes (small fill kernels instead), so the launches may be captured.
 * The descriptor, the accumulators and a log ring of
 * RSOS_STATIC_MAX_SWEEPS + 1 records live in a fixed 128 KiB device array
 * of the library (one per GPU, held until the process ends).
 *   p       parameters as for rsos_init; flags 0 or RSOS_FLAG_DT4 (no
 *           16-bit storage, no autotuner: the first variant that fits);
 *   d_h, d_work  caller-owned device int32[L*L] (16-byte aligned); the
 *           state after t0 sweeps is in d_h if t0 is even, else in d_work,
 *           and after the call the state after t0 + n_mcs sweeps is in the
 *           buffer of that parity (the same convention as rsos_init);
 *   t0      sweeps already done, 0 <= t0, t0 + n_mcs <= 2^32;
 *   s1, s2  exact sum h and sum h^2 of that state (0, 0 for a flat start;
 *           the last record of the previous call when continuing);
 *   n_mcs   sweeps, 0 <= n_mcs <= RSOS_STATIC_MAX_SWEEPS (RSOS_E_INVAL
 *           beyond);
 *   d_log   caller-owned device int64[3 * n_mcs] receiving (S1, S2, A) of
 *           times t0+1 .. t0+n_mcs, as rsos_log's records;
 *   stream  hipStream_t (NULL = default stream); everything is enqueued
 *           asynchronously on it.
 * Same results as rsos_init / rsos_sweep with the same arguments.  Checks
 * the overflow bound (with max h0 <= s1 / L^2 + N L) before enqueuing
 * (RSOS_E_OVERFLOW).  Calls that overlap on one GPU (other streams, other
 * host threads) share the array and race; serialize them. */
rsos_status rsos_sweep_static(const rsos_params *p, int32_t *d_h, int32_t *d_work, int64_t t0, int64_t s1,
                              int64_t s2, int64_t n_mcs, int64_t *d_log, void *stream);

/* --------------------------------------------------------------------- */
/* Multisurface lock-step mode (Sec. II: multisurface coding).  Groups of  */
/* 128 realizations of one L x L surface share the sequence of selected    */
/* sites; each realization applies a selection with probability 1/2 (its   */
/* own coin), which breaks the correlation between them.                   */
/* --------------------------------------------------------------------- */

typedef struct rsos_ms rsos_ms;

/* Creates `groups` groups of 128 realizations, flat start, t = 0.
 *   p       L (multiple of 16, 16 <= L <= 65536), N (N*L <= 32766), D = 8,
 *           flags = 0, seed; group g uses the Philox key seed + g;
 *   d_lat   caller-owned device memory of groups * L*L * 256 bytes,
 *           16-byte aligned (NULL: the library allocates): per group and
 *           site, 128 16-bit residues of the heights, realization r at
 *           halfword r (a 256-byte record);
 *   log_cap sweeps kept per realization (0 = 65536).
 * Besides the log (128 * log_cap * 24 bytes per group) the library owns
 * 8 * L*L bytes per group of per-tile partial sums.
 * Schedule: per sweep s, origin from Philox (0, 0, s, 2) mod 2D; colour-0
 * then colour-1 tiles of the checkerboard; a tile makes 2 D^2 selections,
 * selection a taking site field a of Philox (j, tile_id, s, p) as in the
 * checkerboard layout; realization r applies it iff bit a mod 32 of word
 * (a div 32) mod 4 of Philox (a div 128, tile_id, s, 8 + 2r + p) is set.
 * Each realization receives L^2 attempts per sweep on average. */
rsos_status rsos_ms_init(rsos_ms **out, const rsos_params *p, int32_t groups, uint32_t *d_lat,
                         int64_t log_cap, void *stream);

/* Enqueues n_mcs sweeps of every realization (asynchronous). */
rsos_status rsos_ms_sweep(rsos_ms *m, int64_t n_mcs);

/* Synchronises; out[g*128 + r] = record of realization r of group g at the
 * current time (s1, s2 exact; accepted = deposits of the last sweep). */
rsos_status rsos_ms_width(rsos_ms *m, rsos_width_t *out);

/* Synchronises; records t_from .. t_from+n-1 of one realization (g*128+r). */
rsos_status rsos_ms_log(rsos_ms *m, int32_t realization, int64_t t_from, int64_t n, rsos_width_t *out);

/* Synchronises; int32 heights of one realization into host memory. */
rsos_status rsos_ms_heights(rsos_ms *m, int32_t realization, int32_t *dst_host);

/* Frees the handle and library-owned memory (never a caller's d_lat). */
rsos_status rsos_ms_free(rsos_ms *m);

/* --------------------------------------------------------------------- */
/* Batched ensemble: many independent surfaces (any L, N, seed; one D) in   */
/* one launch per sweep.  Independent realization sets, Sec. II.          */
/* --------------------------------------------------------------------- */

/* n surfaces; p[i] their parameters (all with the same D and flags; with
 * RSOS_FLAG_TUNE each (L, N) class gets the autotuner's batched choice, and
 * surfaces with different choices are swept by separate kernel instances
 * in the same sweep);
 * d_pool / d_work_pool caller-owned device int32 pools, surface i at
 * element offsets[i] of each (L_i^2 elements, offsets[] host array);
 * d_work_pool NULL makes the library allocate the second pool.  Flat start,
 * t = 0 for all. */
rsos_status rsos_batch_init(rsos_batch **out, int32_t n, const rsos_params *p, int32_t *d_pool,
                            int32_t *d_work_pool, const int64_t *offsets, int64_t log_cap,
                            void *stream);

/* Enqueues sweeps: surface i advances n_mcs[i] sweeps (n_mcs NULL: every
 * surface advances n_all).  Surfaces that are done idle in later launches. */
rsos_status rsos_batch_sweep(rsos_batch *b, const int64_t *n_mcs, int64_t n_all);

/* Synchronises; out[i] = record of surface i at its current time. */
rsos_status rsos_batch_width(rsos_batch *b, rsos_width_t *out);

/* Synchronises; per-sweep records of surface i, as rsos_log. */
rsos_status rsos_batch_log(rsos_batch *b, int32_t i, int64_t t_from, int64_t n, rsos_width_t *out);

/* Synchronises; height-distribution moments of surface i, as rsos_moments. */
rsos_status rsos_batch_moments(rsos_batch *b, int32_t i, rsos_moments_t *out);

/* Synchronises; copies surface i's current heights. */
rsos_status rsos_batch_heights(rsos_batch *b, int32_t i, int32_t *dst, int dst_is_device);

rsos_status rsos_batch_free(rsos_batch *b);

/* --------------------------------------------------------------------- */
/* Serving engine: continuous batching of simulation jobs.                 */
/* --------------------------------------------------------------------- */

/* Job states reported by rsos_engine_poll. */
enum { RSOS_JOB_QUEUED = 0, RSOS_JOB_RUNNING = 1, RSOS_JOB_DONE = 2, RSOS_JOB_CANCELLED = 3 };

/* Creates an engine over a caller-owned device pool of pool_bytes bytes.
 * Jobs are admitted in arrival order (strict FIFO) while their footprint
 * (two L^2 int32 lattices, each 256-byte aligned) fits in the free part of
 * the pool and fewer than max_running jobs run.  Every running job advances
 * one sweep per tick; a tick is one launch over all running jobs (jobs whose
 * L^2 int32 fit in LDS run on a second stream).  Ticks are issued in chunks
 * of up to 16; admission, retirement and result collection happen between
 * chunks.  d_pool must be 256-byte aligned; all jobs share the engine's D. */
rsos_status rsos_engine_create(rsos_engine **out, void *d_pool, int64_t pool_bytes,
                               int32_t max_running, int32_t D, void *stream);

/* Flags of rsos_engine_submit. */
enum { RSOS_JOB_KEEP_HEIGHTS = 1 };

/* Queues a job: parameters p (p->D must equal the engine's D), t_max >= 1
 * sweeps, and the sweep times (1 <= t <= t_max, strictly increasing) whose
 * width records are kept.  With RSOS_JOB_KEEP_HEIGHTS the final heights
 * are copied to host memory when the job finishes.  *job_id receives the
 * id.  RSOS_E_INVAL if the job could never fit the pool. */
rsos_status rsos_engine_submit(rsos_engine *e, const rsos_params *p, int64_t t_max,
                               const int64_t *sample_t, int32_t n_samples, int32_t flags,
                               int64_t *job_id);

/* Admits what fits, then runs up to max_ticks ticks (stopping early when
 * nothing runs), retiring finished jobs and admitting queued ones between
 * chunks.  *n_finished (may be NULL) receives the jobs that finished. */
rsos_status rsos_engine_step(rsos_engine *e, int64_t max_ticks, int32_t *n_finished);

/* State of a job (RSOS_JOB_*) and its current sweep count. */
rsos_status rsos_engine_poll(rsos_engine *e, int64_t job_id, int32_t *state, int64_t *t);

/* Results of a finished job: its n_samples width records (at the requested
 * times; a cancelled job fills only the records it reached and sets the
 * rest to t = -1) and, if heights_host is non-NULL and the job kept them,
 * its final int32[L*L] heights.  *latency_s (may be NULL) receives the time
 * from submission to completion in seconds.  Results stay until
 * rsos_engine_release. */
rsos_status rsos_engine_result(rsos_engine *e, int64_t job_id, rsos_width_t *samples,
                               int32_t *heights_host, double *latency_s);

/* Drops a queued or running job; a running job's memory is freed at the
 * next chunk boundary. */
rsos_status rsos_engine_cancel(rsos_engine *e, int64_t job_id);

/* Forgets a finished or cancelled job's stored results. */
rsos_status rsos_engine_release(rsos_engine *e, int64_t job_id);

/* Counters: [0] queued, [1] running, [2] finished, [3] pool bytes in use,
 * [4] ticks, [5] attempted site updates so far. */
rsos_status rsos_engine_stats(rsos_engine *e, int64_t out[6]);

/* Launch choice of the engine's tile-block jobs: with enable != 0 each
 * chunk sweeps the running jobs with the autotuner's batched choice for the
 * (L, N) class that holds the most sites among them, when that variant fits
 * every running job (a class is tuned on first use, between chunks; load a
 * saved cache with rsos_tune_load to avoid that); otherwise, and with
 * enable = 0 (the default), with the first variant that fits them all.
 * Results never change. */
rsos_status rsos_engine_tune(rsos_engine *e, int32_t enable);

rsos_status rsos_engine_destroy(rsos_engine *e);

/* --------------------------------------------------------------------- */
/* Autotuner.  The paper chooses its tile layout for the GPU it runs on    */
/* (Sec. II; domain sizes compared in Sec. III.C).  Here the domain size D */
/* is part of the result and is never tuned; the autotuner picks, per key  */
/* (device, D, L, N, storage and schedule flags, alone or batched), the    */
/* launch knobs that leave every result unchanged: the tile-block variant  */
/* (block shape, threads per workgroup, LDS staging type), the order in    */
/* which workgroups take blocks across the 8 XCDs, and the sweeps per      */
/* captured hipGraph.  It times every candidate with HIP events on a       */
/* scratch workload of the key (flat surfaces; one surface when alone,     */
/* ceil(2^24 / L^2) surfaces in one launch when batched; L > 16384 tuned   */
/* on a 16384^2 stand-in) and caches the fastest for the process.  Tuning */
/* allocates scratch device memory (two int32 pools of the workload) and   */
/* synchronises; it never touches a caller's surface.  The cache is        */
/* process-wide and guarded by a mutex.                                    */
/* --------------------------------------------------------------------- */

/* One launch configuration.
 *   TX, TY, NT    tiles per block in x and y, threads per workgroup;
 *   elem          LDS bytes per staged site (1: int8, with int16
 *                 sub-blocks where a block's range does not fit; 2; 4);
 *   xmode         workgroup -> block order: 0 in order, 1 runs of 16
 *                 blocks per XCD, 2 one column strip of blocks per XCD
 *                 (single surfaces whose block columns divide by 8);
 *   graph_sweeps  sweeps per captured hipGraph;
 *   candidates    configurations timed for the key;
 *   measured      1 if chosen by timing on this process's device, 0 if
 *                 entered by rsos_tune_set (or loaded as such);
 *   ms_per_sweep  the chosen configuration's mean sweep time on the
 *                 tuning workload (0 if not measured);
 *   ms_first_fit  the untuned default's (first fitting variant, xmode 1)
 *                 on the same workload. */
typedef struct {
    int32_t TX, TY, NT, elem;
    int32_t xmode;
    int32_t graph_sweeps;
    int32_t candidates;
    int32_t measured;
    double ms_per_sweep;
    double ms_first_fit;
} rsos_tune_t;

/* The cached configuration of p's key (batch != 0: tuned for surfaces
 * swept together with others), tuning it now if there is none.  L must be
 * on the tile-block path (L^2 * 4 > 64 KiB; RSOS_E_INVAL otherwise). */
rsos_status rsos_tune(const rsos_params *p, int32_t batch, rsos_tune_t *out);

/* Lists the candidates of p's key: *n receives their number, the first
 * min(*n, cap) are written to out (shape fields; and, if the key has been
 * tuned in this process, measured = 1 and the candidate's own time in
 * ms_per_sweep). */
rsos_status rsos_tune_candidates(const rsos_params *p, int32_t batch, rsos_tune_t *out, int32_t cap, int32_t *n);

/* Enters a configuration for p's key without timing (it must fit the key:
 * RSOS_E_INVAL otherwise); later handles created with RSOS_FLAG_TUNE use
 * it.  Meant for tests and for reusing results of another process. */
rsos_status rsos_tune_set(const rsos_params *p, int32_t batch, const rsos_tune_t *choice);

/* Empties the cache. */
rsos_status rsos_tune_clear(void);

/* Writes the cache as text, one line per key; reads such a file back into
 * the cache (lines whose configuration no longer exists or fits are
 * skipped).  RSOS_E_INVAL if the file cannot be written or read. */
rsos_status rsos_tune_save(const char *path);
rsos_status rsos_tune_load(const char *path);

/* --------------------------------------------------------------------- */
/* Utilities.                                                             */
/* --------------------------------------------------------------------- */

/* The library's own Philox4x32-10 block function, run on the host: out =
 * f_key(ctr).  The device kernels use the same code. */
void rsos_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* W^2 of Eq. (2) from the exact sums, as stored in rsos_width_t.w2. */
double rsos_w2(int32_t L, int64_t s1, int64_t s2);

const char *rsos_strerror(rsos_status st);
const char *rsos_last_error(void);

/* Library version string. */
const char *rsos_version(void);

/* For tests of the error paths, on the calling thread: the after-th HIP
 * runtime call the library makes from now on is not made and reports a
 * runtime error instead (RSOS_E_DEVICE, and the handle it belongs to is
 * failed for good, exactly as after a real one); 0 turns this off.  No
 * device work is involved. */
rsos_status rsos_debug_fail(int32_t after);

#ifdef __cplusplus
}
#endif
#endif

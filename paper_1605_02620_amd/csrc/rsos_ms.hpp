// rsos_ms.hpp -- gfx950 kernels of the multisurface lock-step mode.
//
// Multisurface coding (Sec. II): a group of 128 realizations shares one
// sequence of selected sites; each realization applies a selection only
// with probability 1/2 (its own coin bit), which breaks the correlation
// between them.  In device memory a site of a group is one 256-byte record
// of 128 16-bit residues (realization r at halfword r).  On the GPU the
// realizations of a tile run side by side, one per lane, with their values
// staged in LDS as [site][realization]: every LDS access of a selection is
// consecutive across the wave (no bank conflicts), global accesses are
// whole records or half records, and the site sequence is uniform across
// the wave.  ms_phase_b (N <= 9) stages bytes relative to a frozen
// reference site, ms_phase 16-bit residues.
//
// Schedule (identical bits for any launch shape): group g uses the Philox
// key seed + g; sweep s: origin from (0, 0, s, 2) as for the checkerboard;
// colour-0 tiles, then colour-1 tiles; a tile makes 2 D^2 selections, site
// field a from Philox (j, tile_id, s, p) in the checkerboard layout; the coin
// of realization r is bit a mod 32 of word (a div 32) mod 4 of Philox
// (a div 128, tile_id, s, 8 + 2r + p).  A selection whose coin is set is an
// RSOS attempt (Sec. I) on that realization.
//
// Storage: residues mod 2^16 with floor(S1_r / L^2) per realization as the
// reference (exact while N L <= 32766, as for 16-bit single surfaces).
#pragma once

#include "rsos_kernels.hpp"

namespace rsosk {

constexpr int kMsReal = 128;    // realizations per group
constexpr int kMsChunks = 64;   // most tile ranges summed per group

struct MsDev {
    uint32_t *lat;        // [G][L*L] records of 128 16-bit residues (realization r at halfword r)
    long long *m0;        // [G][128] floor(S1 / L^2) of the current time
    int *part;            // [G][T*T][128]: 256 H + A of each tile's update in the current sweep
    long long *acc;       // [G][128][2]: (A, H) of the current sweep summed so far (zero between sweeps)
    long long *done;      // [G][16]: ranges of tiles summed in the current sweep (word 0 of a 128-byte line)
    long long *log;       // [G][128][log_cap][3]: (S1, S2, A) of time tau at slot tau % log_cap
    long long *t;         // [G] sweeps done
    long long log_cap;
    long long t_end;
    unsigned long long seed;
    int L, N, T, G, nchunk;
};

// A tile's update of one realization is recorded as 256 H + A, where A is
// its accepted count (at most 2 D^2 = 128) and H the sum of h - m0 over its
// accepted deposits (|h - m0| <= N L <= 32766, so |H| < 2^22 and the record
// fits in 32 bits).  Plain stores, one per tile and realization: the sums
// over tiles are formed by ms_partial, which adds one sum per range of at
// least 64 tiles and realization with a device-scope atomic (one such
// addition per tile serialised the whole phase on a few words).
__device__ __forceinline__ void ms_record(const MsDev &d, int g, uint32_t tile_id, int r, int A, int H)
{
    d.part[((size_t)g * d.T * d.T + tile_id) * kMsReal + r] = H * 256 + A;
}

typedef __attribute__((address_space(1))) uint32_t gu32;

// One wavefront per (group, tile of colour p, half of the group): lane l
// runs realization r = 64 h + l.  The padded tile of the 64 realizations
// (10 x 10 sites x 128 bytes) is staged in LDS as [site][lane] 16-bit
// residues, so every LDS access of a selection is 64 consecutive halfwords.
template <int D>
__global__ __launch_bounds__(64) void ms_phase(const MsDev *__restrict__ dp, int p)
{
    constexpr int P = D + 2;            // padded tile side (tile plus a one-site ring)
    constexpr int SEL = 2 * D * D;      // selections per tile
    using TB = TileBits<D>;
    static_assert(SEL == 128, "one coin block per tile (D = 8)");
    __shared__ __attribute__((aligned(16))) uint16_t lds[P * P * 64];   // [padded site][lane]

    const MsDev &d = *dp;
    const int L = d.L, T = d.T, N = d.N;
    const int half = T * T / 2;
    const int hh = (int)(blockIdx.x & 1u);
    const int wid = (int)(blockIdx.x >> 1);
    const int g = wid / half, k = wid - g * half;
    // the time is uniform: keep it (and everything derived from it, such as
    // the site stream) in scalar registers
    const long long tv = d.t[g];
    const long long t = (long long)(((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)tv));
    if (t >= d.t_end) return;
    const int ty = k / (T / 2), tx = 2 * (k % (T / 2)) + ((ty + p) & 1);
    const unsigned long long key = d.seed + (unsigned long long)g;
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    const uint32_t s = (uint32_t)t;
    const u32x4 org = philox4x32_10(0u, 0u, s, 2u, k0, k1);
    const int ox = (int)(org.v[0] % (2u * D)), oy = (int)(org.v[1] % (2u * D));
    int X0 = ox + tx * D - 1, Y0 = oy + ty * D - 1;   // global site of padded (0, 0)
    if (X0 < 0) X0 += L;
    if (Y0 < 0) Y0 += L;
    if (X0 >= L) X0 -= L;
    if (Y0 >= L) Y0 -= L;
    const int lane = threadIdx.x;
    // this half's 128 bytes of each 256-byte site record
    const gu32 *lat = (const gu32 *)(d.lat + (size_t)g * L * L * 64) + 32 * hh;
    gu32 *latw = (gu32 *)(d.lat + (size_t)g * L * L * 64) + 32 * hh;

    // ---- load the padded tile: 8 sites per instruction, 8 lanes x 16 B per
    // site; every load is issued before the first is used (the last pass's
    // surplus lanes load the last site again and do not write it)
    {
        constexpr int NLD = (P * P + 7) / 8;
        v4u vin[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int site = min(8 * i + (lane >> 3), P * P - 1);
            const int sy = site / P, sx = site - sy * P;
            int gx = X0 + sx, gy = Y0 + sy;
            if (gx >= L) gx -= L;
            if (gy >= L) gy -= L;
            vin[i] = *reinterpret_cast<const gv4u *>(lat + ((size_t)gy * L + gx) * 64 + 4 * (lane & 7));
        }
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int site = 8 * i + (lane >> 3);
            if (site < P * P)
                *reinterpret_cast<uint4 *>(&lds[site * 64 + 8 * (lane & 7)]) =
                    make_uint4(vin[i].x, vin[i].y, vin[i].z, vin[i].w);
        }
    }
    __syncthreads();

    const int r = 64 * hh + lane;   // realization within the group
    const long long m0 = d.m0[(size_t)g * kMsReal + r];
    const uint32_t m0r = (uint32_t)m0 & 0xFFFFu;
    const uint32_t tile_id = (uint32_t)(ty * T + tx);
    int A = 0;   // accepted deposits
    int q = 0;   // sum of h - m0 before the accepted deposits
    // this realization's coins for the tile's 128 selections
    const u32x4 cw = philox4x32_10(0u, tile_id, s, 8u + 2u * (uint32_t)r + (uint32_t)p, k0, k1);
    constexpr int NFULL = SEL / TB::PER, TAIL = SEL % TB::PER;
    auto select = [&](int call, int nsel) {
        // site fields of this call (uniform across the wave) and the coin
        // bits of its selections, bits [call*PER, call*PER + nsel) of the
        // realization's 128 coin bits
        const u32x4 rr = philox4x32_10((uint32_t)call, tile_id, s, (uint32_t)p, k0, k1);
        const int b0 = call * TB::PER, lo = b0 >> 5, sh = b0 & 31;
        const uint32_t w0 = lo == 0 ? cw.v[0] : lo == 1 ? cw.v[1] : lo == 2 ? cw.v[2] : cw.v[3];
        const uint32_t w1 = lo == 0 ? cw.v[1] : lo == 1 ? cw.v[2] : lo == 2 ? cw.v[3] : 0u;
        const uint32_t ch = (uint32_t)((((unsigned long long)w1 << 32) | w0) >> sh);
#pragma unroll
        for (int kk = 0; kk < TB::PER; ++kk) {
            if (kk < nsel) {
                const uint32_t f = (rr.v[kk / TB::F] >> ((kk % TB::F) * TB::B)) & (uint32_t)(D * D - 1);
                const int idx = ((int)(f >> TB::LOG2D) + 1) * P + (int)(f & (D - 1)) + 1;
                const uint32_t c = lds[idx * 64 + lane];
                // c - h_j, exact in int16; accept iff every one < N
                const int d1 = (int)(int16_t)(uint16_t)(c - lds[(idx - 1) * 64 + lane]);
                const int d2 = (int)(int16_t)(uint16_t)(c - lds[(idx + 1) * 64 + lane]);
                const int d3 = (int)(int16_t)(uint16_t)(c - lds[(idx - P) * 64 + lane]);
                const int d4 = (int)(int16_t)(uint16_t)(c - lds[(idx + P) * 64 + lane]);
                const int dm = max(max(d1, d2), max(d3, d4));
                const int acc = (int)(((uint32_t)(dm - N) >> 31) & (ch >> kk) & 1u);
                lds[idx * 64 + lane] = (uint16_t)(c + (uint32_t)acc);
                A += acc;
                q += (int)(int16_t)(uint16_t)(c - m0r) & -acc;
            }
        }
    };
#pragma unroll 1
    for (int j = 0; j < NFULL; ++j) select(j, TB::PER);
    if constexpr (TAIL > 0) select(NFULL, TAIL);

    // ---- store the tile interior: 8 sites per instruction
#pragma unroll 4
    for (int i = 0; i < D * D / 8; ++i) {
        const int site = 8 * i + (lane >> 3);
        const int sy = site / D, sx = site - sy * D;
        int gx = X0 + 1 + sx, gy = Y0 + 1 + sy;
        if (gx >= L) gx -= L;
        if (gy >= L) gy -= L;
        const uint4 v = *reinterpret_cast<const uint4 *>(&lds[((sy + 1) * P + sx + 1) * 64 + 8 * (lane & 7)]);
        const v4u o = {v.x, v.y, v.z, v.w};
        *reinterpret_cast<gv4u *>(latw + ((size_t)gy * L + gx) * 64 + 4 * (lane & 7)) = o;
    }

    ms_record(d, g, tile_id, r, A, q);
}

// Largest N for which ms_phase_b's byte staging is exact: every staged site
// lies within 14 bonds of the frozen reference site (padded row 0, column
// 5), so its height differs from the reference by at most 14 N <= 127.
constexpr int kMsByteMaxN = 9;
constexpr int kMsRefSite = 5;

// The same schedule as ms_phase with the padded tile staged as bytes: one
// workgroup of 128 threads per (group, tile of colour p), thread r running
// realization r (wave 0 the first half of the group, wave 1 the second),
// LDS [padded site][realization] holding h - h_ref + 128, where h_ref is the
// realization's height at the reference site.  Half the LDS of the 16-bit
// staging, so twice as many tiles are resident per CU.  Requires
// N <= kMsByteMaxN (checked on the host).
template <int D>
__global__ __launch_bounds__(128) void ms_phase_b(const MsDev *__restrict__ dp, int p)
{
    constexpr int P = D + 2;
    constexpr int SEL = 2 * D * D;
    using TB = TileBits<D>;
    static_assert(SEL == 128, "one coin block per tile (D = 8)");
    __shared__ __attribute__((aligned(16))) uint8_t lds[P * P * kMsReal];   // [padded site][realization]

    const MsDev &d = *dp;
    const int L = d.L, T = d.T, N = d.N;
    const int half = T * T / 2;
    const int g = (int)blockIdx.x / half, k = (int)blockIdx.x - g * half;
    const long long tv = d.t[g];
    const long long t = (long long)(((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)tv));
    if (t >= d.t_end) return;
    const int ty = k / (T / 2), tx = 2 * (k % (T / 2)) + ((ty + p) & 1);
    const unsigned long long key = d.seed + (unsigned long long)g;
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    const uint32_t s = (uint32_t)t;
    const u32x4 org = philox4x32_10(0u, 0u, s, 2u, k0, k1);
    const int ox = (int)(org.v[0] % (2u * D)), oy = (int)(org.v[1] % (2u * D));
    int X0 = ox + tx * D - 1, Y0 = oy + ty * D - 1;   // global site of padded (0, 0)
    if (X0 < 0) X0 += L;
    if (Y0 < 0) Y0 += L;
    if (X0 >= L) X0 -= L;
    if (Y0 >= L) Y0 -= L;
    const int tid = threadIdx.x;
    const int ck = tid & 15;   // this thread's 16-byte chunk of a record: realizations 8 ck .. 8 ck + 7
    const gu32 *lat = (const gu32 *)(d.lat + (size_t)g * L * L * 64);
    gu32 *latw = (gu32 *)(d.lat + (size_t)g * L * L * 64);
    auto site_of = [&](int sy, int sx) {
        int gx = X0 + sx, gy = Y0 + sy;
        if (gx >= L) gx -= L;
        if (gy >= L) gy -= L;
        return (size_t)gy * L + gx;
    };

    // reference residues of this thread's chunk, and the bias that maps a
    // residue u to the byte u - ref + 128 in each 16-bit lane
    const size_t sref = site_of(0, kMsRefSite);
    const v4u rv = *reinterpret_cast<const gv4u *>(lat + sref * 64 + 4 * ck);
    const uint32_t bias = 0x00800080u;
    const v4u sub = {pk_sub16(rv.x, bias), pk_sub16(rv.y, bias), pk_sub16(rv.z, bias), pk_sub16(rv.w, bias)};

    // ---- load the padded tile: 8 sites per pass, 16 threads x 16 bytes per
    // site; every load is issued before the first is used (the last pass's
    // surplus threads load the last site again and do not write it)
    {
        constexpr int NLD = (P * P + 7) / 8;
        v4u vin[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int site = min(8 * i + (tid >> 4), P * P - 1);
            const int sy = site / P, sx = site - sy * P;
            vin[i] = *reinterpret_cast<const gv4u *>(lat + site_of(sy, sx) * 64 + 4 * ck);
        }
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int site = 8 * i + (tid >> 4);
            if (site < P * P) {
                const v4u &v = vin[i];
                const uint32_t w0 = pk_sub16(v.x, sub.x), w1 = pk_sub16(v.y, sub.y);
                const uint32_t w2 = pk_sub16(v.z, sub.z), w3 = pk_sub16(v.w, sub.w);
                *reinterpret_cast<uint2 *>(&lds[site * kMsReal + 8 * ck]) =
                    make_uint2(__builtin_amdgcn_perm(w1, w0, 0x06040200u), __builtin_amdgcn_perm(w3, w2, 0x06040200u));
            }
        }
    }
    __syncthreads();

    const int r = tid;   // realization within the group
    const long long m0 = d.m0[(size_t)g * kMsReal + r];
    // h - m0 = byte - 128 + dref for this realization
    const uint32_t ref_r = reinterpret_cast<const uint16_t *>(d.lat + (size_t)g * L * L * 64 + sref * 64)[r];
    const int dref = (int)(int16_t)(uint16_t)(ref_r - ((uint32_t)m0 & 0xFFFFu)) - 128;
    const uint32_t tile_id = (uint32_t)(ty * T + tx);
    int A = 0;   // accepted deposits
    int q = 0;   // sum of the staged bytes before the accepted deposits
    const u32x4 cw = philox4x32_10(0u, tile_id, s, 8u + 2u * (uint32_t)r + (uint32_t)p, k0, k1);
    constexpr int NFULL = SEL / TB::PER, TAIL = SEL % TB::PER;
    auto select = [&](int call, int nsel) {
        const u32x4 rr = philox4x32_10((uint32_t)call, tile_id, s, (uint32_t)p, k0, k1);
        const int b0 = call * TB::PER, lo = b0 >> 5, sh = b0 & 31;
        const uint32_t w0 = lo == 0 ? cw.v[0] : lo == 1 ? cw.v[1] : lo == 2 ? cw.v[2] : cw.v[3];
        const uint32_t w1 = lo == 0 ? cw.v[1] : lo == 1 ? cw.v[2] : lo == 2 ? cw.v[3] : 0u;
        const uint32_t ch = (uint32_t)((((unsigned long long)w1 << 32) | w0) >> sh);
#pragma unroll
        for (int kk = 0; kk < TB::PER; ++kk) {
            if (kk < nsel) {
                const uint32_t f = (rr.v[kk / TB::F] >> ((kk % TB::F) * TB::B)) & (uint32_t)(D * D - 1);
                const int idx = ((int)(f >> TB::LOG2D) + 1) * P + (int)(f & (D - 1)) + 1;
                const int c = lds[idx * kMsReal + r];
                const int m = min(min((int)lds[(idx - 1) * kMsReal + r], (int)lds[(idx + 1) * kMsReal + r]),
                                  min((int)lds[(idx - P) * kMsReal + r], (int)lds[(idx + P) * kMsReal + r]));
                // accept iff c + 1 - h_j <= N for every neighbour j
                const int acc = (int)(((uint32_t)(c - m - N) >> 31) & (ch >> kk) & 1u);
                lds[idx * kMsReal + r] = (uint8_t)(c + acc);
                A += acc;
                q += c & -acc;
            }
        }
    };
#pragma unroll 1
    for (int j = 0; j < NFULL; ++j) select(j, TB::PER);
    if constexpr (TAIL > 0) select(NFULL, TAIL);
    __syncthreads();

    // ---- store the tile interior: 8 sites per pass
#pragma unroll 4
    for (int i = 0; i < D * D / 8; ++i) {
        const int site = 8 * i + (tid >> 4);
        const int sy = site / D, sx = site - sy * D;
        const uint2 b = *reinterpret_cast<const uint2 *>(&lds[((sy + 1) * P + sx + 1) * kMsReal + 8 * ck]);
        // byte u -> residue u + ref - 128
        const v4u o = {pk_add16(__builtin_amdgcn_perm(0u, b.x, 0x0C010C00u), sub.x),
                       pk_add16(__builtin_amdgcn_perm(0u, b.x, 0x0C030C02u), sub.y),
                       pk_add16(__builtin_amdgcn_perm(0u, b.y, 0x0C010C00u), sub.z),
                       pk_add16(__builtin_amdgcn_perm(0u, b.y, 0x0C030C02u), sub.w)};
        *reinterpret_cast<gv4u *>(latw + site_of(sy + 1, sx + 1) * 64 + 4 * ck) = o;
    }

    ms_record(d, g, tile_id, r, A, q + dref * A);
}

// The sums over a range of tiles: a workgroup of kMsSub x 128 threads,
// thread (sub, r) adds every kMsSub-th value for realization r
// (independent loads, unrolled, so the loads overlap), then the kMsSub
// partial sums are combined in LDS.
constexpr int kMsSub = 4;

__device__ __forceinline__ void ms_combine(long long &A, long long &H)
{
    __shared__ long long sa[kMsSub][kMsReal], sh[kMsSub][kMsReal];
    const int sub = threadIdx.x / kMsReal, r = threadIdx.x % kMsReal;
    sa[sub][r] = A;
    sh[sub][r] = H;
    __syncthreads();
    if (sub == 0) {
#pragma unroll
        for (int k = 1; k < kMsSub; ++k) {
            A += sa[k][r];
            H += sh[k][r];
        }
    }
}

// After both phases: workgroup (c, g) sums the tile records of tile range c
// of group g for each of its 128 realizations and adds the sums into the
// group's accumulators; the workgroup that completes the group's count
// folds them into each realization's log (a deposit on height h adds 2h + 1
// to S2, and h = m0 + (h - m0)), updates floor(S1 / L^2), clears the
// accumulators and advances the group's time.  Device-scope atomics without
// fences, as for the block sweep: a workgroup counts itself only after its
// additions have been performed, and the last one reads the accumulators
// with device-scope atomic loads.
__global__ __launch_bounds__(kMsSub * kMsReal) void ms_partial(const MsDev *__restrict__ dp)
{
    const MsDev &d = *dp;
    const int c = blockIdx.x, g = blockIdx.y;
    const int sub = threadIdx.x / kMsReal, r = threadIdx.x % kMsReal;
    const long long t = d.t[g];
    if (t >= d.t_end) return;
    const long long tiles = (long long)d.T * d.T;
    const long long cs = (tiles + d.nchunk - 1) / d.nchunk;
    const long long lo = c * cs, hi = min(tiles, lo + cs);
    const int *p = d.part + (size_t)g * tiles * kMsReal + r;
    long long A = 0, H = 0;
#pragma unroll 16
    for (long long k = lo + sub; k < hi; k += kMsSub) {
        const int v = p[k * kMsReal];
        A += v & 255;
        H += v >> 8;
    }
    ms_combine(A, H);
    __shared__ int s_last;
    typedef __attribute__((address_space(1))) unsigned long long gu64m;
    gu64m *acc = (gu64m *)(d.acc + ((size_t)g * kMsReal + r) * 2);
    if (sub == 0) {
        __hip_atomic_fetch_add(acc + 0, (unsigned long long)A, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(acc + 1, (unsigned long long)H, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the additions are performed before the workgroup is counted
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long prev = __hip_atomic_fetch_add((gu64m *)(d.done + 16 * (size_t)g), 1ull,
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev + 1 == (unsigned long long)d.nchunk;
    }
    __syncthreads();
    if (!s_last || sub != 0) return;
    A = (long long)__hip_atomic_load(acc + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    H = (long long)__hip_atomic_load(acc + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(acc + 0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(acc + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const size_t id = (size_t)g * kMsReal + r;
    const long long S2 = 2 * (d.m0[id] * A + H) + A;
    const long long *prev = d.log + (id * d.log_cap + t % d.log_cap) * 3;
    long long *e = d.log + (id * d.log_cap + (t + 1) % d.log_cap) * 3;
    const long long s1 = prev[0] + A;
    e[0] = s1;
    e[1] = prev[1] + S2;
    e[2] = A;
    d.m0[id] = s1 / ((long long)d.L * d.L);
    if (r == 0) {
        __hip_atomic_store((gu64m *)(d.done + 16 * (size_t)g), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // every workgroup of the group read t before it was counted
        d.t[g] = t + 1;
    }
}

// Realization r of group g as int32 heights (grid-stride).
__global__ void ms_unpack(const MsDev *__restrict__ dp, int g, int r, int32_t *__restrict__ dst)
{
    const MsDev &d = *dp;
    const long long n = (long long)d.L * d.L;
    const long long m0 = d.m0[(size_t)g * kMsReal + r];
    const uint32_t r0 = (uint32_t)m0 & 0xFFFFu;
    const uint32_t *lat = d.lat + (size_t)g * n * 64;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const uint32_t w = lat[i * 64 + (r >> 1)];
        const uint32_t res = (r & 1) ? (w >> 16) : (w & 0xFFFFu);
        dst[i] = (int32_t)(m0 + (long long)(int16_t)(uint16_t)(res - r0));
    }
}

}  // namespace rsosk

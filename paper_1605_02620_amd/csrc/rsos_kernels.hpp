// rsos_kernels.hpp -- gfx950 kernels of the RSOS deposition sweep.
//
// Model (Kelling, Odor & Gemming): RSOS deposition on an L x L periodic
// lattice, accepted iff afterwards |h_i - h_j| <= N for the 4 nearest
// neighbours (Sec. I); one sweep = L^2 attempts scheduled over D x D domains
// whose origin moves randomly each sweep (Sec. II); per-sweep exact sums
// S1 = sum h, S2 = sum h^2 for Eq. (2).
//
// Schedule of one sweep s (identical bits for any launch shape):
//   origin (ox, oy) = Philox(0, 0, s, 2) words 0, 1 mod 2D;
//   colour-0 tiles of the shifted frame make D^2 attempts each, then the
//   colour-1 tiles; tile tile_id = ty*T + tx (T = L/D) in phase p takes its
//   sites from Philox counters (j, tile_id, s, p).
//
// Kernels:
//   block_sweep  one workgroup owns a TX x TY tile block of the shifted frame
//                plus a ring of D+1 sites.  It loads the block and ring from
//                the input buffer into LDS (aligned 16-byte chunks, stored
//                as int8 or int16 offsets from a per-block reference height
//                when they fit), recomputes the phase-0 update of the
//                colour-0 tiles just outside the block (their inputs are all
//                in the ring, and the update is a pure function of them),
//                runs phase 1 on the block, stores the block into the output
//                buffer and adds its (S1, S2, A) increments to one of the
//                surface's 64 accumulator slots; the surface's last block
//                folds them into the per-sweep log.  A sweep, sums included,
//                is one launch and costs one read and one write of every
//                site.  An int8 block whose range does not fit is swept
//                again by the same workgroup as int16 sub-blocks.
//   block_sweep16  the same on heights kept in HBM as 16-bit residues
//                (half the bytes per sweep) when N L <= 32766.
//   lds_run      a whole small surface (L^2 * 4 bytes fits in LDS) lives in
//                one workgroup's LDS for many sweeps; no per-sweep launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rsosk {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).  Ten rounds; each round multiplies
// counter words 0 and 2 by the two round multipliers, mixes the high halves
// with words 1, 3 and the key, and the key advances by the two Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t v[4];
};

__host__ __device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                         uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)c0 * 0xD2511F53ull;
        const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57ull;
        const uint32_t n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    u32x4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// ---------------------------------------------------------------------------
// Per-surface state shared by the kernels.  Lives in device memory; the
// host writes it at setup and sets t_end before a run; the sweep's last
// block (or lds_run) advances t.
// ---------------------------------------------------------------------------
constexpr int kAccSlots = 64;  // per-surface spread of the (S1, S2, A) atomics
// Per-surface accumulator area: 3 * kAccSlots words of increments, then
// word kMeanWord = floor(S1 / L^2) of the current time (kept by the sweep's
// last block; the 16-bit storage mode recovers true heights from it, every
// block reads it) and, in a 128-byte line of its own so that the blocks'
// atomic additions to it do not stall those reads, word kDoneWord, the
// blocks of the running sweep that have committed.  All words but
// kMeanWord are zero between sweeps.  Areas are 128-byte aligned.
constexpr int kMeanWord = 3 * kAccSlots;
constexpr int kDoneWord = kMeanWord + 16;
constexpr int kAccWords = kDoneWord + 16;

// Lattice pointers reach the kernels through descriptors in memory, so the
// compiler sees generic pointers and would emit flat memory instructions
// (which also count against the LDS wait counter).  They always point to
// device global memory: accesses go through these global-address-space
// views.
typedef __attribute__((address_space(1))) int32_t gint32;
typedef __attribute__((address_space(1))) unsigned long long gu64;
typedef __attribute__((address_space(1))) long long gi64;
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4i gv4i;

__device__ __forceinline__ const gint32 *as_global(const int32_t *p) { return (const gint32 *)p; }
__device__ __forceinline__ gint32 *as_global(int32_t *p) { return (gint32 *)p; }

__device__ __forceinline__ int4 load4(const gint32 *p)
{
    const v4i x = *reinterpret_cast<const gv4i *>(p);
    return make_int4(x.x, x.y, x.z, x.w);
}

__device__ __forceinline__ void store4(gint32 *p, const int4 v)
{
    const v4i x = {v.x, v.y, v.z, v.w};
    *reinterpret_cast<gv4i *>(p) = x;
}

struct SurfDev {
    int32_t *buf[2];      // state after t sweeps is in buf[t & 1]
    long long *log;       // 3 * log_cap int64: (S1, S2, A) of time tau at slot tau % log_cap
    long long *acc;       // kAccWords int64: accumulators (zero between sweeps), mean floor
    long long log_cap;
    long long t;          // sweeps done
    long long t_end;      // run while t < t_end
    uint32_t key0, key1;  // Philox key = seed
    int L, N, T;          // T = L / D
    int nbx;              // blocks along x (block path)
    int nblocks;          // blocks of this surface (block path)
    int block_start;      // first global block index of this surface
};

template <int D>
struct TileBits {
    static constexpr int LOG2D = (D == 2) ? 1 : (D == 4) ? 2 : (D == 8) ? 3 : (D == 16) ? 4 : 5;
    static constexpr int B = 2 * LOG2D;               // bits per site field
    static constexpr int F = 32 / B;                  // fields per 32-bit word
    static constexpr int PER = 4 * F;                 // attempts per Philox call
    static constexpr int NCALL = (D * D + PER - 1) / PER;
};

// Geometry of a TX x TY tile block with its ring of D+1 sites, as staged in
// LDS: region rows of RW sites in RWL elements (CH chunks; the rows are laid
// RWL elements apart, or RowPitch below for byte staging), shifted right by
// the alignment pad (0..CPC-1) of the region's first column so that every
// global load is an aligned 16-byte chunk of CPC cells (4 int32 or 8 uint16).
template <int D, int TX, int TY, int CPC = 4>
struct BlockGeom {
    static constexpr int RING = D + 1;
    static constexpr int RW = TX * D + 2 * RING;
    static constexpr int RH = TY * D + 2 * RING;
    static constexpr int RWL = (RW + 2 * (CPC - 1)) & ~(CPC - 1);
    static constexpr int CH = RWL / CPC;
    static constexpr int HALF = TX * TY / 2;
    static constexpr int P0 = HALF + TX + TY;
    static constexpr int BW = TX * D, BH = TY * D;
};

// One attempt on the site at field f of a tile whose site (u, v) sits at LDS
// index base + v*P + u (neighbours at +-1 and +-P).  E is the LDS element
// type: narrow types hold heights relative to a per-block base, int32 raw
// heights.  Adds the acceptance to acc (minus the acceptance with unsigned
// byte staging) and, when accepted, the staged value c before the deposit
// to q (a deposit on height h raises sum h^2 by 2h + 1).
template <int D, int P, typename E, typename Q>
__device__ __forceinline__ void attempt(E *lds, int base, uint32_t f, int N, int &acc, Q &q)
{
    constexpr int LOG2D = TileBits<D>::LOG2D;
    const int idx = base + (int)(f >> LOG2D) * P + (int)(f & (D - 1));
    int c, m;
    if constexpr (std::is_same<E, uint8_t>::value) {
        // unsigned byte staging (LDS-bound): the left neighbour, the site and
        // the right neighbour from one read of the two aligned words around
        // them (measured slower on the HBM-bound int8 path, so not used there).
        // Every access is addressed from i1 = idx - 1; the byte shift of
        // v_alignbyte uses the low two bits of its operand only.
        const int i1 = (base - 1) + (int)__umul24(f >> LOG2D, (uint32_t)P) + (int)(f & (D - 1));
        const uint32_t *w = reinterpret_cast<const uint32_t *>(lds + (i1 & ~3));
        const uint32_t t3 = __builtin_amdgcn_alignbyte(w[1], w[0], (uint32_t)i1);
        // min(left, right) straight from bytes 0 and 2 of t3 (one instruction
        // where the compiler would extract both bytes first)
        uint32_t lr;
        asm("v_min_u16_sdwa %0, %1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:BYTE_2"
            : "=v"(lr) : "v"(t3));
        c = (int)((t3 >> 8) & 0xFFu);
        m = (int)min(min(lr, (uint32_t)lds[i1 + 1 - P]), (uint32_t)lds[i1 + 1 + P]);
        // all ones if accepted, else zero
        const int nok = (c - m - N) >> 31;
        // c & nok and c - nok with c taken as byte 1 of t3 by the
        // instructions themselves
        int qc, cn;
        asm("v_and_b32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
            : "=v"(qc) : "v"(nok), "v"(t3));
        asm("v_sub_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1 src1_sel:DWORD"
            : "=v"(cn) : "v"(t3), "v"(nok));
        q += qc;
        lds[i1 + 1] = (E)cn;
        // this staging counts acceptances negatively (one instruction less
        // per attempt); region_sweep16 negates the block's count
        acc += nok;
        return;
    } else {
        c = lds[idx];
        m = min(min((int)lds[idx - 1], (int)lds[idx + 1]), min((int)lds[idx - P], (int)lds[idx + P]));
    }
    // h_c + 1 - h_j <= N for every neighbour j; the lower side cannot fail
    // because |h_c - h_j| <= N held before.
    int ok;
    if constexpr (sizeof(E) <= 2) {
        // narrow staging: c - m and N are far inside int range, so the sign
        // of c - m - N decides
        ok = (int)((uint32_t)(c - m - N) >> 31);
        q += __mul24(c, ok);
    } else {
        ok = (c - m) < N;
        q += ok ? (Q)c : (Q)0;
    }
    lds[idx] = (E)(c + ok);
    acc += ok;
}

// D^2 sequential attempts of one tile: the Philox calls whose fields are
// all used, then the call that holds the last D^2 mod (fields per call).
template <int D, int P, typename E, typename Q>
__device__ __forceinline__ void tile_attempts(E *lds, int base, uint32_t tile_id, uint32_t s,
                                              uint32_t p, int N, uint32_t k0, uint32_t k1,
                                              int &acc, Q &q)
{
    using TB = TileBits<D>;
    constexpr int NFULL = (D * D) / TB::PER, TAIL = (D * D) % TB::PER;
    constexpr uint32_t MASK = (uint32_t)(D * D - 1);
#pragma unroll 1
    for (int j = 0; j < NFULL; ++j) {
        const u32x4 r = philox4x32_10((uint32_t)j, tile_id, s, p, k0, k1);
#pragma unroll
        for (int k = 0; k < TB::PER; ++k)
            attempt<D, P, E, Q>(lds, base, (r.v[k / TB::F] >> ((k % TB::F) * TB::B)) & MASK, N, acc, q);
    }
    if constexpr (TAIL > 0) {
        const u32x4 r = philox4x32_10((uint32_t)NFULL, tile_id, s, p, k0, k1);
#pragma unroll
        for (int k = 0; k < TAIL; ++k)
            attempt<D, P, E, Q>(lds, base, (r.v[k / TB::F] >> ((k % TB::F) * TB::B)) & MASK, N, acc, q);
    }
}

__device__ __forceinline__ void wave_reduce3(long long &a, long long &b, long long &c)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
        c += __shfl_xor(c, off, 64);
    }
}

// Result valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_reduce3(long long &a, long long &b, long long &c)
{
    __shared__ long long red[3][NT / 64 > 0 ? NT / 64 : 1];
    wave_reduce3(a, b, c);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (NT > 64) {
        if (l == 0) { red[0][w] = a; red[1][w] = b; red[2][w] = c; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < NT / 64; ++i) { a += red[0][i]; b += red[1][i]; c += red[2][i]; }
        }
    }
}

template <typename E>
__device__ __forceinline__ void lds_put4(E *dst, const int4 v, int ref);

template <>
__device__ __forceinline__ void lds_put4<int16_t>(int16_t *dst, const int4 v, int ref)
{
    const uint32_t lo = (uint32_t)(uint16_t)(v.x - ref) | ((uint32_t)(uint16_t)(v.y - ref) << 16);
    const uint32_t hi = (uint32_t)(uint16_t)(v.z - ref) | ((uint32_t)(uint16_t)(v.w - ref) << 16);
    *reinterpret_cast<uint2 *>(dst) = make_uint2(lo, hi);
}

template <>
__device__ __forceinline__ void lds_put4<int8_t>(int8_t *dst, const int4 v, int ref)
{
    const uint32_t w = (uint32_t)(uint8_t)(v.x - ref) | ((uint32_t)(uint8_t)(v.y - ref) << 8) |
                       ((uint32_t)(uint8_t)(v.z - ref) << 16) | ((uint32_t)(uint8_t)(v.w - ref) << 24);
    *reinterpret_cast<uint32_t *>(dst) = w;
}

template <>
__device__ __forceinline__ void lds_put4<int32_t>(int32_t *dst, const int4 v, int)
{
    *reinterpret_cast<int4 *>(dst) = v;
}

template <typename E> struct Lds4;
template <> struct Lds4<int16_t> {
    typedef uint2 raw;
    __device__ static int4 widen(const uint2 w, int ref)
    {
        return make_int4(ref + (int)(int16_t)(w.x & 0xFFFF), ref + (int)(int16_t)(w.x >> 16),
                         ref + (int)(int16_t)(w.y & 0xFFFF), ref + (int)(int16_t)(w.y >> 16));
    }
};
template <> struct Lds4<int8_t> {
    typedef uint32_t raw;
    __device__ static int4 widen(const uint32_t w, int ref)
    {
        return make_int4(ref + (int)(int8_t)(w & 0xFF), ref + (int)(int8_t)((w >> 8) & 0xFF),
                         ref + (int)(int8_t)((w >> 16) & 0xFF), ref + (int)(int8_t)(w >> 24));
    }
};
template <> struct Lds4<int32_t> {
    typedef int4 raw;
    __device__ static int4 widen(const int4 w, int) { return w; }
};





// The next sweep reads the output from HBM long after this one wrote it:
// stream the full 16-byte chunks past the caches.
__device__ __forceinline__ void store4_stream(gint32 *dst, const int4 v)
{
    const v4i x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<gv4i *>(dst));
}

// Descriptor index of the surface that owns global block lb: from the
// host-built table when there is one (one load), else by binary search over
// the descriptors (sorted by block_start).
__device__ __forceinline__ int find_surface(const SurfDev *descs, int nsurf, const int *owner, int lb)
{
    if (owner) return owner[lb];
    int lo = 0, hi = nsurf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].block_start <= lb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Both phases of one sweep on a block staged in LDS with row pitch RWL and
// block column 0 at column off of region row RING.  Phase 0: the colour-0
// tiles of the block, then the colour-0 ring tiles that touch the block's
// colour-1 border tiles (their counts belong to the neighbouring blocks and
// are dropped); phase 1: the colour-1 tiles of the block.  acc and q receive
// this thread's accepted count and sum of accepted staged values.
template <int D, int TX, int TY, int NT, int RWL, typename E, typename Q>
__device__ __forceinline__ void block_phases(E *lds, int off, int bx, int by, int T, uint32_t s, int N,
                                             uint32_t k0, uint32_t k1, int &acc, Q &q)
{
    constexpr int RING = D + 1, HALF = TX * TY / 2, P0 = HALF + TX + TY;
    for (int k = threadIdx.x; k < P0; k += NT) {
        int ltx, lty;
        if (k < HALF) {
            lty = k / (TX / 2);
            ltx = 2 * (k % (TX / 2)) + (lty & 1);
        } else {
            const int g = k - HALF;
            if (g < TX / 2) { lty = -1; ltx = 2 * g + 1; }
            else if (g < TX) { lty = TY; ltx = 2 * (g - TX / 2); }
            else if (g < TX + TY / 2) { ltx = -1; lty = 2 * (g - TX) + 1; }
            else { ltx = TX; lty = 2 * (g - TX - TY / 2); }
        }
        int gtx = bx * TX + ltx, gty = by * TY + lty;
        gtx = gtx < 0 ? gtx + T : (gtx >= T ? gtx - T : gtx);
        gty = gty < 0 ? gty + T : (gty >= T ? gty - T : gty);
        const int base = (lty * D + RING) * RWL + ltx * D + off;
        int a = 0;
        Q qq = 0;
        tile_attempts<D, RWL, E, Q>(lds, base, (uint32_t)(gty * T + gtx), s, 0u, N, k0, k1, a, qq);
        if (k < HALF) { acc += a; q += qq; }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < HALF; k += NT) {
        const int lty = k / (TX / 2);
        const int ltx = 2 * (k % (TX / 2)) + 1 - (lty & 1);
        const int gtx = bx * TX + ltx, gty = by * TY + lty;
        const int base = (lty * D + RING) * RWL + ltx * D + off;
        tile_attempts<D, RWL, E, Q>(lds, base, (uint32_t)(gty * T + gtx), s, 1u, N, k0, k1, acc, q);
    }
    __syncthreads();
}

// The double-tiling schedule on the same block (TX x TY sub-tiles of D,
// TX and TY even, so a block holds whole 2 x 2 tiles).  Set k = (sx mod 2)
// + 2 (sy mod 2) is updated in phase k with Philox phase code 4 + k.  The
// block's border sub-tiles read sub-tiles of the neighbouring blocks; those
// updated in an earlier phase are recomputed here, in their phase: the
// set-0 sub-tiles of the frame column right of the block and of the frame
// row below it (and the corner between them) in phase 0, the set-1
// sub-tiles of the row below in phase 1, the set-2 sub-tiles of the column
// to the right in phase 2.  Their inputs are original values or values
// this block has already brought to the same phase; the frames above and
// to the left are read only before their own updates.  Counts of frame
// sub-tiles are dropped.
template <int D, int TX, int TY, int NT, int RWL, typename E, typename Q>
__device__ __forceinline__ void block_phases_dt(E *lds, int off, int bx, int by, int T, uint32_t s, int N,
                                                uint32_t k0, uint32_t k1, int &acc, Q &q)
{
    static_assert(TX % 2 == 0 && TY % 2 == 0, "blocks hold whole 2 x 2 tiles");
    constexpr int RING = D + 1, Q4 = TX * TY / 4;
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        const int extra = k == 0 ? TX / 2 + TY / 2 + 1 : k == 1 ? TX / 2 : k == 2 ? TY / 2 : 0;
        for (int i = threadIdx.x; i < Q4 + extra; i += NT) {
            int ltx, lty;
            if (i < Q4) {
                lty = 2 * (i / (TX / 2)) + (k >> 1);
                ltx = 2 * (i % (TX / 2)) + (k & 1);
            } else {
                const int g = i - Q4;
                if (k == 0) {
                    if (g < TY / 2) { ltx = TX; lty = 2 * g; }
                    else if (g < TY / 2 + TX / 2) { lty = TY; ltx = 2 * (g - TY / 2); }
                    else { ltx = TX; lty = TY; }
                } else if (k == 1) {
                    lty = TY;
                    ltx = 2 * g + 1;
                } else {
                    ltx = TX;
                    lty = 2 * g + 1;
                }
            }
            int gsx = bx * TX + ltx, gsy = by * TY + lty;
            if (gsx >= T) gsx -= T;
            if (gsy >= T) gsy -= T;
            const int base = (lty * D + RING) * RWL + ltx * D + off;
            int a = 0;
            Q qq = 0;
            tile_attempts<D, RWL, E, Q>(lds, base, (uint32_t)(gsy * T + gsx), s, 4u + (uint32_t)k, N, k0, k1, a, qq);
            if (i < Q4) { acc += a; q += qq; }
        }
        __syncthreads();
    }
}

// Schedule selector: 0 = tile checkerboard, 1 = double tiling.
template <int SCHED, int D, int TX, int TY, int NT, int RWL, typename E, typename Q>
__device__ __forceinline__ void sweep_phases(E *lds, int off, int bx, int by, int T, uint32_t s, int N,
                                             uint32_t k0, uint32_t k1, int &acc, Q &q)
{
    if constexpr (SCHED == 0)
        block_phases<D, TX, TY, NT, RWL, E, Q>(lds, off, bx, by, T, s, N, k0, k1, acc, q);
    else
        block_phases_dt<D, TX, TY, NT, RWL, E, Q>(lds, off, bx, by, T, s, N, k0, k1, acc, q);
}

// ---------------------------------------------------------------------------
// End of a sweep.  Every block adds its increments (A, sum(2h + 1) over its
// accepted deposits, A) of S1, S2 and the accepted count to one of the
// surface's 64 accumulator slots and counts itself in the surface's done
// word; the block that completes the count folds the slots into the record
// of time t + 1 (the record of t plus the increments), clears them, keeps
// floor(S1 / L^2) and advances the surface's time.  So one launch is a
// whole sweep, and the sums are exact whatever order the blocks finish in.
// All of it uses device-scope atomics without fences (an acquire or release
// at device scope would write back or invalidate the XCD's whole L2 in
// every block): a block counts itself only after its three slot additions
// have been performed (it waits for them), and the last block reads the
// slots with device-scope atomic loads.  Its plain stores (time, log
// record, mean) are read by later launches only.
// ---------------------------------------------------------------------------

// Wave 0 of the block that completed the count.
__device__ __forceinline__ void finish_sweep(SurfDev &d, long long t)
{
    const int lane = threadIdx.x;  // < 64
    gu64 *a = (gu64 *)(d.acc + 3 * lane);
    long long x = (long long)__hip_atomic_load(a + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long long y = (long long)__hip_atomic_load(a + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long long z = (long long)__hip_atomic_load(a + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a + 0, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a + 2, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wave_reduce3(x, y, z);
    if (lane == 0) {
        const gi64 *prev = (const gi64 *)(d.log + 3 * (t % d.log_cap));
        gi64 *e = (gi64 *)(d.log + 3 * ((t + 1) % d.log_cap));
        const long long s1 = prev[0] + x, s2 = prev[1] + y;
        e[0] = s1;
        e[1] = s2;
        e[2] = z;
        *(gi64 *)(d.acc + kMeanWord) = s1 / ((long long)d.L * d.L);
        __hip_atomic_store((gu64 *)(d.acc + kDoneWord), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *(gi64 *)&d.t = t + 1;
    }
}

// a = this thread's accepted count, s2 = its share of the S2 increment.
// Called by the whole workgroup once its sums are final (before its
// stores: nothing here depends on them).
template <int NT>
__device__ __forceinline__ void commit_sweep(SurfDev &d, int b, long long a, long long s2, long long t)
{
    __shared__ int s_last;
    long long unused = 0;
    block_reduce3<NT>(a, s2, unused);
    if (threadIdx.x == 0) {
        gu64 *slot = (gu64 *)(d.acc + 3 * (b & (kAccSlots - 1)));
        __hip_atomic_fetch_add(slot + 0, (unsigned long long)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(slot + 1, (unsigned long long)s2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(slot + 2, (unsigned long long)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the three additions are performed before the block is counted
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        const unsigned long long prev = __hip_atomic_fetch_add((gu64 *)(d.acc + kDoneWord), 1ull,
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = prev + 1 == (unsigned long long)d.nblocks;
    }
    __syncthreads();
    if (s_last && threadIdx.x < 64) finish_sweep(d, t);
}

// Workgroup -> global block.  Mode 1: the dispatcher hands consecutive
// workgroup ids to the 8 XCDs in turn; each XCD takes runs of 16 consecutive
// blocks (left and right neighbours share its L2 for their ring columns)
// while the 8 XCDs together walk the lattice in memory order; blocks beyond
// the last whole group of 8 x 16 keep their number.  Mode 2 (one surface,
// nbx % 8 == 0): XCD x owns the block columns [x nbx/8, (x+1) nbx/8) and
// walks them row by row, so a block's upper and lower neighbours, whose
// regions overlap its ring rows, run on the same XCD; all XCDs still move
// down the lattice together.  Mode 0: identity.
__device__ __forceinline__ int block_map(int wg, int n, int mode, int nbx)
{
    if (mode == 1) {
        constexpr int C = 16;
        const int full = n - n % (8 * C);
        if (wg >= full) return wg;
        const int x = wg & 7, j = wg >> 3;
        return (j / C) * (8 * C) + x * C + (j % C);
    }
    if (mode == 2) {
        const int sw = nbx >> 3, x = wg & 7, j = wg >> 3;
        return (j / sw) * nbx + x * sw + j % sw;
    }
    return wg;
}

// LDS row pitch of a byte-staged region.  Rounded up to a multiple of 64
// bytes (half the 32 banks) it spreads the lanes of a wavefront over the
// banks more evenly than the bare row length does, at the price of LDS per
// block: done for the tile checkerboard where that price is at most 15%
// (rows of 32 tiles at D = 8: 280 or 288 -> 320 bytes; measured faster),
// not for narrower rows or the double-tiling schedule, whose latency-bound
// phases need the blocks per CU more (measured slower).
template <int ES, int RWL, int SCHED>
struct RowPitch {
    static constexpr int padded = (RWL + 63) & ~63;
    static constexpr int v = (ES == 1 && SCHED == 0 && 100 * padded <= 115 * RWL) ? padded : RWL;
};

// LDS bytes of a block's narrow staging with its row pitch.
template <int D, int TX, int TY, int CPC, int ES, int SCHED>
struct NarrowBytes {
    using G = BlockGeom<D, TX, TY, CPC>;
    static constexpr int v = RowPitch<ES, G::RWL, SCHED>::v * G::RH * ES;
};

// Where a block's staging does not fit its narrow element type, the same
// workgroup sweeps it again as SX x SY sub-blocks with the wide type EW.
// The tile block shape never changes results (each sub-block recomputes the
// ring tiles it reads), so the sub-blocks reproduce the block's bits.  The
// split is the smallest one whose wide staging fits the LDS of the narrow
// one (sub-blocks keep whole checkerboard pairs: even tile counts, and rows
// the store can tile); with no such split the LDS is the larger of the two.
template <int D, int TX, int TY, int NT, int CPC, int ES, int EWS>
struct WideSplit {
    template <int SX, int SY>
    static constexpr bool ok()
    {
        return TX % SX == 0 && TY % SY == 0 && (TX / SX) % 2 == 0 && (TY / SY) % 2 == 0 &&
               ((TX / SX) * D) % CPC == 0 && NT % ((TX / SX) * D / CPC) == 0;
    }
    template <int SX, int SY>
    static constexpr int bytes()
    {
        using G = BlockGeom<D, TX / SX, TY / SY, CPC>;
        return G::RWL * G::RH * EWS;
    }
    static constexpr int MAIN = BlockGeom<D, TX, TY, CPC>::RWL * BlockGeom<D, TX, TY, CPC>::RH * ES;
    static constexpr int pick()  // 0: 1x1, 1: 2x1, 2: 1x2, 3: 2x2
    {
        if (EWS == 0) return 0;
        if (bytes<1, 1>() <= MAIN) return 0;
        if (ok<2, 1>() && bytes<2, 1>() <= MAIN) return 1;
        if (ok<1, 2>() && bytes<1, 2>() <= MAIN) return 2;
        if (ok<2, 2>() && bytes<2, 2>() <= MAIN) return 3;
        if (ok<2, 2>()) return 3;
        return 0;
    }
    static constexpr int K = pick();
    static constexpr int SX = (K & 1) ? 2 : 1, SY = (K & 2) ? 2 : 1;
    static constexpr int WIDE = EWS == 0 ? 0 : bytes<(K & 1) ? 2 : 1, (K & 2) ? 2 : 1>();
    static constexpr int BYTES = MAIN > WIDE ? MAIN : WIDE;
};

template <typename EW> struct WideSize { static constexpr int v = sizeof(EW); };
template <> struct WideSize<void> { static constexpr int v = 0; };

// Waves per SIMD that the LDS of a kernel with a wide path allows (the
// larger of its narrow staging, with its row pitch, and its wide sub-blocks;
// 160 KB per CU, 4 SIMDs, at most 7).  For D = 8 the register budget is held to
// it, so that the rarely taken wide path (whose registers the compiler then
// spills, in that path only) does not lower the occupancy of the main one;
// for the other domain sizes the budget would force spills into the main
// path, and the compiler's own allocation is kept.  A workgroup of NT
// threads puts NT / 256 waves on each SIMD, so the count is a multiple of
// that; 256 bytes stand for the kernel's small static arrays.
template <int D, int TX, int TY, int NT, int CPC, int ES, int EWS, int SCHED = 0>
struct WideOcc {
    static constexpr int W = WideSplit<D, TX, TY, NT, CPC, ES, EWS>::BYTES;
    static constexpr int N = NarrowBytes<D, TX, TY, CPC, ES, SCHED>::v;
    static constexpr int lds = (W > N ? W : N) + 256;
    static constexpr int per = NT >= 256 ? NT / 256 : 1;
    static constexpr int w0 = (163840 / lds) * (NT / 64) / 4;
    static constexpr int w = ((w0 > 7 ? 7 : w0) / per) * per;
    static constexpr int v = (EWS == 0 || D != 8) ? 1 : (w < 1 ? 1 : w);
};

// ---------------------------------------------------------------------------
// One region (a TX x TY tile block of the shifted frame, block coordinates
// (bx, by) in units of that shape) of sweep s, int32 heights in HBM: stage
// the region and its ring of D+1 sites in LDS, run both phases, store the
// region's tiles.  With a narrow element type that is range-checked (int8)
// it returns false, having written nothing, when some staged value could
// leave the type during the sweep.  Adds the thread's accepted count to ca
// and its share of the S2 increment to cs2.
// Host requirements: T % TX == 0, T % TY == 0, TX and TY even, RWL <= L,
// RH <= L, 16-byte aligned buffers, and for E = int16
// N * (RW + RH + 4) + D^2 <= 32767 (every staged value stays within int16
// of the reference: any two region sites are joined by a path of at most
// RW + RH - 2 bonds, each of height difference <= N, and no site gains
// more than D^2 in a sweep).
// ---------------------------------------------------------------------------
template <int D, int TX, int TY, int NT, typename E, int SCHED, int U = 8>
__device__ __forceinline__ bool region_sweep(E *lds, SurfDev &d, int bx, int by, long long t, int ox, int oy,
                                             int *s_bad, long long &ca, long long &cs2, bool commit_here, int b)
{
    constexpr int PP = RowPitch<(int)sizeof(E), BlockGeom<D, TX, TY, 4>::RWL, SCHED>::v;
    const uint32_t s = (uint32_t)t;
    using G = BlockGeom<D, TX, TY>;
    using Q = typename std::conditional<sizeof(E) <= 2, int, long long>::type;
    constexpr bool checked = sizeof(E) == 1;
    const int L = d.L, N = d.N, T = d.T;
    const uint32_t k0 = d.key0, k1 = d.key1;
    const gint32 *__restrict__ hin = as_global(d.buf[s & 1u]);
    gint32 *__restrict__ hout = as_global(d.buf[(s + 1u) & 1u]);

    int gx0 = ox + bx * TX * D - G::RING;
    int gy0 = oy + by * TY * D - G::RING;
    if (gx0 < 0) gx0 += L;
    if (gy0 < 0) gy0 += L;
    const int cpad = gx0 & 3;
    const int gxa = gx0 - cpad;  // LDS column c holds global column gxa + c (mod L)
    const int ref = (sizeof(E) <= 2) ? hin[(size_t)gy0 * L + gx0] : 0;

    int vmin = 0x7FFFFFFF, vmax = -0x7FFFFFFF;  // range of the staged heights (int8 staging)
    // ---- load the region in aligned 16-byte chunks, consecutive threads on
    // consecutive chunks (rows run on into the next), U chunks in flight per
    // thread; chunk i sits at region row i / CH, chunk column i % CH
    {
        constexpr int NCH = G::CH * G::RH;
        constexpr int FULL = NCH / (NT * U);  // groups in which every thread has U chunks
        auto fetch = [&](int i) {
            const int r = i / G::CH, cc = i - r * G::CH;
            int gy = gy0 + r;
            if (gy >= L) gy -= L;
            int gx = gxa + 4 * cc;
            if (gx >= L) gx -= L;
            if (gx >= L) gx -= L;  // a block as wide as the lattice: the region wraps twice
            return load4(hin + (size_t)gy * L + gx);
        };
        auto stage = [&](int i, const int4 &v) {
            const int r = i / G::CH, cc = i - r * G::CH;
            lds_put4<E>(lds + r * PP + 4 * cc, v, ref);
            if (checked) {
                vmin = min(vmin, min(min(v.x, v.y), min(v.z, v.w)));
                vmax = max(vmax, max(max(v.x, v.y), max(v.z, v.w)));
            }
        };
#pragma unroll 1
        for (int g = 0; g < FULL; ++g) {
            const int i0 = g * NT * U + threadIdx.x;
            int4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = fetch(i0 + u * NT);
#pragma unroll
            for (int u = 0; u < U; ++u) stage(i0 + u * NT, v[u]);
        }
        {
            const int i0 = FULL * NT * U + threadIdx.x;
            int4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < NCH) v[u] = fetch(i0 + u * NT);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < NCH) stage(i0 + u * NT, v[u]);
        }
    }
    if (checked) {
        // every value of the sweep stays in [min, max + N D]: heights never
        // decrease, and a tile site is never more than N D/2 above the
        // frozen sites around its tile (a path of at most D/2 bonds), whose
        // values grow by at most N D/2 in the first phase
        if (vmin - ref < -128 || (long long)vmax - ref + (long long)N * D > 127) *s_bad = 1;
    }
    __syncthreads();
    if (checked && *(volatile int *)s_bad) return false;  // uniform: the whole workgroup

    const int off = G::RING + cpad;  // LDS column of block column 0
    int acc = 0;
    Q q = 0;
    sweep_phases<SCHED, D, TX, TY, NT, PP, E, Q>(lds, off, bx, by, T, s, N, k0, k1, acc, q);
    // a deposit on h raises S2 by 2h + 1; the staged value c stands for ref + c
    ca += acc;
    cs2 += 2ll * (long long)q + (long long)acc + 2ll * (long long)ref * acc;
    // the block's sums are final: commit them before the stores, which
    // other workgroups then overlap
    if (commit_here) commit_sweep<NT>(d, b, ca, cs2, t);

    // ---- store the block: aligned 16-byte chunks (LDS and global columns
    // share their alignment), masked single stores in the partial chunks
    {
        constexpr int SPR = G::BW / 4;  // chunk slots per row, from the first (maybe partial) one
        static_assert(NT % SPR == 0, "threads must tile whole block rows");
        constexpr int RPP = NT / SPR;   // rows per pass of the workgroup
        const int m = off & 3;
        const int slot = threadIdx.x % SPR;
        const int kslot = (off >> 2) + slot;  // LDS chunk index of this thread
        int gc = gxa + 4 * kslot;
        if (gc >= L) gc -= L;
        if (gc >= L) gc -= L;
        const bool partial = slot == 0 && m != 0;
        // chunks whose 128-byte line lies wholly inside the block row are
        // streamed past the caches; lines shared with the neighbouring block
        // go through L2, where the two halves merge (row bases are
        // line-aligned when L % 32 == 0)
        const int row_lo = 4 * (gxa + off), row_hi = row_lo + 4 * G::BW;
        const int line = (4 * (gxa + 4 * kslot)) & ~127;
        const bool whole_line = (L % 32 == 0) && line >= row_lo && line + 128 <= row_hi &&
                                gxa + off + G::BW <= L;
        // (separate loops: the compiler would otherwise merge the two kinds
        // of store into one plain store)
        if (whole_line) {
            for (int r = threadIdx.x / SPR; r < G::BH; r += RPP) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                const E *src = lds + (G::RING + r) * PP + 4 * kslot;
                store4_stream(hout + (size_t)gy * L + gc,
                              Lds4<E>::widen(*reinterpret_cast<const typename Lds4<E>::raw *>(src), ref));
            }
        } else {
            for (int r = threadIdx.x / SPR; r < G::BH; r += RPP) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                gint32 *row = hout + (size_t)gy * L;
                const E *src = lds + (G::RING + r) * PP + 4 * kslot;
                const int4 v = Lds4<E>::widen(*reinterpret_cast<const typename Lds4<E>::raw *>(src), ref);
                if (!partial) {
                    store4(row + gc, v);
                } else {
                    if (m <= 1) row[gc + 1] = v.y;
                    if (m <= 2) row[gc + 2] = v.z;
                    row[gc + 3] = v.w;
                }
            }
        }
        // the trailing partial chunk of each row (cells 0 .. m-1)
        if (m != 0) {
            const int kt = (off >> 2) + SPR;
            int gct = gxa + 4 * kt;
            if (gct >= L) gct -= L;
            if (gct >= L) gct -= L;
            for (int r = threadIdx.x; r < G::BH; r += NT) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                gint32 *row = hout + (size_t)gy * L;
                const E *src = lds + (G::RING + r) * PP + 4 * kt;
                row[gct] = ref + (int)src[0];
                if (m >= 2) row[gct + 1] = ref + (int)src[1];
                if (m >= 3) row[gct + 2] = ref + (int)src[2];
            }
        }
    }
    return true;
}

// The SX x SY sub-blocks (shape TX x TY each) of block (bx, by) with wide
// staging.
template <int D, int TX, int TY, int NT, typename E, int SCHED, int SX, int SY>
__device__ __forceinline__ void wide_sweep(E *lds, SurfDev &d, int bx, int by, long long t, int ox, int oy,
                                           int *s_bad, long long &ca, long long &cs2, int b)
{
#pragma unroll 1
    for (int j = 0; j < SY; ++j)
#pragma unroll 1
        for (int i = 0; i < SX; ++i) {
            __syncthreads();  // the previous stores have read the LDS
            region_sweep<D, TX, TY, NT, E, SCHED, 4>(lds, d, bx * SX + i, by * SY + j, t, ox, oy, s_bad, ca, cs2,
                                                     i == SX - 1 && j == SY - 1, b);
        }
}

// ---------------------------------------------------------------------------
// block_sweep: one sweep for every active surface of the descriptor table,
// int32 heights in HBM; one workgroup per tile block, E the LDS element
// type, EW the wider type for blocks whose range does not fit E (void: E
// always fits).  The whole sweep, its exact sums included, is this one
// launch.
// ---------------------------------------------------------------------------
template <int D, int TX, int TY, int NT, typename E, typename EW, int SCHED = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(
    WideOcc<D, TX, TY, NT, 4, (int)sizeof(E), WideSize<EW>::v, SCHED>::v))) void block_sweep(SurfDev *__restrict__ descs, int nsurf,
                                                  const int *__restrict__ owner, int xmode, int xnbx)
{
    using W = WideSplit<D, TX, TY, NT, 4, (int)sizeof(E), WideSize<EW>::v>;
    constexpr int NB = NarrowBytes<D, TX, TY, 4, (int)sizeof(E), SCHED>::v;
    __shared__ __attribute__((aligned(16))) uint8_t lds_raw[NB > W::BYTES ? NB : W::BYTES];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;

    const int lb = block_map(blockIdx.x, gridDim.x, xmode, xnbx);
    SurfDev &d = descs[find_surface(descs, nsurf, owner, lb)];
    const long long t = d.t;
    if (t >= d.t_end) return;
    const uint32_t s = (uint32_t)t;
    const u32x4 org = philox4x32_10(0u, 0u, s, 2u, d.key0, d.key1);
    const int ox = (int)(org.v[0] % (2u * D));
    const int oy = (int)(org.v[1] % (2u * D));
    const int b = lb - d.block_start;
    const int bx = b % d.nbx, by = b / d.nbx;
    long long ca = 0, cs2 = 0;
    __syncthreads();  // s_bad cleared
    if (__builtin_expect(!region_sweep<D, TX, TY, NT, E, SCHED>((E *)lds_raw, d, bx, by, t, ox, oy, &s_bad, ca, cs2,
                                                                 true, b), 0)) {
        if constexpr (!std::is_void<EW>::value)
            wide_sweep<D, TX / W::SX, TY / W::SY, NT, EW, SCHED, W::SX, W::SY>((EW *)lds_raw, d, bx, by, t, ox, oy,
                                                                           &s_bad, ca, cs2, b);
    }
}

// ---------------------------------------------------------------------------
// 16-bit storage.  Heights live in HBM as residues mod 2^16.  On the torus
// the restriction bounds the spread max h - min h by N L (any two sites are
// joined by a path of at most L bonds), and the mean grows by at most one per
// sweep, so while N L <= 32766 every height of a sweep lies within 2^15 of
// m0 = floor(S1 / L^2) at the sweep's start: h = m0 + int16(r - m0 mod 2^16)
// recovers it from its residue r, and the difference of any two heights is
// the int16 difference of their residues.  The sweep's last block keeps m0
// in the accumulator area.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(1))) uint16_t gu16;
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4u gv4u;

// two 16-bit lanes per 32-bit word, each wrapping mod 2^16
__device__ __forceinline__ uint32_t pk_sub16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_add16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_max16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t,
                              __builtin_elementwise_max(__builtin_bit_cast(u16x2, a), __builtin_bit_cast(u16x2, b)));
}

// Staging from 16-bit residues.  uint8 staging holds u = h - (h_ref - 128),
// checked to lie in [0, 255 - N D] at load time (the same bound as the int8
// staging of int32 heights); int16 staging holds h - h_ref.
template <typename E> struct Stage16;
template <> struct Stage16<uint8_t> {
    static constexpr int bias = 128;
    typedef uint2 raw;
    // 8 lanes of u (two per word) -> 8 bytes; lane maximum into umax
    __device__ static void put(uint8_t *dst, const v4u w, uint32_t &umax)
    {
        umax = pk_max16(umax, pk_max16(pk_max16(w.x, w.y), pk_max16(w.z, w.w)));
        const uint32_t lo = __builtin_amdgcn_perm(w.y, w.x, 0x06040200u);
        const uint32_t hi = __builtin_amdgcn_perm(w.w, w.z, 0x06040200u);
        *reinterpret_cast<uint2 *>(dst) = make_uint2(lo, hi);
    }
    // 8 bytes -> 8 residues (bytes spread to the low halves of 16-bit lanes)
    __device__ static v4u get(const raw r, uint32_t basep)
    {
        v4u o;
        o.x = pk_add16(__builtin_amdgcn_perm(0u, r.x, 0x0C010C00u), basep);
        o.y = pk_add16(__builtin_amdgcn_perm(0u, r.x, 0x0C030C02u), basep);
        o.z = pk_add16(__builtin_amdgcn_perm(0u, r.y, 0x0C010C00u), basep);
        o.w = pk_add16(__builtin_amdgcn_perm(0u, r.y, 0x0C030C02u), basep);
        return o;
    }
};
template <> struct Stage16<int16_t> {
    static constexpr int bias = 0;
    typedef uint4 raw;
    __device__ static void put(int16_t *dst, const v4u w, uint32_t &)
    {
        *reinterpret_cast<uint4 *>(dst) = make_uint4(w.x, w.y, w.z, w.w);
    }
    __device__ static v4u get(const raw r, uint32_t basep)
    {
        v4u o;
        o.x = pk_add16(r.x, basep);
        o.y = pk_add16(r.y, basep);
        o.z = pk_add16(r.z, basep);
        o.w = pk_add16(r.w, basep);
        return o;
    }
};

// region_sweep on 16-bit residues: E = uint8 (range-checked; returns false
// when the region does not fit) or int16.  Host requirements as for
// region_sweep, with chunks of 8 cells: L % 8 == 0, RWL <= L, N L <= 32766,
// N D <= 96, and N (RW + RH + 4) + D^2 <= 32767 for int16.
template <int D, int TX, int TY, int NT, typename E, int SCHED, int U = 8>
__device__ __forceinline__ bool region_sweep16(E *lds, SurfDev &d, int bx, int by, long long t, int ox, int oy,
                                               int *s_bad, long long &ca, long long &cs2, bool commit_here, int b)
{
    const uint32_t s = (uint32_t)t;
    using G = BlockGeom<D, TX, TY, 8>;
    using S = Stage16<E>;
    constexpr int PP = RowPitch<(int)sizeof(E), G::RWL, SCHED>::v;
    constexpr bool checked = sizeof(E) == 1;
    const int L = d.L, N = d.N, T = d.T;
    const uint32_t k0 = d.key0, k1 = d.key1;
    const gu16 *__restrict__ hin = (const gu16 *)d.buf[s & 1u];
    gu16 *__restrict__ hout = (gu16 *)d.buf[(s + 1u) & 1u];

    int gx0 = ox + bx * TX * D - G::RING;
    int gy0 = oy + by * TY * D - G::RING;
    if (gx0 < 0) gx0 += L;
    if (gy0 < 0) gy0 += L;
    const int cpad = gx0 & 7;
    const int gxa = gx0 - cpad;  // LDS column c holds global column gxa + c (mod L)
    const uint32_t ref_r = hin[(size_t)gy0 * L + gx0];
    const uint32_t base_r = (ref_r - S::bias) & 0xFFFFu;  // residue of staged value 0
    const uint32_t basep = base_r * 0x10001u;

    uint32_t umax = 0;
    {
        constexpr int NCH = G::CH * G::RH;
        constexpr int FULL = NCH / (NT * U);
        auto fetch = [&](int i) {
            const int r = i / G::CH, cc = i - r * G::CH;
            int gy = gy0 + r;
            if (gy >= L) gy -= L;
            int gx = gxa + 8 * cc;
            if (gx >= L) gx -= L;
            if (gx >= L) gx -= L;
            return *reinterpret_cast<const gv4u *>(hin + (size_t)gy * L + gx);
        };
        auto stage = [&](int i, const v4u &v) {
            const int r = i / G::CH, cc = i - r * G::CH;
            v4u w;
            w.x = pk_sub16(v.x, basep);
            w.y = pk_sub16(v.y, basep);
            w.z = pk_sub16(v.z, basep);
            w.w = pk_sub16(v.w, basep);
            S::put(lds + r * PP + 8 * cc, w, umax);
        };
#pragma unroll 1
        for (int g = 0; g < FULL; ++g) {
            const int i0 = g * NT * U + threadIdx.x;
            v4u v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = fetch(i0 + u * NT);
#pragma unroll
            for (int u = 0; u < U; ++u) stage(i0 + u * NT, v[u]);
        }
        {
            const int i0 = FULL * NT * U + threadIdx.x;
            v4u v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < NCH) v[u] = fetch(i0 + u * NT);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + u * NT < NCH) stage(i0 + u * NT, v[u]);
        }
    }
    if (checked) {
        // u = h - h_ref + 128 must lie in [0, 255 - N D] (see region_sweep);
        // |h - h_ref| < 2^15, so an out-of-range u shows as a 16-bit lane
        // above 255 - N D
        if ((int)max(umax & 0xFFFFu, umax >> 16) > 255 - N * D) *s_bad = 1;
    }
    __syncthreads();
    if (checked && *(volatile int *)s_bad) return false;

    const int off = G::RING + cpad;
    int acc = 0;
    int q = 0;
    sweep_phases<SCHED, D, TX, TY, NT, PP, E, int>(lds, off, bx, by, T, s, N, k0, k1, acc, q);
    // the unsigned byte staging counts acceptances negatively
    if constexpr (std::is_same<E, uint8_t>::value) acc = -acc;
    {
        // true height of staged value 0: the reference site's height,
        // recovered from m0 of the sweep's start, less the staging bias
        // (read before the block is counted: the sweep's last block
        // rewrites m0)
        const long long m0 = *(const gi64 *)(d.acc + kMeanWord);
        const long long base = m0 + (long long)(int16_t)(uint16_t)(ref_r - (uint32_t)m0) - S::bias;
        ca += acc;
        cs2 += 2ll * (long long)q + (long long)acc + 2ll * base * acc;
    }
    if (commit_here) commit_sweep<NT>(d, b, ca, cs2, t);

    // ---- store: 16-byte chunks of 8 residues; 16-bit stores in the partial
    // chunks at both ends of each row
    {
        constexpr int SPR = G::BW / 8;
        static_assert(NT % SPR == 0, "threads must tile whole block rows");
        constexpr int RPP = NT / SPR;
        const int m = off & 7;
        const int slot = threadIdx.x % SPR;
        const int kslot = (off >> 3) + slot;
        int gc = gxa + 8 * kslot;
        if (gc >= L) gc -= L;
        if (gc >= L) gc -= L;
        const bool partial = slot == 0 && m != 0;
        // byte offsets within the row; rows are 128-byte aligned when L % 64 == 0
        const int row_lo = 2 * (gxa + off), row_hi = row_lo + 2 * G::BW;
        const int line = (2 * (gxa + 8 * kslot)) & ~127;
        const bool whole_line = (L % 64 == 0) && line >= row_lo && line + 128 <= row_hi &&
                                gxa + off + G::BW <= L;
        if (whole_line) {
            for (int r = threadIdx.x / SPR; r < G::BH; r += RPP) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                const E *src = lds + (G::RING + r) * PP + 8 * kslot;
                __builtin_nontemporal_store(S::get(*reinterpret_cast<const typename S::raw *>(src), basep),
                                            reinterpret_cast<gv4u *>(hout + (size_t)gy * L + gc));
            }
        } else {
            for (int r = threadIdx.x / SPR; r < G::BH; r += RPP) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                gu16 *row = hout + (size_t)gy * L;
                const E *src = lds + (G::RING + r) * PP + 8 * kslot;
                if (!partial) {
                    *reinterpret_cast<gv4u *>(row + gc) = S::get(*reinterpret_cast<const typename S::raw *>(src), basep);
                } else {
#pragma unroll
                    for (int k = 1; k < 8; ++k)
                        if (k >= m) row[gc + k] = (uint16_t)(base_r + (uint32_t)(int)src[k]);
                }
            }
        }
        if (m != 0) {
            const int kt = (off >> 3) + SPR;
            int gct = gxa + 8 * kt;
            if (gct >= L) gct -= L;
            if (gct >= L) gct -= L;
            for (int r = threadIdx.x; r < G::BH; r += NT) {
                int gy = gy0 + G::RING + r;
                if (gy >= L) gy -= L;
                gu16 *row = hout + (size_t)gy * L;
                const E *src = lds + (G::RING + r) * PP + 8 * kt;
#pragma unroll
                for (int k = 0; k < 7; ++k)
                    if (k < m) row[gct + k] = (uint16_t)(base_r + (uint32_t)(int)src[k]);
            }
        }
    }
    return true;
}

// int16 sub-blocks of a 16-bit storage block (see wide_sweep).
template <int D, int TX, int TY, int NT, int SCHED, int SX, int SY>
__device__ __forceinline__ void wide_sweep16(int16_t *lds, SurfDev &d, int bx, int by, long long t, int ox, int oy,
                                             int *s_bad, long long &ca, long long &cs2, int b)
{
#pragma unroll 1
    for (int j = 0; j < SY; ++j)
#pragma unroll 1
        for (int i = 0; i < SX; ++i) {
            __syncthreads();  // the previous stores have read the LDS
            region_sweep16<D, TX, TY, NT, int16_t, SCHED, 4>(lds, d, bx * SX + i, by * SY + j, t, ox, oy, s_bad, ca,
                                                             cs2, i == SX - 1 && j == SY - 1, b);
        }
}

// block_sweep on 16-bit residues: uint8 staging, int16 for the blocks that
// do not fit it.
template <int D, int TX, int TY, int NT, int SCHED = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WideOcc<D, TX, TY, NT, 8, 1, 2, SCHED>::v))) void block_sweep16(SurfDev *__restrict__ descs, int nsurf,
                                                    const int *__restrict__ owner, int xmode, int xnbx)
{
    using W = WideSplit<D, TX, TY, NT, 8, 1, 2>;
    constexpr int NB = NarrowBytes<D, TX, TY, 8, 1, SCHED>::v;
    __shared__ __attribute__((aligned(16))) uint8_t lds_raw[NB > W::BYTES ? NB : W::BYTES];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;

    const int lb = block_map(blockIdx.x, gridDim.x, xmode, xnbx);
    SurfDev &d = descs[find_surface(descs, nsurf, owner, lb)];
    const long long t = d.t;
    if (t >= d.t_end) return;
    const uint32_t s = (uint32_t)t;
    const u32x4 org = philox4x32_10(0u, 0u, s, 2u, d.key0, d.key1);
    const int ox = (int)(org.v[0] % (2u * D));
    const int oy = (int)(org.v[1] % (2u * D));
    const int b = lb - d.block_start;
    const int bx = b % d.nbx, by = b / d.nbx;
    long long ca = 0, cs2 = 0;
    __syncthreads();  // s_bad cleared
    // twelve 16-byte loads in flight per thread (the 32 x 8 region of 16-bit
    // residues in one round of 256 threads; measured 1% faster than eight,
    // within the same registers)
    constexpr int U16 = SCHED == 0 ? 12 : 8;
    if (__builtin_expect(!region_sweep16<D, TX, TY, NT, uint8_t, SCHED, U16>(lds_raw, d, bx, by, t, ox, oy, &s_bad, ca,
                                                                              cs2, true, b), 0))
        wide_sweep16<D, TX / W::SX, TY / W::SY, NT, SCHED, W::SX, W::SY>((int16_t *)lds_raw, d, bx, by, t, ox, oy,
                                                                     &s_bad, ca, cs2, b);
}

// Conversions between int32 heights and 16-bit residues (grid-stride).
__global__ void pack16(const int32_t *__restrict__ src, uint16_t *__restrict__ dst, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (uint16_t)(uint32_t)src[i];
}

__global__ void unpack16(const uint16_t *__restrict__ src, int32_t *__restrict__ dst, long long n,
                         const long long *__restrict__ mean_floor)
{
    const long long m0 = *mean_floor;
    const uint32_t r0 = (uint32_t)m0 & 0xFFFFu;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (int32_t)(m0 + (long long)(int16_t)(uint16_t)((uint32_t)src[i] - r0));
}

// ---------------------------------------------------------------------------
// lds_run: surfaces small enough to live in LDS, one workgroup each, all
// their sweeps in one launch.  which[] lists descriptor indices; the LDS is
// L_max^2 int32 of dynamic shared memory.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ int tile_attempts_torus(int32_t *h, int L, int x0, int y0,
                                                   uint32_t tile_id, uint32_t s, uint32_t p, int N,
                                                   uint32_t k0, uint32_t k1)
{
    using TB = TileBits<D>;
    int acc = 0;
#pragma unroll 1
    for (int j = 0; j < TB::NCALL; ++j) {
        const u32x4 r = philox4x32_10((uint32_t)j, tile_id, s, p, k0, k1);
#pragma unroll
        for (int q = 0; q < TB::PER; ++q) {
            if (j * TB::PER + q < D * D) {
                const uint32_t f = (r.v[q / TB::F] >> ((q % TB::F) * TB::B)) & (uint32_t)(D * D - 1);
                int x = x0 + (int)(f & (D - 1));
                int y = y0 + (int)(f >> TB::LOG2D);
                if (x >= L) x -= L;
                if (y >= L) y -= L;
                const int xl = x == 0 ? L - 1 : x - 1, xr = x == L - 1 ? 0 : x + 1;
                const int yu = y == 0 ? L - 1 : y - 1, yd = y == L - 1 ? 0 : y + 1;
                const int c = h[y * L + x];
                const int m = min(min(h[y * L + xl], h[y * L + xr]), min(h[yu * L + x], h[yd * L + x]));
                const int ok = (c - m) < N;
                h[y * L + x] = c + ok;
                acc += ok;
            }
        }
    }
    return acc;
}

template <int D, int NT, int SCHED = 0>
__global__ __launch_bounds__(NT) void lds_run(SurfDev *__restrict__ descs, const int *__restrict__ which)
{
    extern __shared__ int32_t lat[];
    SurfDev &d = descs[which[blockIdx.x]];
    long long t = d.t;
    const long long t_end = d.t_end;
    if (t >= t_end) return;
    const int L = d.L, N = d.N, T = d.T;
    const int n = L * L;
    const uint32_t k0 = d.key0, k1 = d.key1;
    {
        const int32_t *src = d.buf[t & 1];
        for (int i = threadIdx.x; i < n; i += NT) lat[i] = src[i];
    }
    __syncthreads();
    const int half = T * T / 2;
    for (; t < t_end; ++t) {
        const uint32_t s = (uint32_t)t;
        const u32x4 org = philox4x32_10(0u, 0u, s, 2u, k0, k1);
        const int ox = (int)(org.v[0] % (2u * D));
        const int oy = (int)(org.v[1] % (2u * D));
        long long acc = 0;
        if constexpr (SCHED == 0) {
            for (int p = 0; p < 2; ++p) {
                for (int k = threadIdx.x; k < half; k += NT) {
                    const int ty = k / (T / 2);
                    const int tx = 2 * (k % (T / 2)) + ((ty + p) & 1);
                    acc += tile_attempts_torus<D>(lat, L, ox + tx * D, oy + ty * D,
                                                  (uint32_t)(ty * T + tx), s, (uint32_t)p, N, k0, k1);
                }
                __syncthreads();
            }
        } else {
            // double tiling: set p = (sx mod 2) + 2 (sy mod 2), phase code 4 + p
            for (int p = 0; p < 4; ++p) {
                for (int k = threadIdx.x; k < half / 2; k += NT) {
                    const int sy = 2 * (k / (T / 2)) + (p >> 1);
                    const int sx = 2 * (k % (T / 2)) + (p & 1);
                    acc += tile_attempts_torus<D>(lat, L, ox + sx * D, oy + sy * D,
                                                  (uint32_t)(sy * T + sx), s, 4u + (uint32_t)p, N, k0, k1);
                }
                __syncthreads();
            }
        }
        long long s1 = 0, s2 = 0;
        for (int i = threadIdx.x; i < n; i += NT) {
            const long long v = lat[i];
            s1 += v;
            s2 += v * v;
        }
        block_reduce3<NT>(s1, s2, acc);
        if (threadIdx.x == 0) {
            long long *e = d.log + 3 * ((t + 1) % d.log_cap);
            e[0] = s1;
            e[1] = s2;
            e[2] = acc;
        }
        __syncthreads();
    }
    {
        int32_t *dst = d.buf[t_end & 1];
        for (int i = threadIdx.x; i < n; i += NT) dst[i] = lat[i];
    }
    if (threadIdx.x == 0) d.t = t_end;
}

}  // namespace rsosk

// rsos.hip -- host runtime and C ABI of librsos.so (see include/rsos.h).
//
// Launch plan per sweep: one block_sweep launch over every tile block of
// every active surface (the last block of each surface also folds its
// exact sums into the per-sweep log).  The kernel reads the surface time t
// from device memory, so a captured hipGraph of K sweeps replays for any t.  Surfaces whose L^2 int32 fit in LDS run all
// their sweeps in one lds_run launch instead.
#include "rsos.h"
#include "rsos_host.hpp"
#include "rsos_kernels.hpp"
#include "rsos_moments.hpp"
#include "rsos_ms.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

using rsosk::SurfDev;
using rsosh::check_overflow;
using rsosh::fail;
using rsosh::g_last_error;
using rsosh::validate_h0;
using rsosh::w2_of;

namespace {

// Every HIP runtime call of the library goes through HIP_TRY.  A test can
// make the n-th next one on its thread report a failure (rsos_debug_fail)
// to exercise the error paths without a real device error.
#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        if (rsosh::g_fail_countdown > 0 && --rsosh::g_fail_countdown == 0)                  \
            return fail(RSOS_E_DEVICE, "%s: failure injected by rsos_debug_fail", #expr);   \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(RSOS_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kLdsMaxBytes = 64 * 1024;  // lds_run: whole surface in LDS
constexpr int kGraphSweeps = 32;
constexpr long long kNoEnd = 0x7FFFFFFFFFFFFFFFll;  // t_end of a surface with no bound
constexpr int kPsGrid = 2048;       // workgroups of the power-sum reduction

// ---------------------------------------------------------------------------
// Block-kernel variants.  The tile block shape never changes results; it
// only has to tile the lattice: T % TX == 0, T % TY == 0, region <= L.
// ---------------------------------------------------------------------------
// e0 / e1: events recorded by the runtime when the kernel starts / ends
// (hipExtLaunchKernel), for the timing mode; nullptr otherwise.
typedef void (*BlockLaunch)(dim3, hipStream_t, SurfDev *, int, const int *, int, int, hipEvent_t, hipEvent_t);

// E: LDS element type; EW: wider type for the blocks whose range does not
// fit E (void: E always fits); SCHED 1: the double-tiling schedule
template <int D, int TX, int TY, int NT, typename E, typename EW, int SCHED>
void launch_block(dim3 grid, hipStream_t st, SurfDev *d, int n, const int *owner, int xmode, int xnbx, hipEvent_t e0,
                  hipEvent_t e1)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL((rsosk::block_sweep<D, TX, TY, NT, E, EW, SCHED>), grid, dim3(NT), 0, st, e0, e1, 0, d,
                              n, owner, xmode, xnbx);
    else
        hipLaunchKernelGGL((rsosk::block_sweep<D, TX, TY, NT, E, EW, SCHED>), grid, dim3(NT), 0, st, d, n, owner,
                           xmode, xnbx);
}

template <int D, int TX, int TY, int NT>
void launch_block16(dim3 grid, hipStream_t st, SurfDev *d, int n, const int *owner, int xmode, int xnbx, hipEvent_t e0,
                    hipEvent_t e1)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL((rsosk::block_sweep16<D, TX, TY, NT>), grid, dim3(NT), 0, st, e0, e1, 0, d, n, owner,
                              xmode, xnbx);
    else
        hipLaunchKernelGGL((rsosk::block_sweep16<D, TX, TY, NT>), grid, dim3(NT), 0, st, d, n, owner, xmode, xnbx);
}

// The double-tiling schedule is built for the domain sizes the paper
// compares (8 and 16) on int32 storage.
template <int D, int TX, int TY, int NT, typename E, typename EW>
constexpr BlockLaunch dt_launcher()
{
    if constexpr (D == 8 || D == 16) return launch_block<D, TX, TY, NT, E, EW, 1>;
    else return nullptr;
}

struct Variant {
    int D, TX, TY, NT, elem;  // elem: LDS bytes per site (1 and 2: offsets from a block reference)
    BlockLaunch launch;       // int32 storage (elem 1: int16 sub-blocks where int8 does not fit)
    BlockLaunch launch16;     // 16-bit storage, uint8 staging with int16 sub-blocks (nullptr: not offered)
    BlockLaunch launch_dt;    // double-tiling schedule, int32 storage (nullptr: not offered)
};

#define P16(D, TX, TY, NT) launch_block16<D, TX, TY, NT>
#define V8(D, TX, TY, NT)                                                                     \
    {D, TX, TY, NT, 1, launch_block<D, TX, TY, NT, int8_t, int16_t, 0>, P16(D, TX, TY, NT),    \
     dt_launcher<D, TX, TY, NT, int8_t, int16_t>()}
#define V8N(D, TX, TY, NT)                                                                     \
    {D, TX, TY, NT, 1, launch_block<D, TX, TY, NT, int8_t, int16_t, 0>, nullptr,                \
     dt_launcher<D, TX, TY, NT, int8_t, int16_t>()}
#define V16(D, TX, TY, NT) \
    {D, TX, TY, NT, 2, launch_block<D, TX, TY, NT, int16_t, void, 0>, nullptr, dt_launcher<D, TX, TY, NT, int16_t, void>()}
#define V16P(D, TX, TY, NT) \
    {D, TX, TY, NT, 2, launch_block<D, TX, TY, NT, int16_t, void, 0>, P16(D, TX, TY, NT), \
     dt_launcher<D, TX, TY, NT, int16_t, void>()}
#define V32(D, TX, TY, NT) \
    {D, TX, TY, NT, 4, launch_block<D, TX, TY, NT, int32_t, void, 0>, nullptr, dt_launcher<D, TX, TY, NT, int32_t, void>()}
// In order of preference; without a tuned choice the first one that fits
// every surface is used.
// (V8N: the same int8 kernel without a 16-bit storage instance, where a
// V16P entry of the same shape already provides it.)  The autotuner times
// every entry that fits.
const Variant kVariants[] = {
    V16P(2, 32, 32, 256), V32(2, 16, 16, 128), V32(2, 2, 2, 64), V8(2, 64, 32, 256),
    V16P(4, 16, 16, 128), V32(4, 16, 16, 128), V32(4, 2, 2, 64), V8(4, 32, 16, 256),
    V8(8, 32, 8, 256), V16P(8, 16, 8, 128), V16(8, 8, 8, 64), V32(8, 16, 8, 128),
    V32(8, 8, 8, 64), V32(8, 2, 2, 64), V8(8, 16, 16, 256), V8N(8, 16, 8, 128),
    V16P(16, 4, 4, 64), V32(16, 4, 4, 64), V32(16, 2, 2, 64), V8(16, 4, 4, 64), V8(16, 8, 8, 256),
    V8(32, 2, 2, 64), V32(32, 2, 2, 64),
};
#undef P16
#undef V8
#undef V8N
#undef V16
#undef V16P
#undef V32

bool variant_fits(const Variant &v, int L, int N, bool packed, bool dt = false)
{
    if (dt && (packed || !v.launch_dt)) return false;
    const int T = L / v.D;
    const int rw = v.TX * v.D + 2 * (v.D + 1), rh = v.TY * v.D + 2 * (v.D + 1);
    const int rwl = packed ? (rw + 14) & ~7 : (rw + 6) & ~3;
    if (T % v.TX != 0 || T % v.TY != 0 || rh > L) return false;
    // a region wider than the lattice only for a block as wide as the
    // lattice (its ring columns are copies of its own far edge, recomputed
    // from the same inputs)
    if (rwl > L && !(v.TX * v.D == L && rwl <= 2 * L)) return false;
    // int16 staging: every staged value within 32767 of the block reference
    // (the int16 sub-blocks of a block that int8 staging does not fit are
    // smaller than the block, so the block's bound covers them)
    const bool i16_ok = (long long)N * (rw + rh + 4) + v.D * v.D <= 32767;
    // 16-bit storage: uint8 staging (N D <= 96) and the int16 sub-blocks
    if (packed) return v.launch16 && L % 8 == 0 && (long long)N * v.D <= 96 && i16_ok;
    if (v.elem == 2 && !i16_ok) return false;
    // int8 staging: the sweep's growth N D must leave room in the byte
    if (v.elem == 1 && ((long long)N * v.D > 96 || !i16_ok)) return false;
    return true;
}

// First fitting variant for D that fits every (L, N) (optionally forced by
// the RSOS_VARIANT environment variable "TXxTYxNTxELEM", e.g. "16x8x128x2";
// ELEM is 16 for the 16-bit storage kernels).
const Variant *pick_variant(int D, const std::vector<std::pair<int, int>> &LN, bool packed = false,
                            bool dt = false)
{
    const char *force = getenv("RSOS_VARIANT");
    for (const Variant &v : kVariants) {
        if (v.D != D) continue;
        if (force) {
            char want[48];
            snprintf(want, sizeof want, "%dx%dx%dx%d", v.TX, v.TY, v.NT, packed ? 16 : v.elem);
            if (strcmp(force, want) != 0) continue;
        }
        bool ok = true;
        for (auto &ln : LN) ok = ok && variant_fits(v, ln.first, ln.second, packed, dt);
        if (ok) return &v;
    }
    return nullptr;
}

bool uses_lds(int L);

// 16-bit storage is exact while every height of a sweep stays within 2^15
// of floor(mean): N L <= 32766 (the torus spread is at most N L, the mean
// moves by at most one per sweep).
rsos_status check_packed(const rsos_params *p)
{
    if (uses_lds(p->L))
        return fail(RSOS_E_INVAL, "16-bit storage: L=%d is small enough for the LDS path, which keeps int32", p->L);
    if ((long long)p->N * p->L > 32766)
        return fail(RSOS_E_INVAL, "16-bit storage needs N*L <= 32766 (N=%d, L=%d)", p->N, p->L);
    if (!pick_variant(p->D, {{p->L, p->N}}, true))
        return fail(RSOS_E_INVAL, "16-bit storage: no tile-block shape fits L=%d, N=%d, D=%d", p->L, p->N, p->D);
    return RSOS_OK;
}

typedef void (*LdsLaunch)(dim3, size_t, hipStream_t, SurfDev *, const int *);
template <int D, int SCHED>
void launch_lds(dim3 grid, size_t shm, hipStream_t st, SurfDev *d, const int *w)
{
    hipLaunchKernelGGL((rsosk::lds_run<D, 256, SCHED>), grid, dim3(256), shm, st, d, w);
}
LdsLaunch lds_launcher(int D, int sched = 0)
{
    if (sched == 1) {
        switch (D) {
        case 8: return launch_lds<8, 1>;
        case 16: return launch_lds<16, 1>;
        }
        return nullptr;
    }
    switch (D) {
    case 2: return launch_lds<2, 0>;
    case 4: return launch_lds<4, 0>;
    case 8: return launch_lds<8, 0>;
    case 16: return launch_lds<16, 0>;
    case 32: return launch_lds<32, 0>;
    }
    return nullptr;
}

bool valid_D(int D) { return D == 2 || D == 4 || D == 8 || D == 16 || D == 32; }

rsos_status check_params(const rsos_params *p)
{
    if (!p) return fail(RSOS_E_INVAL, "params is NULL");
    if (!valid_D(p->D)) return fail(RSOS_E_INVAL, "D=%d: must be 2, 4, 8, 16 or 32", p->D);
    if (p->L < 2 * p->D || p->L > 65536 || p->L % (2 * p->D) != 0)
        return fail(RSOS_E_INVAL, "L=%d: must be a multiple of 2D=%d in [2D, 65536]", p->L, 2 * p->D);
    if (p->N < 1) return fail(RSOS_E_INVAL, "N=%d: must be >= 1", p->N);
    if (p->flags & ~(RSOS_FLAG_PACKED16 | RSOS_FLAG_DT4 | RSOS_FLAG_TUNE))
        return fail(RSOS_E_INVAL, "unknown flags 0x%x", (unsigned)p->flags);
    if (p->flags & RSOS_FLAG_DT4) {
        if (p->flags & RSOS_FLAG_PACKED16)
            return fail(RSOS_E_INVAL, "the double-tiling schedule runs on int32 storage");
        if (p->D != 8 && p->D != 16) return fail(RSOS_E_INVAL, "double tiling: D must be 8 or 16");
        if (!uses_lds(p->L) && !pick_variant(p->D, {{p->L, p->N}}, false, true))
            return fail(RSOS_E_INVAL, "double tiling: no tile-block shape fits L=%d, N=%d", p->L, p->N);
    }
    if (p->flags & RSOS_FLAG_PACKED16) return check_packed(p);
    return RSOS_OK;
}

bool uses_lds(int L) { return (long long)L * L * 4 <= kLdsMaxBytes; }

// Pinned staging for small host->device descriptor updates; the event makes
// sure the previous copy is done before the buffer is rewritten.
struct Staging {
    void *host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;

    rsos_status ensure(size_t n)
    {
        if (!done) HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        if (pending) {
            HIP_TRY(hipEventSynchronize(done));
            pending = false;
        }
        if (n > bytes) {
            if (host) HIP_TRY(hipHostFree(host));
            host = nullptr;
            HIP_TRY(hipHostMalloc(&host, n, hipHostMallocDefault));
            bytes = n;
        }
        return RSOS_OK;
    }
    rsos_status copy_to(void *dev, size_t n, hipStream_t st)
    {
        HIP_TRY(hipMemcpyAsync(dev, host, n, hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(done, st));
        pending = true;
        return RSOS_OK;
    }
    void release()
    {
        if (pending && done) (void)hipEventSynchronize(done);
        if (host) (void)hipHostFree(host);
        if (done) (void)hipEventDestroy(done);
        host = nullptr;
        done = nullptr;
    }
};

}  // namespace

// Block-path surfaces swept by one kernel instance: rows [first, first +
// count) of the descriptor table, blocks numbered from 0 within the shape.
struct Shape {
    const Variant *variant = nullptr;
    int xmode = 1;
    int first = 0, count = 0;
    int total_blocks = 0;
    int *d_owner = nullptr;  // block -> row within the shape (count > 1)
};

// A launch choice for one surface: kernel variant, block order and sweeps
// per captured graph (none of them changes results).
struct Choice {
    const Variant *v = nullptr;
    int xmode = 1;
    int graph_k = 0;
};

// ---------------------------------------------------------------------------
// A group of surfaces sharing one D: the common core of the single-surface,
// batch and engine front ends.
// ---------------------------------------------------------------------------
struct SurfaceGroup {
    int D = 8;
    bool packed = false;               // heights kept as 16-bit residues
    int sched = 0;                     // 0: tile checkerboard, 1: double tiling
    hipStream_t stream = nullptr;
    bool failed = false;
    std::vector<SurfDev> host;         // host mirror (t, t_end kept current)
    std::vector<long long> dev_t_end;  // t_end values last uploaded
    std::vector<long long> max_h0, t0; // per surface
    SurfDev *d_desc = nullptr;
    long long *d_acc = nullptr;        // kAccWords per block-path surface
    std::vector<int32_t *> readout;    // 16-bit storage: int32[L^2] device scratch per surface
    long long *d_ps = nullptr;         // power sums: per-workgroup partials, then the result
    int xmode = 1;                     // workgroup -> block order (rsosk::block_map) without a choice
    std::vector<Shape> shapes;         // block-path surfaces by kernel instance
    std::vector<Choice> want;          // per surface: a tuned launch choice (or none); read by setup()
    std::vector<int> rows;             // device-table row -> surface index
    std::vector<int> lds_idx, blk_idx; // surfaces on each path
    int *d_lds_idx = nullptr;
    int graph_k = kGraphSweeps;        // sweeps per captured graph
    size_t lds_bytes = 0;
    Staging staging;
    hipGraphExec_t graph = nullptr;
    int graph_sweeps = 0;
    bool timing = false;                             // bracket block launches with events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
    std::vector<void *> owned;         // library-owned device allocations

    rsos_status dev_alloc(void **p, size_t n)
    {
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess) return fail(RSOS_E_NOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
        owned.push_back(*p);
        return RSOS_OK;
    }

    // Builds the descriptor table (host side must be filled: buf, log, L, N,
    // key, t, t_end).  Groups the block-path surfaces by kernel instance:
    // each surface's tuned choice where want[] holds one for every
    // block-path surface, else one first-fit variant for all of them.
    rsos_status setup()
    {
        const int n = (int)host.size();
        std::vector<std::pair<int, int>> LN;
        for (int i = 0; i < n; ++i) {
            if (uses_lds(host[i].L)) lds_idx.push_back(i);
            else { blk_idx.push_back(i); LN.push_back({host[i].L, host[i].N}); }
            for (int k = 0; k < 2; ++k)
                if (((uintptr_t)host[i].buf[k] & 15) != 0)
                    return fail(RSOS_E_INVAL, "height buffers must be 16-byte aligned");
        }
        if (packed && !lds_idx.empty()) return fail(RSOS_E_INVAL, "16-bit storage needs the tile-block path");
        if (const char *xm = getenv("RSOS_XMODE")) xmode = atoi(xm) == 0 ? 0 : atoi(xm) == 2 ? 2 : 1;
        bool tuned = !blk_idx.empty() && want.size() == host.size();
        for (int i : blk_idx) tuned = tuned && want[i].v != nullptr;
        std::vector<std::vector<int>> members;
        if (tuned) {
            for (int i : blk_idx) {
                size_t g = 0;
                while (g < shapes.size() && !(shapes[g].variant == want[i].v && shapes[g].xmode == want[i].xmode)) ++g;
                if (g == shapes.size()) {
                    shapes.push_back(Shape());
                    shapes.back().variant = want[i].v;
                    shapes.back().xmode = want[i].xmode;
                    members.emplace_back();
                }
                members[g].push_back(i);
            }
            graph_k = 0;
            for (int i : blk_idx) graph_k = std::max(graph_k, want[i].graph_k);
            if (graph_k < 1) graph_k = kGraphSweeps;
        } else if (!blk_idx.empty()) {
            const Variant *v = pick_variant(D, LN, packed, sched == 1);
            if (!v) return fail(RSOS_E_INVAL, "no tile-block shape fits these lattice sizes");
            shapes.push_back(Shape());
            shapes.back().variant = v;
            shapes.back().xmode = xmode;
            members.push_back(blk_idx);
        }
        // rows: each shape's surfaces in turn (block numbers restart at 0 in
        // every shape), then the LDS-path surfaces
        rows.clear();
        for (size_t g = 0; g < shapes.size(); ++g) {
            Shape &sh = shapes[g];
            sh.first = (int)rows.size();
            sh.count = (int)members[g].size();
            long long blocks = 0;
            for (int i : members[g]) {
                SurfDev &sd = host[i];
                const int T = sd.L / D;
                sd.nbx = T / sh.variant->TX;
                sd.nblocks = sd.nbx * (T / sh.variant->TY);
                sd.block_start = (int)blocks;
                blocks += sd.nblocks;
                if (blocks > (1ll << 30)) return fail(RSOS_E_INVAL, "too many tile blocks");
                rows.push_back(i);
            }
            sh.total_blocks = (int)blocks;
            if (sh.xmode == 2 && !(sh.count == 1 && host[members[g][0]].nbx % 8 == 0)) sh.xmode = 1;
        }
        const int nblk_rows = (int)rows.size();
        for (int i : lds_idx) {
            host[i].nbx = 0;
            host[i].nblocks = 0;
            host[i].block_start = 1 << 30;  // never matched by a block workgroup
            rows.push_back(i);
        }
        rsos_status st;
        if ((st = dev_alloc((void **)&d_desc, sizeof(SurfDev) * n)) != RSOS_OK) return st;
        if (nblk_rows) {
            const size_t bytes = sizeof(long long) * rsosk::kAccWords * nblk_rows;
            if ((st = dev_alloc((void **)&d_acc, bytes)) != RSOS_OK) return st;
            HIP_TRY(hipMemset(d_acc, 0, bytes));
            for (int r = 0; r < nblk_rows; ++r) host[rows[r]].acc = d_acc + rsosk::kAccWords * r;
        }
        for (Shape &sh : shapes) {
            if (sh.count < 2) continue;
            // owner of every block of the shape: its row within the shape
            std::vector<int> own((size_t)sh.total_blocks);
            for (int k = 0; k < sh.count; ++k) {
                const SurfDev &sd = host[rows[sh.first + k]];
                for (int b = 0; b < sd.nblocks; ++b) own[(size_t)sd.block_start + b] = k;
            }
            if ((st = dev_alloc((void **)&sh.d_owner, sizeof(int) * own.size())) != RSOS_OK) return st;
            HIP_TRY(hipMemcpy(sh.d_owner, own.data(), sizeof(int) * own.size(), hipMemcpyHostToDevice));
        }
        if (!lds_idx.empty()) {
            if ((st = dev_alloc((void **)&d_lds_idx, sizeof(int) * lds_idx.size())) != RSOS_OK) return st;
            std::vector<int> pos(lds_idx.size());
            for (size_t k = 0; k < pos.size(); ++k) pos[k] = nblk_rows + (int)k;
            HIP_TRY(hipMemcpy(d_lds_idx, pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice));
            int maxL = 0;
            for (int i : lds_idx) maxL = std::max(maxL, host[i].L);
            lds_bytes = (size_t)maxL * maxL * 4;
        }
        return upload_all();
    }

    rsos_status upload_all()
    {
        const int n = (int)host.size();
        rsos_status st = staging.ensure(sizeof(SurfDev) * n);
        if (st != RSOS_OK) return st;
        SurfDev *h = (SurfDev *)staging.host;
        for (int k = 0; k < n; ++k) h[k] = host[rows[k]];
        return staging.copy_to(d_desc, sizeof(SurfDev) * n, stream);
    }

    // Sets every surface's end time for the next launch_sweeps(n).  A
    // block-path surface that advances by all n sweeps needs no bound (the
    // launch count is the bound) and keeps an unbounded t_end on the device,
    // so a run of such calls rewrites nothing; the others, and LDS-path
    // surfaces (which run to their t_end in one launch), get their exact
    // t_end.  A rewrite uploads the whole (small) table, t included: the
    // host mirror of t is exact, since sweep counts are deterministic.
    rsos_status set_t_end(const std::vector<long long> &t_end, long long n)
    {
        bool changed = dev_t_end.size() != host.size();
        for (size_t i = 0; i < host.size(); ++i) {
            const bool blk = !uses_lds(host[i].L);
            host[i].t_end = (blk && t_end[i] - host[i].t == n) ? kNoEnd : t_end[i];
            changed = changed || host[i].t_end != dev_t_end[i];
        }
        if (!changed) return RSOS_OK;
        dev_t_end.resize(host.size());
        for (size_t i = 0; i < host.size(); ++i) dev_t_end[i] = host[i].t_end;
        return upload_all();
    }

    rsos_status launch_sweeps(long long n)
    {
        if (n <= 0) return RSOS_OK;
        if (!lds_idx.empty()) {
            lds_launcher(D, sched)(dim3((unsigned)lds_idx.size()), lds_bytes, stream, d_desc, d_lds_idx);
            HIP_TRY(hipGetLastError());
        }
        if (blk_idx.empty()) return RSOS_OK;
        long long left = n;
        if (stream != nullptr && n >= 2 * graph_k && !timing) {
            if (!graph) {
                rsos_status st = capture_graph(graph_k);
                if (st != RSOS_OK) return st;
            }
            while (left >= graph_sweeps) {
                HIP_TRY(hipGraphLaunch(graph, stream));
                left -= graph_sweeps;
            }
        }
        for (; left > 0; --left) {
            rsos_status st = enqueue_one();
            if (st != RSOS_OK) return st;
        }
        return RSOS_OK;
    }

    // the tile-block sweep proper: one workgroup per block, the whole sweep
    // in one launch per kernel instance
    void launch_block_sweep(hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
    {
        for (size_t i = 0; i < shapes.size(); ++i) {
            const Shape &sh = shapes[i];
            const Variant *v = sh.variant;
            BlockLaunch k = packed ? v->launch16 : sched == 1 ? v->launch_dt : v->launch;
            const int nbx = sh.count == 1 ? host[rows[sh.first]].nbx : 0;
            k(dim3(sh.total_blocks), stream, d_desc + sh.first, sh.count, sh.d_owner, sh.xmode, nbx,
              i == 0 ? e0 : nullptr, i + 1 == shapes.size() ? e1 : nullptr);
        }
    }

    rsos_status enqueue_one()
    {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            // recorded by the runtime at the start of the sweep's first
            // kernel and the end of its last
            HIP_TRY(hipEventCreate(&e0));
            HIP_TRY(hipEventCreate(&e1));
            timed.push_back({e0, e1});
        }
        launch_block_sweep(e0, e1);
        HIP_TRY(hipGetLastError());
        return RSOS_OK;
    }

    // Captures the graph of graph_k sweeps when the group is created, so
    // that no rsos_sweep call pays for a capture (surfaces on a stream).
    rsos_status prepare_graph()
    {
        if (stream == nullptr || blk_idx.empty() || graph) return RSOS_OK;
        return capture_graph(graph_k);
    }

    rsos_status capture_graph(int k)
    {
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < k; ++i) launch_block_sweep();
        HIP_TRY(hipStreamEndCapture(stream, &g));
        HIP_TRY(hipGraphInstantiate(&graph, g, nullptr, nullptr, 0));
        HIP_TRY(hipGraphDestroy(g));
        graph_sweeps = k;
        return RSOS_OK;
    }

    // Reads log records of surface i for times [t_from, t_from + n).
    rsos_status read_log(int i, long long t_from, long long n, rsos_width_t *out)
    {
        const SurfDev &s = host[i];
        if (n < 0 || t_from < t0[i] || t_from + n > s.t + 1)
            return fail(RSOS_E_INVAL, "times [%lld, %lld) outside [t0=%lld, t=%lld]", t_from,
                        t_from + n, t0[i], s.t);
        if (t_from + s.log_cap <= s.t && n > 0)
            return fail(RSOS_E_INVAL, "records before t=%lld are no longer kept", s.t - s.log_cap + 1);
        HIP_TRY(hipStreamSynchronize(stream));
        std::vector<long long> buf((size_t)(3 * std::max<long long>(n, 1)));
        for (long long k = 0; k < n;) {
            const long long slot = (t_from + k) % s.log_cap;
            const long long run = std::min(n - k, s.log_cap - slot);
            HIP_TRY(hipMemcpy(buf.data() + 3 * k, s.log + 3 * slot, sizeof(long long) * 3 * run,
                              hipMemcpyDeviceToHost));
            k += run;
        }
        for (long long k = 0; k < n; ++k) {
            out[k].t = t_from + k;
            out[k].s1 = buf[3 * k];
            out[k].s2 = buf[3 * k + 1];
            out[k].accepted = buf[3 * k + 2];
            out[k].w2 = w2_of(s.L, out[k].s1, out[k].s2);
        }
        return RSOS_OK;
    }

    rsos_status copy_heights(int i, int32_t *dst, int dst_is_device)
    {
        const SurfDev &s = host[i];
        const size_t n = (size_t)s.L * s.L;
        if (packed) {
            // residues -> int32 on the device (needs floor(S1 / L^2) of time t)
            int32_t *out = dst_is_device ? dst : readout[i];
            hipLaunchKernelGGL(rsosk::unpack16, dim3(grid_for(n)), dim3(256), 0, stream,
                               (const uint16_t *)s.buf[s.t & 1], out, (long long)n,
                               (const long long *)(s.acc + rsosk::kMeanWord));
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(stream));
            if (!dst_is_device) HIP_TRY(hipMemcpy(dst, out, n * 4, hipMemcpyDeviceToHost));
            return RSOS_OK;
        }
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipMemcpy(dst, s.buf[s.t & 1], n * 4,
                          dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
        return RSOS_OK;
    }

    // Initial state of surface i into its buffer of parity t: int32 heights
    // from host memory (nullptr: flat), as residues in 16-bit storage, and
    // floor(S1 / L^2) into the accumulator area.
    rsos_status load_initial(int i, const int32_t *h0_host, long long s1)
    {
        const SurfDev &s = host[i];
        const size_t n = (size_t)s.L * s.L;
        int32_t *cur = s.buf[s.t & 1];
        if (!packed) {
            HIP_TRY(h0_host ? hipMemcpyAsync(cur, h0_host, n * 4, hipMemcpyHostToDevice, stream)
                            : hipMemsetAsync(cur, 0, n * 4, stream));
        } else if (h0_host) {
            HIP_TRY(hipMemcpyAsync(readout[i], h0_host, n * 4, hipMemcpyHostToDevice, stream));
            hipLaunchKernelGGL(rsosk::pack16, dim3(grid_for(n)), dim3(256), 0, stream,
                               (const int32_t *)readout[i], (uint16_t *)cur, (long long)n);
            HIP_TRY(hipGetLastError());
        } else {
            HIP_TRY(hipMemsetAsync(cur, 0, n * 2, stream));
        }
        if (s.acc) {
            const long long m0 = s1 / ((long long)s.L * s.L);
            HIP_TRY(hipMemcpyAsync(s.acc + rsosk::kMeanWord, &m0, sizeof m0, hipMemcpyHostToDevice, stream));
        }
        HIP_TRY(hipStreamSynchronize(stream));
        return RSOS_OK;
    }

    static unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + 255) / 256, 8192); }

    // Exact power sums of surface i's current heights about floor(S1/L^2)
    // (rsosk::power_sums_partial / power_sums_final), then the central
    // moments from them.
    rsos_status moments(int i, rsos_moments_t *out)
    {
        const SurfDev &s = host[i];
        const long long n = (long long)s.L * s.L;
        // at most 2^16 sites per thread: grid >= n / 2^24
        const int grid = (int)std::min<long long>(kPsGrid, std::max<long long>(1, n / (256 * 64)));
        rsos_status st;
        if (!d_ps && (st = dev_alloc((void **)&d_ps, sizeof(long long) * (8 * (size_t)kPsGrid + 8))) != RSOS_OK)
            return st;
        const long long *rec = s.log + 3 * (s.t % s.log_cap);
        if (packed)
            hipLaunchKernelGGL(rsosk::power_sums_partial<uint16_t>, dim3(grid), dim3(256), 0, stream,
                               (const uint16_t *)s.buf[s.t & 1], n, rec, d_ps);
        else
            hipLaunchKernelGGL(rsosk::power_sums_partial<int32_t>, dim3(grid), dim3(256), 0, stream,
                               (const int32_t *)s.buf[s.t & 1], n, rec, d_ps);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(rsosk::power_sums_final, dim3(1), dim3(256), 0, stream, d_ps, grid,
                           d_ps + 8 * (size_t)kPsGrid);
        HIP_TRY(hipGetLastError());
        rsos_width_t w;
        if ((st = read_log(i, s.t, 1, &w)) != RSOS_OK) return st;  // synchronises
        unsigned long long r[8];
        HIP_TRY(hipMemcpy(r, d_ps + 8 * (size_t)kPsGrid, sizeof r, hipMemcpyDeviceToHost));
        __int128 c[4];
        for (int k = 0; k < 4; ++k) c[k] = (__int128)(((unsigned __int128)r[2 * k + 1] << 64) | r[2 * k]);
        out->t = s.t;
        out->ref = w.s1 / n;
        out->c1 = (int64_t)c[0];
        out->c2 = (int64_t)c[1];
        out->c3[0] = r[4];
        out->c3[1] = r[5];
        out->c4[0] = r[6];
        out->c4[1] = r[7];
        // central moments: with d = c1/n in [0, 1), expand (h - ref - d)^k
        const long double N_ = (long double)n, d = (long double)c[0] / N_;
        const long double m2 = (long double)c[1] / N_, m3 = (long double)c[2] / N_, m4 = (long double)c[3] / N_;
        out->phi2 = (double)(m2 - d * d);
        out->phi3 = (double)(m3 - 3 * d * m2 + 2 * d * d * d);
        out->phi4 = (double)(m4 - 4 * d * m3 + 6 * d * d * m2 - 3 * d * d * d * d);
        return RSOS_OK;
    }

    // Writes the initial log record (time t0) of surface i.
    rsos_status init_record(int i, long long s1, long long s2)
    {
        long long rec[3] = {s1, s2, 0};
        const SurfDev &s = host[i];
        HIP_TRY(hipMemcpy(s.log + 3 * (s.t % s.log_cap), rec, sizeof rec, hipMemcpyHostToDevice));
        return RSOS_OK;
    }

    rsos_status read_timing(int64_t *launches, double *mean_ms, double *total_ms)
    {
        HIP_TRY(hipStreamSynchronize(stream));
        double tot = 0.0;
        for (auto &pr : timed) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
            tot += ms;
        }
        if (launches) *launches = (int64_t)timed.size();
        if (total_ms) *total_ms = tot;
        if (mean_ms) *mean_ms = timed.empty() ? 0.0 : tot / (double)timed.size();
        clear_timing();
        return RSOS_OK;
    }

    void clear_timing()
    {
        for (auto &pr : timed) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        timed.clear();
    }

    void destroy()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        else (void)hipDeviceSynchronize();
        clear_timing();
        if (graph) (void)hipGraphExecDestroy(graph);
        staging.release();
        for (void *p : owned) (void)hipFree(p);
        owned.clear();
    }
};

struct rsos_surface {
    rsos_params p;
    SurfaceGroup g;
};

struct rsos_batch {
    std::vector<rsos_params> p;
    SurfaceGroup g;
};

// ---------------------------------------------------------------------------
// autotuner of the launch knobs -- see rsos_tune.inc
// ---------------------------------------------------------------------------
#include "rsos_tune.inc"

#define CHECK_HANDLE(h, grp)                                                           \
    do {                                                                               \
        if (!(h)) return fail(RSOS_E_INVAL, "NULL handle");                           \
        if ((grp).failed) return fail(RSOS_E_STATE, "handle failed after a device error"); \
    } while (0)

static rsos_status mark(SurfaceGroup &g, rsos_status st)
{
    if (st == RSOS_E_DEVICE) g.failed = true;
    return st;
}

extern "C" {

const char *rsos_version(void) { return "rsos-gfx950 1.0"; }

const char *rsos_strerror(rsos_status st)
{
    switch (st) {
    case RSOS_OK: return "ok";
    case RSOS_E_INVAL: return "invalid argument";
    case RSOS_E_RSOS: return "initial heights violate the RSOS restriction";
    case RSOS_E_OVERFLOW: return "heights or sums could overflow";
    case RSOS_E_DEVICE: return "HIP runtime error";
    case RSOS_E_NOMEM: return "out of memory";
    case RSOS_E_STATE: return "handle failed or call out of sequence";
    case RSOS_E_BUSY: return "no room for the job now";
    }
    return "unknown status";
}

const char *rsos_last_error(void) { return g_last_error.c_str(); }

rsos_status rsos_debug_fail(int32_t after)
{
    if (after < 0) return fail(RSOS_E_INVAL, "after < 0");
    rsosh::g_fail_countdown = after;
    return RSOS_OK;
}

void rsos_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const rsosk::u32x4 r = rsosk::philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

double rsos_w2(int32_t L, int64_t s1, int64_t s2) { return w2_of(L, s1, s2); }

rsos_status rsos_init(rsos_surface **out, const rsos_params *p, int32_t *d_h, int32_t *d_work,
                      const int32_t *h0_host, int64_t t0, int64_t log_cap, void *stream)
{
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    *out = nullptr;
    rsos_status st = check_params(p);
    if (st != RSOS_OK) return st;
    if (!d_h) return fail(RSOS_E_INVAL, "d_h is NULL");
    if (t0 < 0 || t0 >= (1ll << 32)) return fail(RSOS_E_INVAL, "t0 outside [0, 2^32)");
    if (log_cap < 0) return fail(RSOS_E_INVAL, "log_cap < 0");
    if (log_cap == 0) log_cap = 65536;
    long long max_h = 0, s1 = 0, s2 = 0;
    if (h0_host && (st = validate_h0(h0_host, p->L, p->N, &max_h, &s1, &s2)) != RSOS_OK) return st;
    if ((st = check_overflow(*p, max_h, 0)) != RSOS_OK) return st;

    rsos_surface *s = new (std::nothrow) rsos_surface();
    if (!s) return fail(RSOS_E_NOMEM, "host allocation failed");
    s->p = *p;
    SurfaceGroup &g = s->g;
    g.D = p->D;
    g.packed = (p->flags & RSOS_FLAG_PACKED16) != 0;
    g.sched = (p->flags & RSOS_FLAG_DT4) ? 1 : 0;
    g.stream = (hipStream_t)stream;
    const size_t n = (size_t)p->L * p->L;
    SurfDev d = {};
    int32_t *work = d_work;
    if (!work && (st = g.dev_alloc((void **)&work, n * 4)) != RSOS_OK) { g.destroy(); delete s; return st; }
    if (g.packed) {
        // both residue buffers in d_h; d_work receives int32 heights on readout
        d.buf[0] = d_h;
        d.buf[1] = (int32_t *)((uint16_t *)d_h + n);
        g.readout.push_back(work);
    } else {
        d.buf[0] = d_h;
        d.buf[1] = work;
    }
    if ((st = g.dev_alloc((void **)&d.log, sizeof(long long) * 3 * log_cap)) != RSOS_OK) { g.destroy(); delete s; return st; }
    d.log_cap = log_cap;
    d.t = t0;
    d.t_end = t0;
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.L = p->L;
    d.N = p->N;
    d.T = p->L / p->D;
    g.host.push_back(d);
    g.max_h0.push_back(max_h);
    g.t0.push_back(t0);
    if (tuning_wanted(p) && !uses_lds(p->L)) {
        Choice c;
        if ((st = tuned_choice(p, 0, &c)) != RSOS_OK) { g.destroy(); delete s; return st; }
        g.want.assign(1, c);
    }
    if ((st = mark(g, g.setup())) != RSOS_OK) { g.destroy(); delete s; return st; }
    // initial state into the buffer of parity t0
    if ((st = g.load_initial(0, h0_host, s1)) != RSOS_OK) { g.destroy(); delete s; return st; }
    if ((st = g.init_record(0, s1, s2)) != RSOS_OK) { g.destroy(); delete s; return st; }
    if ((st = mark(g, g.prepare_graph())) != RSOS_OK) { g.destroy(); delete s; return st; }
    *out = s;
    return RSOS_OK;
}

rsos_status rsos_sweep(rsos_surface *s, int64_t n_mcs)
{
    CHECK_HANDLE(s, s->g);
    if (n_mcs < 0) return fail(RSOS_E_INVAL, "n_mcs < 0");
    if (n_mcs == 0) return RSOS_OK;
    SurfaceGroup &g = s->g;
    const long long t = g.host[0].t;
    if (t + n_mcs > (1ll << 32)) return fail(RSOS_E_INVAL, "sweep index would exceed 2^32");
    rsos_status st = check_overflow(s->p, g.max_h0[0], t + n_mcs - g.t0[0]);
    if (st != RSOS_OK) return st;
    if ((st = mark(g, g.set_t_end({t + n_mcs}, n_mcs))) != RSOS_OK) return st;
    if ((st = mark(g, g.launch_sweeps(n_mcs))) != RSOS_OK) return st;
    g.host[0].t = t + n_mcs;
    return RSOS_OK;
}

rsos_status rsos_width(rsos_surface *s, rsos_width_t *out)
{
    CHECK_HANDLE(s, s->g);
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    return mark(s->g, s->g.read_log(0, s->g.host[0].t, 1, out));
}

rsos_status rsos_log(rsos_surface *s, int64_t t_from, int64_t n, rsos_width_t *out)
{
    CHECK_HANDLE(s, s->g);
    if (!out && n > 0) return fail(RSOS_E_INVAL, "out is NULL");
    return mark(s->g, s->g.read_log(0, t_from, n, out));
}

rsos_status rsos_heights(rsos_surface *s, int32_t *dst, int dst_is_device)
{
    CHECK_HANDLE(s, s->g);
    if (!dst) return fail(RSOS_E_INVAL, "dst is NULL");
    return mark(s->g, s->g.copy_heights(0, dst, dst_is_device));
}

rsos_status rsos_moments(rsos_surface *s, rsos_moments_t *out)
{
    CHECK_HANDLE(s, s->g);
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    return mark(s->g, s->g.moments(0, out));
}

rsos_status rsos_time(rsos_surface *s, int64_t *t, int32_t **d_current)
{
    CHECK_HANDLE(s, s->g);
    const SurfDev &d = s->g.host[0];
    if (t) *t = d.t;
    if (d_current) *d_current = s->g.packed ? nullptr : d.buf[d.t & 1];
    return RSOS_OK;
}

rsos_status rsos_timing(rsos_surface *s, int enable)
{
    CHECK_HANDLE(s, s->g);
    s->g.timing = enable != 0;
    return RSOS_OK;
}

rsos_status rsos_timing_read(rsos_surface *s, int64_t *launches, double *mean_ms, double *total_ms)
{
    CHECK_HANDLE(s, s->g);
    return mark(s->g, s->g.read_timing(launches, mean_ms, total_ms));
}

rsos_status rsos_kernel_name(rsos_surface *s, char *buf, int32_t len)
{
    CHECK_HANDLE(s, s->g);
    if (!buf || len < 1) return fail(RSOS_E_INVAL, "bad buffer");
    const SurfaceGroup &g = s->g;
    const Variant *v = g.shapes.empty() ? nullptr : g.shapes[0].variant;
    if (v && g.packed)
        snprintf(buf, (size_t)len, "block_sweep16<%d,%d,%d,%d,0>", v->D, v->TX, v->TY, v->NT);
    else if (v)
        snprintf(buf, (size_t)len, "block_sweep<%d,%d,%d,%d,%s,%d>", v->D, v->TX, v->TY, v->NT,
                 v->elem == 1 ? "int8,int16" : v->elem == 2 ? "int16,void" : "int32,void", g.sched);
    else
        snprintf(buf, (size_t)len, "lds_run<%d,256,%d>", g.D, g.sched);
    return RSOS_OK;
}

rsos_status rsos_free(rsos_surface *s)
{
    if (!s) return RSOS_OK;
    s->g.destroy();
    delete s;
    return RSOS_OK;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
rsos_status rsos_batch_init(rsos_batch **out, int32_t n, const rsos_params *p, int32_t *d_pool,
                            int32_t *d_work_pool, const int64_t *offsets, int64_t log_cap,
                            void *stream)
{
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !p || !d_pool || !offsets) return fail(RSOS_E_INVAL, "bad batch arguments");
    if (log_cap < 0) return fail(RSOS_E_INVAL, "log_cap < 0");
    if (log_cap == 0) log_cap = 65536;
    rsos_status st;
    for (int i = 0; i < n; ++i) {
        if ((st = check_params(&p[i])) != RSOS_OK) return fail(st, "surface %d: %s", i, g_last_error.c_str());
        if (p[i].D != p[0].D) return fail(RSOS_E_INVAL, "all surfaces of a batch share one D");
        if (p[i].flags != p[0].flags) return fail(RSOS_E_INVAL, "all surfaces of a batch share one storage mode");
        if (offsets[i] < 0) return fail(RSOS_E_INVAL, "negative offset");
    }
    // surfaces must not overlap in the pool
    {
        std::vector<std::pair<long long, long long>> iv;
        for (int i = 0; i < n; ++i) iv.push_back({offsets[i], offsets[i] + (long long)p[i].L * p[i].L});
        std::sort(iv.begin(), iv.end());
        for (int i = 1; i < n; ++i)
            if (iv[i].first < iv[i - 1].second) return fail(RSOS_E_INVAL, "surfaces overlap in the pool");
    }
    rsos_batch *b = new (std::nothrow) rsos_batch();
    if (!b) return fail(RSOS_E_NOMEM, "host allocation failed");
    b->p.assign(p, p + n);
    SurfaceGroup &g = b->g;
    g.D = p[0].D;
    g.packed = (p[0].flags & RSOS_FLAG_PACKED16) != 0;
    g.sched = (p[0].flags & RSOS_FLAG_DT4) ? 1 : 0;
    g.stream = (hipStream_t)stream;
    long long pool_elems = 0;
    for (int i = 0; i < n; ++i) pool_elems = std::max(pool_elems, offsets[i] + (long long)p[i].L * p[i].L);
    int32_t *work = d_work_pool;
    if (!work && (st = g.dev_alloc((void **)&work, (size_t)pool_elems * 4)) != RSOS_OK) { delete b; return st; }
    long long *logs = nullptr;
    if ((st = g.dev_alloc((void **)&logs, sizeof(long long) * 3 * log_cap * n)) != RSOS_OK) { g.destroy(); delete b; return st; }
    for (int i = 0; i < n; ++i) {
        SurfDev d = {};
        if (g.packed) {
            // the surface's int32[L^2] of the pool holds both residue buffers
            d.buf[0] = d_pool + offsets[i];
            d.buf[1] = (int32_t *)((uint16_t *)(d_pool + offsets[i]) + (size_t)p[i].L * p[i].L);
            g.readout.push_back(work + offsets[i]);
        } else {
            d.buf[0] = d_pool + offsets[i];
            d.buf[1] = work + offsets[i];
        }
        d.log = logs + 3 * log_cap * i;
        d.log_cap = log_cap;
        d.key0 = (uint32_t)(p[i].seed & 0xFFFFFFFFu);
        d.key1 = (uint32_t)(p[i].seed >> 32);
        d.L = p[i].L;
        d.N = p[i].N;
        d.T = p[i].L / p[i].D;
        g.host.push_back(d);
        g.max_h0.push_back(0);
        g.t0.push_back(0);
    }
    if (tuning_wanted(&p[0])) {
        // one tuned choice per (L, N) class, grouped into kernel instances,
        // unless one variant for all times faster on this mix
        g.want.assign(n, Choice());
        std::vector<std::pair<int, int>> LN;
        std::vector<Choice> plan;
        for (int i = 0; i < n; ++i) {
            if (uses_lds(p[i].L)) continue;
            if ((st = tuned_choice(&p[i], 1, &g.want[i])) != RSOS_OK) {
                g.destroy();
                delete b;
                return st;
            }
            LN.push_back({p[i].L, p[i].N});
            plan.push_back(g.want[i]);
        }
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            st = batch_plan(p[0].D, (int)p[0].flags, LN, &plan);
        }
        if (st != RSOS_OK) { g.destroy(); delete b; return st; }
        for (int i = 0, k = 0; i < n; ++i)
            if (!uses_lds(p[i].L)) g.want[i] = plan[k++];
    }
    if ((st = mark(g, g.setup())) != RSOS_OK) { g.destroy(); delete b; return st; }
    for (int i = 0; i < n; ++i)
        if ((st = g.load_initial(i, nullptr, 0)) != RSOS_OK || (st = g.init_record(i, 0, 0)) != RSOS_OK) {
            g.destroy();
            delete b;
            return st;
        }
    if ((st = mark(g, g.prepare_graph())) != RSOS_OK) { g.destroy(); delete b; return st; }
    *out = b;
    return RSOS_OK;
}

rsos_status rsos_batch_sweep(rsos_batch *b, const int64_t *n_mcs, int64_t n_all)
{
    CHECK_HANDLE(b, b->g);
    SurfaceGroup &g = b->g;
    const int n = (int)g.host.size();
    std::vector<long long> t_end(n);
    long long most = 0;
    for (int i = 0; i < n; ++i) {
        const long long k = n_mcs ? n_mcs[i] : n_all;
        if (k < 0) return fail(RSOS_E_INVAL, "negative sweep count for surface %d", i);
        if (g.host[i].t + k > (1ll << 32)) return fail(RSOS_E_INVAL, "sweep index would exceed 2^32");
        rsos_status st = check_overflow(b->p[i], g.max_h0[i], g.host[i].t + k - g.t0[i]);
        if (st != RSOS_OK) return st;
        t_end[i] = g.host[i].t + k;
        most = std::max(most, k);
    }
    if (most == 0) return RSOS_OK;
    rsos_status st;
    if ((st = mark(g, g.set_t_end(t_end, most))) != RSOS_OK) return st;
    if ((st = mark(g, g.launch_sweeps(most))) != RSOS_OK) return st;
    for (int i = 0; i < n; ++i) g.host[i].t = t_end[i];
    return RSOS_OK;
}

rsos_status rsos_batch_width(rsos_batch *b, rsos_width_t *out)
{
    CHECK_HANDLE(b, b->g);
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    for (size_t i = 0; i < b->g.host.size(); ++i) {
        rsos_status st = mark(b->g, b->g.read_log((int)i, b->g.host[i].t, 1, out + i));
        if (st != RSOS_OK) return st;
    }
    return RSOS_OK;
}

rsos_status rsos_batch_log(rsos_batch *b, int32_t i, int64_t t_from, int64_t n, rsos_width_t *out)
{
    CHECK_HANDLE(b, b->g);
    if (i < 0 || i >= (int)b->g.host.size()) return fail(RSOS_E_INVAL, "surface index out of range");
    if (!out && n > 0) return fail(RSOS_E_INVAL, "out is NULL");
    return mark(b->g, b->g.read_log(i, t_from, n, out));
}

rsos_status rsos_batch_moments(rsos_batch *b, int32_t i, rsos_moments_t *out)
{
    CHECK_HANDLE(b, b->g);
    if (i < 0 || i >= (int)b->g.host.size()) return fail(RSOS_E_INVAL, "surface index out of range");
    if (!out) return fail(RSOS_E_INVAL, "out is NULL");
    return mark(b->g, b->g.moments(i, out));
}

rsos_status rsos_batch_heights(rsos_batch *b, int32_t i, int32_t *dst, int dst_is_device)
{
    CHECK_HANDLE(b, b->g);
    if (i < 0 || i >= (int)b->g.host.size()) return fail(RSOS_E_INVAL, "surface index out of range");
    if (!dst) return fail(RSOS_E_INVAL, "dst is NULL");
    return mark(b->g, b->g.copy_heights(i, dst, dst_is_device));
}

rsos_status rsos_batch_free(rsos_batch *b)
{
    if (!b) return RSOS_OK;
    b->g.destroy();
    delete b;
    return RSOS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Sweeps without any allocation (rsos_sweep_static).  The descriptor, the
// accumulator area and the log ring of the one surface live in `scratch`, a
// file-scope device array that every GPU the library runs on holds once
// until the process ends.  In host code its name is a host-side stand-in;
// the entry point takes the array's device address on each device with
// hipGetSymbolAddress the first time it runs there and uses that address
// only.  Calls on one GPU share the array: they must not overlap.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = 128 * 1024;
constexpr size_t kScratchDesc = 0;      // SurfDev
constexpr size_t kScratchIdx = 128;     // int 0: the LDS-path kernel's descriptor index
constexpr size_t kScratchAcc = 256;     // kAccWords int64
constexpr size_t kScratchLog = 2048;    // log ring of kStaticLogCap records of 3 int64
constexpr long long kStaticLogCap = RSOS_STATIC_MAX_SWEEPS + 1;
static_assert(sizeof(SurfDev) <= kScratchIdx, "descriptor slot");
static_assert(kScratchAcc + 8 * rsosk::kAccWords <= kScratchLog, "accumulator slot");
static_assert(kScratchLog + 24 * (size_t)kStaticLogCap <= kScratchBytes, "log ring");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device.
rsos_status scratch_ptr(unsigned char **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RSOS_E_INVAL, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(RSOS_E_DEVICE, "no device address for the scratch array");
        g_scratch[dev] = (unsigned char *)p;
    }
    *out = g_scratch[dev];
    return RSOS_OK;
}

}  // namespace

// Writes the descriptor, clears the accumulators and stores the record of
// time t0 (a fill kernel, not a memset: callers may capture the launches).
__global__ void static_setup(SurfDev d, unsigned char *base, long long s1, long long s2)
{
    long long *acc = (long long *)(base + kScratchAcc);
    for (int i = threadIdx.x; i < rsosk::kAccWords; i += blockDim.x) acc[i] = 0;
    if (threadIdx.x == 0) {
        *(int *)(base + kScratchIdx) = 0;
        const long long L2 = (long long)d.L * d.L;
        acc[rsosk::kMeanWord] = s1 / L2;
        long long *rec = d.log + 3 * (d.t % d.log_cap);
        rec[0] = s1;
        rec[1] = s2;
        rec[2] = 0;
        *(SurfDev *)(base + kScratchDesc) = d;
    }
}

// Records of times t0+1 .. t0+n from the ring into the caller's int64[3n].
__global__ void static_copy_log(const unsigned char *base, long long t0, long long n, long long *out)
{
    const long long *ring = (const long long *)(base + kScratchLog);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long k = i / 3, w = i % 3;
        out[i] = ring[3 * ((t0 + 1 + k) % kStaticLogCap) + w];
    }
}

extern "C" rsos_status rsos_sweep_static(const rsos_params *p, int32_t *d_h, int32_t *d_work, int64_t t0,
                                         int64_t s1, int64_t s2, int64_t n_mcs, int64_t *d_log, void *stream)
{
    rsos_status st = check_params(p);
    if (st != RSOS_OK) return st;
    if (p->flags & ~RSOS_FLAG_DT4)
        return fail(RSOS_E_INVAL, "rsos_sweep_static: flags may only select the schedule (RSOS_FLAG_DT4)");
    if (!d_h || !d_work || (n_mcs > 0 && !d_log)) return fail(RSOS_E_INVAL, "NULL buffer");
    if (n_mcs < 0 || n_mcs > RSOS_STATIC_MAX_SWEEPS)
        return fail(RSOS_E_INVAL, "n_mcs=%lld outside [0, %d]", (long long)n_mcs, RSOS_STATIC_MAX_SWEEPS);
    if (t0 < 0 || t0 + n_mcs > (1ll << 32)) return fail(RSOS_E_INVAL, "sweep index would exceed 2^32");
    if ((((uintptr_t)d_h) | ((uintptr_t)d_work)) & 15) return fail(RSOS_E_INVAL, "height buffers must be 16-byte aligned");
    const long long L2 = (long long)p->L * p->L;
    if (s1 < 0 || s2 < 0 || (__int128)s1 * s1 > (__int128)L2 * s2)
        return fail(RSOS_E_INVAL, "s1, s2 are not the sums of any heights (need 0 <= s1, s1^2 <= L^2 s2)");
    // every height is within N L of the mean s1 / L^2
    if ((st = check_overflow(*p, s1 / L2 + 1 + (long long)p->N * p->L, n_mcs)) != RSOS_OK) return st;
    if (n_mcs == 0) return RSOS_OK;
    unsigned char *base = nullptr;
    if ((st = scratch_ptr(&base)) != RSOS_OK) return st;
    const int D = p->D, sched = (p->flags & RSOS_FLAG_DT4) ? 1 : 0;
    SurfDev d = {};
    d.buf[0] = d_h;
    d.buf[1] = d_work;
    d.log = (long long *)(base + kScratchLog);
    d.acc = (long long *)(base + kScratchAcc);
    d.log_cap = kStaticLogCap;
    d.t = t0;
    d.t_end = t0 + n_mcs;
    d.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(p->seed >> 32);
    d.L = p->L;
    d.N = p->N;
    d.T = p->L / D;
    const Variant *v = nullptr;
    if (!uses_lds(p->L)) {
        v = pick_variant(D, {{p->L, p->N}}, false, sched == 1);
        if (!v) return fail(RSOS_E_INVAL, "no tile-block shape fits L=%d, N=%d, D=%d", p->L, p->N, D);
        d.nbx = d.T / v->TX;
        d.nblocks = d.nbx * (d.T / v->TY);
        d.block_start = 0;
    }
    hipStream_t s = (hipStream_t)stream;
    SurfDev *dd = (SurfDev *)(base + kScratchDesc);
    hipLaunchKernelGGL(static_setup, dim3(1), dim3(256), 0, s, d, base, (long long)s1, (long long)s2);
    HIP_TRY(hipGetLastError());
    if (!v) {
        // the whole surface in one workgroup's LDS, all sweeps in one launch
        lds_launcher(D, sched)(dim3(1), (size_t)L2 * 4, s, dd, (const int *)(base + kScratchIdx));
        HIP_TRY(hipGetLastError());
    } else {
        BlockLaunch k = sched == 1 ? v->launch_dt : v->launch;
        for (long long i = 0; i < n_mcs; ++i) k(dim3(d.nblocks), s, dd, 1, nullptr, 1, d.nbx, nullptr, nullptr);
        HIP_TRY(hipGetLastError());
    }
    const unsigned grid = (unsigned)std::min<long long>((3 * n_mcs + 255) / 256, 64);
    hipLaunchKernelGGL(static_copy_log, dim3(grid), dim3(256), 0, s, base, (long long)t0, (long long)n_mcs,
                       (long long *)d_log);
    HIP_TRY(hipGetLastError());
    return RSOS_OK;
}

// ---------------------------------------------------------------------------
// serving engine (continuous batching) -- see rsos_engine.inc
// ---------------------------------------------------------------------------
#include "rsos_engine.inc"

// ---------------------------------------------------------------------------
// multisurface lock-step mode -- see rsos_ms.inc
// ---------------------------------------------------------------------------
#include "rsos_ms.inc"

// rsos_host.hpp -- host-only logic of librsos.so: error reporting, the
// validation of initial heights, the overflow bound and W^2 from the exact
// sums (Eq. (2)), and the serving engine's pool allocator.  No HIP here, so
// the same code also builds with g++ and the sanitizers for the host tests.
#pragma once

#include "rsos.h"

#include <stdint.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <iterator>
#include <map>
#include <string>

namespace rsosh {

inline thread_local std::string g_last_error;
// rsos_debug_fail: the HIP runtime check that brings this to 0 reports a
// failure (0: off)
inline thread_local int g_fail_countdown = 0;

inline rsos_status fail(rsos_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}


// H bounds every height after dt more sweeps: the mean grows at most one
// per sweep and the restriction keeps the spread on the torus <= N L; also
// no site gets more than D^2 deposits per sweep.
inline rsos_status check_overflow(const rsos_params &p, long long max_h0, long long dt)
{
    const __int128 a = (__int128)dt + (__int128)p.N * p.L;
    const __int128 b = (__int128)dt * p.D * p.D;
    const __int128 H = (__int128)max_h0 + (a < b ? a : b);
    if (H >= ((__int128)1 << 31) - 1) return fail(RSOS_E_OVERFLOW, "heights could reach 2^31");
    const __int128 LH = (__int128)p.L * H;
    if (LH * LH >= ((__int128)1 << 63)) return fail(RSOS_E_OVERFLOW, "sum h^2 could reach 2^63");
    return RSOS_OK;
}

inline double w2_of(int L, long long s1, long long s2)
{
    const __int128 L2 = (__int128)L * L;
    const __int128 num = L2 * s2 - (__int128)s1 * s1;
    return (double)num / ((double)L2 * (double)L2);
}

inline rsos_status validate_h0(const int32_t *h, int L, int N, long long *max_h, long long *s1, long long *s2)
{
    long long mx = 0, a = 0, b = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const long long c = h[(size_t)y * L + x];
            if (c < 0 || c >= (1ll << 30)) return fail(RSOS_E_INVAL, "h0 outside [0, 2^30)");
            const long long r = h[(size_t)y * L + (x + 1) % L];
            const long long u = h[(size_t)((y + 1) % L) * L + x];
            if (llabs(c - r) > N || llabs(c - u) > N)
                return fail(RSOS_E_RSOS, "h0 violates |dh| <= %d at (%d, %d)", N, x, y);
            mx = std::max(mx, c);
            a += c;
            b += c * c;
        }
    *max_h = mx;
    *s1 = a;
    *s2 = b;
    return RSOS_OK;
}


constexpr size_t kPoolAlign = 256;

// First-fit allocator over [0, total) with coalescing free list.
struct PoolAlloc {
    std::map<size_t, size_t> free_;  // offset -> size
    size_t total = 0, used = 0;

    void init(size_t n)
    {
        total = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + kPoolAlign - 1) & ~(kPoolAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used += n;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + kPoolAlign - 1) & ~(kPoolAlign - 1);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace rsosh

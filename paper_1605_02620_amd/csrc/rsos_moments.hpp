// rsos_moments.hpp -- gfx950 kernels of the height-distribution moments.
//
// The skewness S_h and kurtosis Q_h of the heights (Eqs. (13)-(15)) are
// ratios of sample averages of the central moments Phi_2..Phi_4 of each
// surface's height distribution.  These kernels compute, for one state, the
// exact power sums about an integer reference, from which the host forms
// the central moments.
#pragma once

#include "rsos_kernels.hpp"

namespace rsosk {

// ---------------------------------------------------------------------------
// Power sums of the height distribution (the moments of Eqs. (13)-(15)):
// C_k = sum over sites of (h - R)^k, k = 1..4, with R = floor(S1 / L^2) of
// the current state, exact.  |h - R| never exceeds the largest height H,
// and the library keeps L^2 H^2 < 2^63, so C_1 and C_2 fit int64 and C_3,
// C_4 fit int128.  A thread sums the sites with |h - R| < 2^11 in int64
// (terms below 2^44, at most 2^16 sites per thread) and the rare others in
// int128; workgroup totals go to part[4 * blockIdx.x + k], and
// power_sums_final adds them into out[0..3].  With 16-bit storage R is also
// the reference the residues are decoded against (floor(S1 / L^2) of the
// same time), so h - R = int16(r - R mod 2^16).
// ---------------------------------------------------------------------------
typedef __int128 i128;

__device__ __forceinline__ i128 shfl_xor_i128(i128 v, int m)
{
    const unsigned long long lo = (unsigned long long)v, hi = (unsigned long long)((unsigned __int128)v >> 64);
    const unsigned long long l2 = __shfl_xor(lo, m, 64), h2 = __shfl_xor(hi, m, 64);
    return (i128)(((unsigned __int128)h2 << 64) | l2);
}

// Sum over the workgroup; result valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_reduce_i128x4(i128 v[4])
{
    __shared__ i128 red[4][NT / 64];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += shfl_xor_i128(v[k], off);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0)
        for (int k = 0; k < 4; ++k) red[k][w] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k)
            for (int i = 1; i < NT / 64; ++i) v[k] += red[k][i];
}

struct PowerAcc {
    long long a[4] = {0, 0, 0, 0};
    i128 b[4] = {0, 0, 0, 0};
    __device__ __forceinline__ void add(int x)
    {
        if (x >= -2048 && x < 2048) {
            const int x2 = x * x;
            a[0] += x;
            a[1] += x2;
            a[2] += (long long)x2 * x;
            a[3] += (long long)x2 * x2;
        } else {
            const i128 X = x, X2 = X * X;
            b[0] += X;
            b[1] += X2;
            b[2] += X2 * X;
            b[3] += X2 * X2;
        }
    }
};

// S = int32_t: heights; S = uint16_t: residues.  n % 8 == 0, 16-byte
// aligned buffer; rec points to the current log record (S1 first).
template <typename S>
__global__ __launch_bounds__(256) void power_sums_partial(const S *__restrict__ h, long long n,
                                                          const long long *__restrict__ rec,
                                                          long long *__restrict__ part)
{
    const long long R = rec[0] / n;
    PowerAcc acc;
    constexpr int CPC = 16 / sizeof(S);
    const long long nch = n / CPC;
    for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < nch; c += (long long)gridDim.x * 256) {
        if constexpr (sizeof(S) == 4) {
            const int4 v = load4(as_global(h) + 4 * c);
            acc.add((int)((long long)v.x - R));
            acc.add((int)((long long)v.y - R));
            acc.add((int)((long long)v.z - R));
            acc.add((int)((long long)v.w - R));
        } else {
            const v4u v = *reinterpret_cast<const gv4u *>((const gu16 *)h + 8 * c);
            const uint32_t r0 = (uint32_t)R & 0xFFFFu;
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc.add((int)(int16_t)(uint16_t)((w[k] & 0xFFFFu) - r0));
                acc.add((int)(int16_t)(uint16_t)((w[k] >> 16) - r0));
            }
        }
    }
    i128 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (i128)acc.a[k] + acc.b[k];
    block_reduce_i128x4<256>(v);
    if (threadIdx.x == 0) {
        i128 *out = reinterpret_cast<i128 *>(part) + 4 * blockIdx.x;
        for (int k = 0; k < 4; ++k) out[k] = v[k];
    }
}

__global__ __launch_bounds__(256) void power_sums_final(const long long *__restrict__ part, int nparts,
                                                        long long *__restrict__ out)
{
    i128 v[4] = {0, 0, 0, 0};
    const i128 *p = reinterpret_cast<const i128 *>(part);
    for (int i = threadIdx.x; i < nparts; i += 256)
        for (int k = 0; k < 4; ++k) v[k] += p[4 * i + k];
    block_reduce_i128x4<256>(v);
    if (threadIdx.x == 0) {
        i128 *o = reinterpret_cast<i128 *>(out);
        for (int k = 0; k < 4; ++k) o[k] = v[k];
    }
}

}  // namespace rsosk

// device_common.h -- device-side building blocks shared by the FRSVT kernels
// (gfx950, wave64): the Philox4x32-10 Gaussian stream, wavefront reductions,
// small helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace frk {

constexpr int kWave = 64;
constexpr int kThreads = 256;
constexpr double kU = 1.1102230246251565e-16;  // unit roundoff of double

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64-bit products; the key advances by the Weyl increments between
// rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// (c + 1/2) 2^-53 for the 53-bit integer c formed by the top 27 bits of a and
// the top 26 bits of b: a uniform number in (0, 1].
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) *
           (1.0 / 9007199254740992.0);
}

// The Gaussian test matrix of the sketch: Omega(k, 2j + e) is output e of a
// Box-Muller transform of the Philox block with counter {k, j, ctr lo, ctr hi}
// and key = seed.
__device__ __forceinline__ void gaussian_pair(uint64_t seed, uint64_t counter, uint32_t row,
                                              uint32_t pair, double &z0, double &z1)
{
    uint32_t c[4] = {row, pair, (uint32_t)counter, (uint32_t)(counter >> 32)};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = uniform53(c[0], c[1]);
    const double u2 = uniform53(c[2], c[3]);
    const double radius = sqrt(-2.0 * log(u1));
    double s, co;
    sincos(6.283185307179586476925286766559 * u2, &s, &co);
    z0 = radius * co;
    z1 = radius * s;
}

// Replacement directions for numerically null basis columns use a disjoint
// part of the counter space (high bit of the pair word set).
constexpr uint32_t kRefillTag = 0x80000000u;

// ---------------------------------------------------------------------------
// Wavefront reductions through DPP lane moves (VALU, no LDS round trip):
// within a 16-lane row the partners are quad_perm [1,0,3,2], quad_perm
// [2,3,0,1], row_half_mirror and row_mirror; after each step every lane of
// the segment holds the same value (x + y and y + x round identically).  The
// four row sums of a wavefront are then read from lanes 0, 16, 32, 48 and
// added in that order.  Floating-point contraction is off inside these
// helpers: an add fused with the caller's product (x*x + dpp(x*x) as one
// FMA) would round differently in the two lanes of a pair, and lanes that
// must agree (a Jacobi rotation) would not.
// ---------------------------------------------------------------------------
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_mov(T v)
{
    // every lane's source is inside its row for the patterns used here, so
    // the old value is never kept (bound_ctrl set, no initialised old)
    if constexpr (sizeof(T) == 8) {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
        return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned)lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
    }
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <typename T>
__device__ __forceinline__ T seg8_sum(T v)
{
#pragma clang fp contract(off)
    v += dpp_mov<kDppXor1>(v);
    v += dpp_mov<kDppXor2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    return v;
}
// Three independent 8-lane sums stepped together, so that the latency of
// one chain's DPP move and add passes while the others issue.  Each result
// is bit-identical to seg8_sum of the same input.
template <typename T>
__device__ __forceinline__ void seg8_sum3(T &a, T &b, T &c)
{
#pragma clang fp contract(off)
    T ta = dpp_mov<kDppXor1>(a), tb = dpp_mov<kDppXor1>(b), tc = dpp_mov<kDppXor1>(c);
    a += ta;
    b += tb;
    c += tc;
    ta = dpp_mov<kDppXor2>(a);
    tb = dpp_mov<kDppXor2>(b);
    tc = dpp_mov<kDppXor2>(c);
    a += ta;
    b += tb;
    c += tc;
    ta = dpp_mov<kDppHalfMirror>(a);
    tb = dpp_mov<kDppHalfMirror>(b);
    tc = dpp_mov<kDppHalfMirror>(c);
    a += ta;
    b += tb;
    c += tc;
}
template <typename T>
__device__ __forceinline__ T seg16_sum(T v)
{
#pragma clang fp contract(off)
    v = seg8_sum(v);
    v += dpp_mov<kDppMirror>(v);
    return v;
}
__device__ __forceinline__ double read_lane(double v, int l)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float read_lane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
// lanes 0-31 get the sum over lanes 0-31, lanes 32-63 over lanes 32-63
template <typename T>
__device__ __forceinline__ T seg32_sum(T v)
{
#pragma clang fp contract(off)
    v = seg16_sum(v);
    const T lo = read_lane(v, 0) + read_lane(v, 16), hi = read_lane(v, 32) + read_lane(v, 48);
    return (threadIdx.x & 32) ? hi : lo;
}
__device__ __forceinline__ double wave_sum(double v)
{
#pragma clang fp contract(off)
    v = seg16_sum(v);
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}
__device__ __forceinline__ float wave_sum(float v)
{
#pragma clang fp contract(off)
    v = seg16_sum(v);
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_mov<kDppXor1>(v));
    v = fmax(v, dpp_mov<kDppXor2>(v));
    v = fmax(v, dpp_mov<kDppHalfMirror>(v));
    v = fmax(v, dpp_mov<kDppMirror>(v));
    return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// 1/sqrt(x) for a normal, finite x > 0 (no denormal or overflow handling):
// the hardware estimate refined by two Newton steps y (3/2 - x y^2 / 2), each
// doubling the correct bits, to within a few units in the last place.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}

__device__ __forceinline__ double soft_shrink(double x, double t)
{
    const double a = fabs(x) - t;
    return a > 0.0 ? copysign(a, x) : 0.0;
}

__device__ __forceinline__ float soft_shrink(float x, float t)
{
    const float a = fabsf(x) - t;
    return a > 0.0f ? copysignf(a, x) : 0.0f;
}

}  // namespace frk

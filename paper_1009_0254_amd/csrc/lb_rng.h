// Device random numbers of the library (private): Philox4x32-10 and Box-Muller.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lbf {

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror & Shaw, SC'11: 10 rounds of two 32x32->64 products with the
// multipliers 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule 0x9E3779B9 / 0xBB67AE85.
// The three-way exclusive or of a round is one gfx950 v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        // The callers vary only the first counter word across lanes, so some words stay uniform
        // for the first rounds: the first round's products of words 2 and 3 and its x, y; the
        // second round's hi0, lo0 (from that x).  There the exclusive ors pair the uniform
        // operands first (scalar instructions), as a three-way vector or may read only one scalar
        // operand and would need a move for the second; from the third round on one v_bitop3 each.
        if (r == 0)
            c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        else if (r == 1)
            c = make_uint4(hi1 ^ (c.y ^ k0), lo1, c.w ^ (hi0 ^ k1), lo0);
        else if (r == 2)
            c = make_uint4(xor3(hi1, c.y, k0), lo1, hi0 ^ (c.w ^ k1), lo0);
        else
            c = make_uint4(xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0);
    }
    return c;
}

// the six 21-bit integers of one Philox block: the top 21 bits of each word, then the
// low 11 bits of words (0,1) and (2,3) joined (dropping one bit of words 1 and 3)
__device__ __forceinline__ void bits21(uint4 x, uint32_t b[6])
{
    b[0] = x.x >> 11;
    b[1] = x.y >> 11;
    b[2] = x.z >> 11;
    b[3] = x.w >> 11;
    b[4] = ((x.x & 0x7FFu) << 10) | ((x.y & 0x7FFu) >> 1);
    b[5] = ((x.z & 0x7FFu) << 10) | ((x.w & 0x7FFu) >> 1);
}

// Box-Muller on u = (b + 1/2) 2^-21 (exact in float and double)
// ------------------------------------------------------------------ FP64 ln u, sin and cos of 2 pi u
// Box-Muller meets these only at u = (b + 1/2) 2^-21 with b a 21-bit integer, which admits exact
// argument reductions and short series instead of the general-argument library routines.  The
// operations are products, sums, explicit fma, one division and bit manipulation, all correctly
// rounded, so a host build of these functions gives the same bits (checked there over every b
// against long-double references).

// ln u: u = (2 b + 1) 2^-22 (exact) = m 2^e with m in [sqrt(1/2), sqrt(2)), m - 1 exact; ln m =
// 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716, by its series to the s^19 term (truncation
// below 3e-17 relative); e ln 2 with ln 2 = hi + lo, hi being ln 2 rounded to 40 significant
// bits (so that e hi is exact for |e| <= 22) and lo the rest rounded to double.
__host__ __device__ inline double u21_ln(uint32_t b)
{
    const double u = (double)(2u * b + 1u) * 0x1p-22;
    const unsigned long long bits = __builtin_bit_cast(unsigned long long, u);
    int e = (int)((bits >> 52) & 0x7FFu) - 1023;
    double m = __builtin_bit_cast(double, (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (m > 1.4142135623730951) {
        m *= 0.5;
        ++e;
    }
    const double f = m - 1.0;
    const double sv = f / (2.0 + f);
    const double z = sv * sv;
    double p = 1.0 / 19.0;
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double s2 = 2.0 * sv;
    const double lnm = fma(s2 * z, p, s2);
    const double de = (double)e;
    return fma(de, 0x1.62e42fefa4000p-1, fma(de, -0x1.8432a1b0e2634p-43, lnm));
}

// sin and cos of 2 pi u: the angle is n pi 2^-21 with n = 2 b + 1; its quarter turns q = n >> 20
// and the odd rest m = n mod 2^20 reduce it exactly to x = m' pi 2^-21 in (0, pi/4] (m' = m, or
// 2^20 - m with sine and cosine exchanged); sin x and cos x by their Taylor series to x^17 and
// x^18 (truncation below 1e-19).
__host__ __device__ inline void u21_sincos_turn(uint32_t b, double &sn, double &cs)
{
    const uint32_t n = 2u * b + 1u, q = n >> 20, m = n & 0xFFFFFu;
    const bool comp = m > 0x80000u;
    const double x = (double)(comp ? 0x100000u - m : m) * 0x1.921fb54442d18p-20;   // pi 2^-21
    const double z = x * x;
    double ps = 1.0 / 355687428096000.0;   // 1/17!
    ps = fma(ps, z, -1.0 / 1307674368000.0);
    ps = fma(ps, z, 1.0 / 6227020800.0);
    ps = fma(ps, z, -1.0 / 39916800.0);
    ps = fma(ps, z, 1.0 / 362880.0);
    ps = fma(ps, z, -1.0 / 5040.0);
    ps = fma(ps, z, 1.0 / 120.0);
    ps = fma(ps, z, -1.0 / 6.0);
    const double sx = fma(x * z, ps, x);
    double pc = -1.0 / 6402373705728000.0;   // -1/18!
    pc = fma(pc, z, 1.0 / 20922789888000.0);
    pc = fma(pc, z, -1.0 / 87178291200.0);
    pc = fma(pc, z, 1.0 / 479001600.0);
    pc = fma(pc, z, -1.0 / 3628800.0);
    pc = fma(pc, z, 1.0 / 40320.0);
    pc = fma(pc, z, -1.0 / 720.0);
    pc = fma(pc, z, 1.0 / 24.0);
    pc = fma(pc, z, -0.5);
    const double cx = fma(z, pc, 1.0);
    const double s0 = comp ? cx : sx, c0 = comp ? sx : cx;   // of the rest m pi 2^-21
    sn = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
    cs = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
}

template <typename R> struct Gauss;

// the angle's revolutions plus one whole turn, 1 + (b + 1/2) 2^-21, assembled from the bits
// (exponent of 1, mantissa 4 b + 2): v_sin/v_cos take revolutions, so the added turn changes
// nothing and saves the conversion
__device__ __forceinline__ float turn21(uint32_t b) { return __builtin_bit_cast(float, 0x3F800002u | (b << 2)); }

template <> struct Gauss<float> {
    static __device__ __forceinline__ void pair(uint32_t be, uint32_t bo, float &a, float &b)
    {
#pragma clang fp contract(on)
        const float ue = ((float)be + 0.5f) * 0x1p-21f;
        const float uo = turn21(bo);
        // -2 ln u = -2 ln(2) log2(u); v_log_f32 is log2, v_sin/v_cos take revolutions
        const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ue));
        a = r * __builtin_amdgcn_cosf(uo);
        b = r * __builtin_amdgcn_sinf(uo);
    }
};

template <> struct Gauss<double> {
    static __device__ __forceinline__ void pair(uint32_t be, uint32_t bo, double &a, double &b)
    {
#pragma clang fp contract(on)
        const double r = sqrt(-2.0 * u21_ln(be));
        double s, c;
        u21_sincos_turn(bo, s, c);
        a = r * c;
        b = r * s;
    }
};

// Box-Muller with the radius scaled: scale * (the pair above)
template <typename R> __device__ __forceinline__ void gauss_pair_scaled(uint32_t be, uint32_t bo, R scale, R &a, R &b);
template <> __device__ __forceinline__ void gauss_pair_scaled<float>(uint32_t be, uint32_t bo, float scale, float &a, float &b)
{
#pragma clang fp contract(on)
    const float ue = ((float)be + 0.5f) * 0x1p-21f;
    const float uo = turn21(bo);
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ue)) * scale;
    a = r * __builtin_amdgcn_cosf(uo);
    b = r * __builtin_amdgcn_sinf(uo);
}
template <> __device__ __forceinline__ void gauss_pair_scaled<double>(uint32_t be, uint32_t bo, double scale, double &a, double &b)
{
#pragma clang fp contract(on)
    const double r = sqrt(-2.0 * u21_ln(be)) * scale;
    double s, c;
    u21_sincos_turn(bo, s, c);
    a = r * c;
    b = r * s;
}

// the six normals of (node, rep, t), each multiplied by `scale`
template <typename R>
__device__ __forceinline__ void normals6s(uint32_t node, uint32_t rep, unsigned long long t, uint32_t k0,
                                          uint32_t k1, R scale, R nu[6])
{
    const uint4 x = philox10(make_uint4(node, rep, (uint32_t)t, (uint32_t)(t >> 32)), k0, k1);
    uint32_t b[6];
    bits21(x, b);
    gauss_pair_scaled<R>(b[0], b[1], scale, nu[0], nu[1]);
    gauss_pair_scaled<R>(b[2], b[3], scale, nu[2], nu[3]);
    gauss_pair_scaled<R>(b[4], b[5], scale, nu[4], nu[5]);
}

template <typename R>
__device__ __forceinline__ void normals6(uint32_t node, uint32_t rep, unsigned long long t, uint32_t k0,
                                         uint32_t k1, R nu[6])
{
    const uint4 x = philox10(make_uint4(node, rep, (uint32_t)t, (uint32_t)(t >> 32)), k0, k1);
    uint32_t b[6];
    bits21(x, b);
    Gauss<R>::pair(b[0], b[1], nu[0], nu[1]);
    Gauss<R>::pair(b[2], b[3], nu[2], nu[3]);
    Gauss<R>::pair(b[4], b[5], nu[4], nu[5]);
}

// element at a 32-bit byte offset from a uniform base (lets the compiler address with an
// SGPR base and one 32-bit VGPR offset)
}  // namespace lbf

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
        const double ue = ((double)be + 0.5) * 0x1p-21;
        const double uo = ((double)bo + 0.5) * 0x1p-21;
        const double r = sqrt(-2.0 * log(ue));
        double s, c;
        sincospi(2.0 * uo, &s, &c);
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
    const double ue = ((double)be + 0.5) * 0x1p-21;
    const double uo = ((double)bo + 0.5) * 0x1p-21;
    const double r = sqrt(-2.0 * log(ue)) * scale;
    double s, c;
    sincospi(2.0 * uo, &s, &c);
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

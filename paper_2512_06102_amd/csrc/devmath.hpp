// devmath.hpp -- device building blocks of the stochastic step: the
// counter-based generator, the exponential, and the neighbour geometry.
//
// The step's results are defined bit for bit, so every routine here uses only
// IEEE fp32 add, subtract, multiply, round-to-nearest-even and compares, in a
// fixed order (the library is built with -ffp-contract=off, so no
// multiply-add is fused, and with fp32 denormals kept).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace firesim {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, section 4.2): ten rounds
// of two 32x32->64 multiplies mixing the four counter words, the two key
// words bumped by Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, uint2 key)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round != 0) {
            key.x += kWeylA;
            key.y += kWeylB;
        }
        // one 32 x 32 -> 64-bit product per multiplier: a single v_mad_u64_u32,
        // which runs Philox 1.26x faster on gfx950 than separate low and high
        // multiplies (same bits)
        const uint64_t pa = (uint64_t)kMulA * x.x, pb = (uint64_t)kMulB * x.z;
        x = make_uint4((uint32_t)(pb >> 32) ^ x.y ^ key.x, (uint32_t)pb, (uint32_t)(pa >> 32) ^ x.w ^ key.y,
                       (uint32_t)pa);
    }
    return x;
}

// 24-bit uniform in [0, 1 - 2^-24] from one Philox word.
__device__ __forceinline__ float word_to_uniform(uint32_t w)
{
    return (float)(w >> 8) * 5.9604644775390625e-8f;  // 2^-24
}

// e^x in fp32: x = n ln2 + r with n = rint(x / ln2) (Cody & Waite 1980
// reduction; ln2 split into a 15-bit head so n * head is exact), e^r from
// its Taylor series through r^7 evaluated by Horner's rule, then scaled by
// 2^n through the exponent field.  Defined on [-87, 88]: 0 below, e^88
// above (results there stay normal, so the scaling is exact).
__device__ __forceinline__ float exp_c(float x)
{
    constexpr float kInvLn2 = (float)1.44269504088896340736;
    constexpr float kLn2Head = 0.693145751953125f;  // 22713 * 2^-15
    constexpr float kLn2Tail = (float)(0.69314718055994530942 - 0.693145751953125);
    constexpr float kT2 = 0.5f, kT3 = (float)(1.0 / 6.0), kT4 = (float)(1.0 / 24.0);
    constexpr float kT5 = (float)(1.0 / 120.0), kT6 = (float)(1.0 / 720.0);
    constexpr float kT7 = (float)(1.0 / 5040.0);
    if (x != x) return x;
    if (x < -87.0f) return 0.0f;
    if (x > 88.0f) x = 88.0f;
    const float n = __builtin_rintf(x * kInvLn2);
    const float r = (x - n * kLn2Head) - n * kLn2Tail;
    float poly = kT7;
    poly = poly * r + kT6;
    poly = poly * r + kT5;
    poly = poly * r + kT4;
    poly = poly * r + kT3;
    poly = poly * r + kT2;
    poly = poly * r + 1.0f;
    poly = poly * r + 1.0f;
    const float two_n = __int_as_float(((int)n + 127) << 23);
    return poly * two_n;
}

// arctan in fp32 for the slope-angle variant: odd; pi/2 - atan(1/x) above
// 1; pi/4 + atan((a-1)/(a+1)) above tan(pi/8); then the Taylor series
// t - t^3/3 + t^5/5 - ... - t^19/19 in t^2 by Horner's rule (|t| <= tan(pi/8),
// truncation below 1e-8 relative).  IEEE divisions, no contraction.
__device__ __forceinline__ float atan_c(float x)
{
    constexpr float kTanPi8 = (float)0.41421356237309504880;
    constexpr float kPi4 = (float)0.78539816339744830962, kPi2 = (float)1.57079632679489661923;
    if (x != x) return x;
    const bool neg = x < 0.0f;
    float a = neg ? -x : x;
    const bool inv = a > 1.0f;
    if (inv) a = 1.0f / a;
    float base = 0.0f, t = a;
    if (a > kTanPi8) {
        t = (a - 1.0f) / (a + 1.0f);
        base = kPi4;
    }
    const float t2 = t * t;
    float poly = (float)(-1.0 / 19.0);
    poly = poly * t2 + (float)(1.0 / 17.0);
    poly = poly * t2 + (float)(-1.0 / 15.0);
    poly = poly * t2 + (float)(1.0 / 13.0);
    poly = poly * t2 + (float)(-1.0 / 11.0);
    poly = poly * t2 + (float)(1.0 / 9.0);
    poly = poly * t2 + (float)(-1.0 / 7.0);
    poly = poly * t2 + (float)(1.0 / 5.0);
    poly = poly * t2 + (float)(-1.0 / 3.0);
    poly = poly * t2 + 1.0f;
    float r = base + t * poly;
    if (inv) r = kPi2 - r;
    return neg ? -r : r;
}

// Neighbour direction k points from a source cell to its target; its angle
// is k*pi/4 counter-clockwise from east and rows grow southward, so
// (drow, dcol) = E(0,1) NE(-1,1) N(-1,0) NW(-1,-1) W(0,-1) SW(1,-1) S(1,0)
// SE(1,1).  kCos/kSin hold cos and sin of the angle rounded to fp32.
__device__ constexpr int kDRow[8] = {0, -1, -1, -1, 0, 1, 1, 1};
__device__ constexpr int kDCol[8] = {1, 1, 0, -1, -1, -1, 0, 1};
constexpr float kHalfSqrt2 = 0.70710678118654752440f;
__device__ constexpr float kCos[8] = {1.0f, kHalfSqrt2, 0.0f, -kHalfSqrt2,
                                      -1.0f, -kHalfSqrt2, 0.0f, kHalfSqrt2};
__device__ constexpr float kSin[8] = {0.0f, kHalfSqrt2, 1.0f, kHalfSqrt2,
                                      0.0f, -kHalfSqrt2, -1.0f, -kHalfSqrt2};

// Exponent of the wind factor (Eq. 1) for direction k at a source with
// wind (V, Vx, Vy): a_w1 V + a_w2 (V cos(angle_k - Theta) - V), with
// V cos(angle_k - Theta) = cos_k Vx + sin_k Vy.
__device__ __forceinline__ float wind_exponent(int k, float a_w1, float a_w2, float V, float Vx,
                                               float Vy)
{
    return a_w1 * V + a_w2 * ((kCos[k] * Vx + kSin[k] * Vy) - V);
}

}  // namespace firesim

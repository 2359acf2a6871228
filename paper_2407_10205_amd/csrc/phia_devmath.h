// Device-side elementary functions and the counter-based Gaussian stream of
// the PHIA sweep, gfx950.
//
// Every routine is a fixed sequence of IEEE binary32 operations (explicit
// __builtin_fmaf, correctly rounded division and square root, no hardware
// approximations such as v_exp_f32 or v_rcp_f32; '/' and sqrtf are the
// correctly rounded forms under HIP's default flags), so that its results are
// fully determined by the sequence and can be reproduced exactly by any other
// implementation of the same sequence.
//
//  * e^y (y <= 0): y = k ln2 + r with a two-part ln2, |r| <= ln2/2, Taylor
//    polynomial of degree 7 for e^r, exact scaling by 2^k; 0 below -80.
//  * ln u (u in (0,1)): u = m 2^e, m folded into (1/sqrt2, sqrt2],
//    ln m = 2 atanh((m-1)/(m+1)) by its series up to t^9/9.
//  * cos/sin(2 pi u): quarter-turn reduction u = k/4 + r, |r| <= 1/8, Taylor
//    series of sin to theta^9 and cos to theta^10, rotation by k quarter turns.
//  * sech^2(u) = 4 e^{-2|u|} / (1 + e^{-2|u|})^2, the factor
//    d tanh(gamma x)/dx / gamma of Eq. 8, with the reciprocal of 1 + e^{-2|u|}
//    from a linear start and three Newton steps (no division).
//  * Gaussians: Philox4x64-10 (Salmon et al., SC'11) keyed by (seed, 0) at
//    counter (i/8, round, replica, tag); word pair (i mod 8)/2 of the output
//    feeds a Box-Muller transform, cosine for even i, sine for odd i.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phia {

enum : uint32_t { kTagX = 0, kTagV = 1 };

#define PHIA_DEV __device__ __forceinline__

PHIA_DEV float bits_to_f(uint32_t b) { return __uint_as_float(b); }
PHIA_DEV uint32_t f_to_bits(float f) { return __float_as_uint(f); }

// ln 2 as the nearest float plus the nearest float to the remainder.
constexpr float kLn2Hi = 0.693147182464599609375f;
constexpr float kLn2Lo = -1.9046542999577e-09f;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kSqrt2 = 1.41421356237309504880f;
constexpr float kTwoPi = 6.28318530717958647692f;

// Branch-free: the polynomial is evaluated for every y and the result is
// replaced by 0 below -80 (or for NaN), so that several elements of a lane
// interleave without divergent branches; the values are those of the early
// return.
PHIA_DEV float dev_exp_nonpos(float y)
{
    const bool in_range = (y >= -80.0f);
    y = in_range ? y : 0.0f;
    const float k = __builtin_rintf(y * kLog2e);
    float r = __builtin_fmaf(-k, kLn2Hi, y);
    r = __builtin_fmaf(-k, kLn2Lo, r);
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 1.0f / 720.0f);
    p = __builtin_fmaf(p, r, 1.0f / 120.0f);
    p = __builtin_fmaf(p, r, 1.0f / 24.0f);
    p = __builtin_fmaf(p, r, 1.0f / 6.0f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    const int ki = static_cast<int>(k);
    const float e = p * bits_to_f(static_cast<uint32_t>(ki + 127) << 23);
    return in_range ? e : 0.0f;
}

PHIA_DEV float dev_ln_unit(float u)
{
    const uint32_t b = f_to_bits(u);
    int e = static_cast<int>((b >> 23) & 0xffu) - 127;
    float m = bits_to_f((b & 0x007fffffu) | 0x3f800000u);
    if (m > kSqrt2) {
        m = m * 0.5f;
        e += 1;
    }
    const float t = (m - 1.0f) / (m + 1.0f);
    const float t2 = t * t;
    float q = __builtin_fmaf(t2, 1.0f / 9.0f, 1.0f / 7.0f);
    q = __builtin_fmaf(q, t2, 1.0f / 5.0f);
    q = __builtin_fmaf(q, t2, 1.0f / 3.0f);
    const float tt = t + t;
    const float lnm = __builtin_fmaf(tt * t2, q, tt);
    const float ef = static_cast<float>(e);
    return __builtin_fmaf(ef, kLn2Hi, __builtin_fmaf(ef, kLn2Lo, lnm));
}

PHIA_DEV void dev_sincos_2pi(float u, float& c, float& s)
{
    const float k = __builtin_rintf(4.0f * u);
    const float r = __builtin_fmaf(k, -0.25f, u);
    const float th = r * kTwoPi;
    const float t2 = th * th;
    float ps = __builtin_fmaf(t2, 1.0f / 362880.0f, -(1.0f / 5040.0f));
    ps = __builtin_fmaf(ps, t2, 1.0f / 120.0f);
    ps = __builtin_fmaf(ps, t2, -(1.0f / 6.0f));
    const float sn = __builtin_fmaf(th * t2, ps, th);
    float pc = __builtin_fmaf(t2, -(1.0f / 3628800.0f), 1.0f / 40320.0f);
    pc = __builtin_fmaf(pc, t2, -(1.0f / 720.0f));
    pc = __builtin_fmaf(pc, t2, 1.0f / 24.0f);
    pc = __builtin_fmaf(pc, t2, -0.5f);
    const float cs = __builtin_fmaf(t2, pc, 1.0f);
    const int q = static_cast<int>(k) & 3;
    c = (q == 0) ? cs : (q == 1) ? -sn : (q == 2) ? -cs : sn;
    s = (q == 0) ? sn : (q == 1) ? cs : (q == 2) ? -sn : -cs;
}

// 1/(1+t) for t in (0, 1]: the line 24/17 - 8q/17 (relative error <= 1/17
// on q in [1, 2]) refined by three Newton steps y += y (1 - q y).
// sech^2 u = 4t / (1 + t)^2, t = e^{-2|u|}: the argument clamped at -80
// (so 4t stays normal), 4t from the exponential's sequence with the Taylor
// coefficients times 4 and ldexp as the scale, 1/(1 + t) from a quadratic
// first guess (relative error <= 1/99 on [1, 2]) and two Newton steps.
PHIA_DEV float dev_sech2(float u)
{
    const float a = __builtin_fabsf(u);
    const float y = __builtin_fmaxf(-(a + a), -80.0f);
    const float k = __builtin_rintf(y * kLog2e);
    float r = __builtin_fmaf(-k, kLn2Hi, y);
    r = __builtin_fmaf(-k, kLn2Lo, r);
    float p = 4.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 4.0f / 720.0f);
    p = __builtin_fmaf(p, r, 4.0f / 120.0f);
    p = __builtin_fmaf(p, r, 4.0f / 24.0f);
    p = __builtin_fmaf(p, r, 4.0f / 6.0f);
    p = __builtin_fmaf(p, r, 2.0f);
    p = __builtin_fmaf(p, r, 4.0f);
    p = __builtin_fmaf(p, r, 4.0f);
    const float t4 = __builtin_ldexpf(p, static_cast<int>(k));
    const float q = __builtin_fmaf(t4, 0.25f, 1.0f);
    float z = __builtin_fmaf(__builtin_fmaf(32.0f / 99.0f, q, -144.0f / 99.0f), q, 210.0f / 99.0f);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const float e = __builtin_fmaf(-q, z, 1.0f);
        z = __builtin_fmaf(z, e, z);
    }
    return t4 * (z * z);
}

// POLY2 mode: max(0, 1 - u^2 / 2.25) in place of sech^2 (t = u*u,
// q = fma(-t, 4/9, 1), d = q > 0 ? q : 0).
PHIA_DEV float dev_poly2(float u)
{
    const float t = u * u;
    const float q = __builtin_fmaf(-t, 4.0f / 9.0f, 1.0f);
    return q > 0.0f ? q : 0.0f;
}

PHIA_DEV float dev_uniform(uint32_t w)
{
    return static_cast<float>(2u * (w >> 9) + 1u) * 0x1p-24f;
}

// 64 x 64 -> 128-bit product.
PHIA_DEV void mul_wide(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
    lo = a * b;
    hi = __umul64hi(a, b);
}

struct u64x4 { uint64_t w[4]; };

PHIA_DEV u64x4 dev_philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1)
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        uint64_t h0, l0, h1, l1;
        mul_wide(M0, c0, h0, l0);
        mul_wide(M1, c2, h1, l1);
        const uint64_t n0 = h1 ^ c1 ^ k0;
        const uint64_t n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
        k0 += W0;
        k1 += W1;
    }
    return u64x4{{c0, c1, c2, c3}};
}

// Standard normal draw number i of the stream (seed, tag, replica, round).
PHIA_DEV float dev_gauss(uint64_t seed, uint32_t tag, uint64_t replica, uint64_t round, uint64_t i)
{
    const u64x4 o = dev_philox(i >> 3, round, replica, tag, seed, 0);
    const unsigned p = static_cast<unsigned>((i & 7u) >> 1);
    const uint64_t word = (p == 0) ? o.w[0] : (p == 1) ? o.w[1] : (p == 2) ? o.w[2] : o.w[3];
    const float ua = dev_uniform(static_cast<uint32_t>(word));
    const float ub = dev_uniform(static_cast<uint32_t>(word >> 32));
    const float rho = sqrtf(-2.0f * dev_ln_unit(ua));
    float c, s;
    dev_sincos_2pi(ub, c, s);
    return (i & 1u) ? rho * s : rho * c;
}

}  // namespace phia

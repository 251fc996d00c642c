// Device arithmetic of the hit simulation: counter-based random numbers,
// FP64 elementary functions for the per-(particle, layer) setup, the
// samplers, and the FP32 per-hit placement and cell lookup.
//
// Every quantity that decides a hit count or a cell index is evaluated with
// IEEE +, -, *, /, sqrt and floor only, in a fixed operation order and with
// floating-point contraction disabled, so that the result is reproducible
// bit for bit (the paper's Validation section traces its two CPU/GPU cell
// mismatches in 62M hits to rounding differences).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcsk {

// ---------------------------------------------------------------- Philox ---
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64 multiplies with a Weyl key schedule.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;  // one v_mad_u64_u32 each
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        const uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        // three-input xor in one v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint32_t y0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);
        const uint32_t y2 = __builtin_amdgcn_bitop3_b32(hi_a, c3, k1, 0x96);
        c0 = y0;
        c1 = lo_b;
        c2 = y2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// The same function for counters whose words 1-3 are wave-uniform (the hits
// of one task): in the first three rounds two of a round's three xor inputs
// are uniform, and they are combined first so that the scalar unit does that
// part; xor is associative, so the words are the same.
__device__ __forceinline__ U4 philox4x32_10_uniform_ctr(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t pb = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t hi_a = (uint32_t)(pa >> 32), lo_a = (uint32_t)pa;
        const uint32_t hi_b = (uint32_t)(pb >> 32), lo_b = (uint32_t)pb;
        uint32_t y0, y2;
        if (r == 0) {         // c1, c2, c3 uniform: y0 uniform
            y0 = hi_b ^ (c1 ^ k0);
            y2 = hi_a ^ (c3 ^ k1);
        } else if (r == 1) {  // c0, c1 uniform
            y0 = hi_b ^ (c1 ^ k0);
            y2 = c3 ^ (hi_a ^ k1);
        } else if (r == 2) {  // c3 uniform
            y0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);
            y2 = hi_a ^ (c3 ^ k1);
        } else {
            y0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);
            y2 = __builtin_amdgcn_bitop3_b32(hi_a, c3, k1, 0x96);
        }
        c0 = y0;
        c1 = lo_b;
        c2 = y2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// Counter words: (draw index, layer | stream tag << 8, particle in event,
// global event index).  Stream tags: 1 layer-energy Gamma, 2 hit-count
// Poisson, 3 per-hit draws.
enum : uint32_t { kTagGamma = 1u, kTagPoisson = 2u, kTagHit = 3u };

// (0,1) uniform of a 32-bit word for the FP64 setup draws
__device__ __forceinline__ double unit_open(uint32_t v) { return ((double)v + 0.5) * 0x1p-32; }
// [0, 1 - 2^-24] uniform with an exact 24-bit conversion, per-hit draws
__device__ __forceinline__ float unit24(uint32_t v) { return (float)(v >> 8) * 0x1p-24f; }

// ------------------------------------------------- FP64 own functions ---
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // 32 trailing zero bits
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kInvLn2 = 1.44269504088896338700e+00;

// The Horner steps of the series below are single-rounding fused
// multiply-adds (v_fma_f64).  The functions are templates on a copy tag
// only so that each setup kernel gets its own compiled copy (and register
// budget); the copies compute the same values.
//
// log for finite normal x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)),
// log m = 2 atanh(s) with s = (m-1)/(m+1), odd series to s^21
template <int kCopy>
__device__ __noinline__ double dlog(double x)
{
    const long long bits = __double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ff) - 1022;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3fe0000000000000LL);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double q = 1.0 / 21.0;
    q = __builtin_fma(q, z, 1.0 / 19.0);
    q = __builtin_fma(q, z, 1.0 / 17.0);
    q = __builtin_fma(q, z, 1.0 / 15.0);
    q = __builtin_fma(q, z, 1.0 / 13.0);
    q = __builtin_fma(q, z, 1.0 / 11.0);
    q = __builtin_fma(q, z, 1.0 / 9.0);
    q = __builtin_fma(q, z, 1.0 / 7.0);
    q = __builtin_fma(q, z, 1.0 / 5.0);
    q = __builtin_fma(q, z, 1.0 / 3.0);
    q = __builtin_fma(q, z, 1.0);
    const double ed = (double)e;
    return ed * kLn2Hi + (ed * kLn2Lo + (2.0 * s) * q);
}

// exp: x = k ln2 + r, Taylor series of e^r to r^13, times 2^k
template <int kCopy>
__device__ __noinline__ double dexp(double x)
{
    if (x < -708.0) return 0.0;
    if (x > 709.0) return __longlong_as_double(0x7ff0000000000000LL);
    const double k = floor(x * kInvLn2 + 0.5);
    const double r = (x - k * kLn2Hi) - k * kLn2Lo;
    double q = 1.0 / 6227020800.0;
    q = __builtin_fma(q, r, 1.0 / 479001600.0);
    q = __builtin_fma(q, r, 1.0 / 39916800.0);
    q = __builtin_fma(q, r, 1.0 / 3628800.0);
    q = __builtin_fma(q, r, 1.0 / 362880.0);
    q = __builtin_fma(q, r, 1.0 / 40320.0);
    q = __builtin_fma(q, r, 1.0 / 5040.0);
    q = __builtin_fma(q, r, 1.0 / 720.0);
    q = __builtin_fma(q, r, 1.0 / 120.0);
    q = __builtin_fma(q, r, 1.0 / 24.0);
    q = __builtin_fma(q, r, 1.0 / 6.0);
    q = __builtin_fma(q, r, 0.5);
    q = __builtin_fma(q, r, 1.0);
    q = __builtin_fma(q, r, 1.0);
    const int ki = (int)k;
    if (ki < -1000) {
        const double sc = __longlong_as_double((long long)(ki + 1000 + 1023) << 52);
        return (q * sc) * 0x1p-1000;
    }
    return q * __longlong_as_double((long long)(ki + 1023) << 52);
}

// cos(2 pi u): exact quarter-turn reduction, then a Taylor series of cos (to
// t^16) or sin (to t^17) on |t| <= pi/4; u in (0,1) for the normal draws and
// in [-1/4, 1) for the FP64 placement (a negative quadrant taken modulo 4)
template <int kCopy>
__device__ __noinline__ double dcos_turns(double u)
{
    const double qt = floor(4.0 * u + 0.5);
    const double f = u - 0.25 * qt;
    const double t = f * 6.28318530717958647692;
    const double z = t * t;
    const int quad = ((int)qt) & 3;
    if ((quad & 1) == 0) {
        double c = 1.0 / 20922789888000.0;
        c = __builtin_fma(c, z, -(1.0 / 87178291200.0));
        c = __builtin_fma(c, z, 1.0 / 479001600.0);
        c = __builtin_fma(c, z, -(1.0 / 3628800.0));
        c = __builtin_fma(c, z, 1.0 / 40320.0);
        c = __builtin_fma(c, z, -(1.0 / 720.0));
        c = __builtin_fma(c, z, 1.0 / 24.0);
        c = __builtin_fma(c, z, -(0.5));
        c = __builtin_fma(c, z, 1.0);
        return quad == 0 ? c : -c;
    }
    double s = 1.0 / 355687428096000.0;
    s = __builtin_fma(s, z, -(1.0 / 1307674368000.0));
    s = __builtin_fma(s, z, 1.0 / 6227020800.0);
    s = __builtin_fma(s, z, -(1.0 / 39916800.0));
    s = __builtin_fma(s, z, 1.0 / 362880.0);
    s = __builtin_fma(s, z, -(1.0 / 5040.0));
    s = __builtin_fma(s, z, 1.0 / 120.0);
    s = __builtin_fma(s, z, -(1.0 / 6.0));
    s = __builtin_fma(s, z, 1.0);
    s = t * s;
    return quad == 1 ? -s : s;
}

// log(k!): exact factorial below 10, Stirling series (to 1/(1260 x^5))
template <int kCopy>
__device__ __noinline__ double dlnfact(long long k)
{
    if (k < 10) {
        double f = 1.0;
        for (long long j = 2; j <= k; ++j) f = f * (double)j;
        return dlog<kCopy>(f);
    }
    const double x = (double)k + 1.0;
    const double ix = 1.0 / x;
    const double ix2 = ix * ix;
    const double corr = ix * (1.0 / 12.0 - ix2 * (1.0 / 360.0 - ix2 * (1.0 / 1260.0)));
    return (((x - 0.5) * dlog<kCopy>(x)) - x) + 0.91893853320467274178 + corr;
}

// ------------------------------------------------------------ samplers ---
// Gamma(alpha, 1): Marsaglia-Tsang acceptance test on a Box-Muller normal;
// for alpha < 1 the draw for alpha + 1 is scaled by u^(1/alpha).
//
// Attempt j (Philox counter (j, layer | 1 << 8, particle, event)) of the
// Marsaglia-Tsang method for Gamma(a), with d = a - 1/3 and c = 1/sqrt(9d):
// true and d v when the draw is accepted; *w is the draw's fourth word (the
// uniform of the alpha < 1 boost).  A task takes attempts j = 0, 1, ... up to
// 64 and then falls back to d.
template <int kCopy>
__device__ __forceinline__ bool gamma_try(double d, double c, uint32_t j, uint32_t k0, uint32_t k1,
                                          uint32_t layer, uint32_t part, uint32_t ev, double* g,
                                          uint32_t* w)
{
    const U4 x = philox4x32_10(j, layer | (kTagGamma << 8), part, ev, k0, k1);
    const double z = sqrt(-2.0 * dlog<kCopy>(unit_open(x.x))) * dcos_turns<kCopy>(unit_open(x.y));
    const double t = 1.0 + c * z;
    if (!(t > 0.0)) return false;
    const double v = (t * t) * t;
    const double lhs = dlog<kCopy>(unit_open(x.z));
    const double rhs = ((((0.5 * z) * z) + d) - d * v) + d * dlog<kCopy>(v);
    if (!(lhs < rhs)) return false;
    *g = d * v;
    *w = x.w;
    return true;
}

// the boost of an accepted draw for alpha < 1: Gamma(alpha) = Gamma(alpha + 1) u^(1/alpha)
template <int kCopy>
__device__ __forceinline__ double gamma_boost(double g, double alpha, uint32_t w)
{
    return alpha < 1.0 ? g * dexp<kCopy>(dlog<kCopy>(unit_open(w)) / alpha) : g;
}

// Poisson(mu): sequential inversion below mu = 10, transformed rejection
// (PTRS, Hoermann 1993) above with two attempts per Philox call.
// Call j uses counter (j, layer | 2 << 8, particle, event).
template <int kCopy>
__device__ __noinline__ long long poisson_draw(double mu, uint32_t k0, uint32_t k1, uint32_t layer,
                                               uint32_t part, uint32_t ev)
{
    if (mu < 10.0) {
        const U4 x = philox4x32_10(0u, layer | (kTagPoisson << 8), part, ev, k0, k1);
        const double u = unit_open(x.x);
        double pk = dexp<kCopy>(-mu);
        double cdf = pk;
        long long k = 0;
        while (u > cdf && k < 200) {
            k = k + 1;
            pk = (pk * mu) / (double)k;
            cdf = cdf + pk;
        }
        return k;
    }
    const double slam = sqrt(mu);
    const double loglam = dlog<kCopy>(mu);
    const double b = 0.931 + 2.53 * slam;
    const double a = -0.059 + 0.02483 * b;
    const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
    const double vr = 0.9277 - 3.6224 / (b - 2.0);
    const double log_ia = dlog<kCopy>(invalpha);
    for (uint32_t j = 0; j < 32; ++j) {
        const U4 x = philox4x32_10(j, layer | (kTagPoisson << 8), part, ev, k0, k1);
        for (int h = 0; h < 2; ++h) {
            const uint32_t wu = h == 0 ? x.x : x.z;
            const uint32_t wv = h == 0 ? x.y : x.w;
            const double U = unit_open(wu) - 0.5;
            const double V = unit_open(wv);
            const double us = 0.5 - fabs(U);
            const double kd = floor((((2.0 * a) / us + b) * U + mu) + 0.43);
            if (us >= 0.07 && V <= vr) return (long long)kd;
            if (kd < 0.0 || (us < 0.013 && V > us)) continue;
            const double lhs = (dlog<kCopy>(V) + log_ia) - dlog<kCopy>(a / (us * us) + b);
            const double rhs = (-mu + kd * loglam) - dlnfact<kCopy>((long long)kd);
            if (lhs <= rhs) return (long long)kd;
        }
    }
    return (long long)floor(mu);
}

// ------------------------------------------------ per-hit FP32 placement ---
// (cos, sin) of alpha = (ia + u) pi/4: even bins rotate forward from a
// multiple of pi/2 by d = u pi/4, odd bins back from the next multiple by
// d = (1-u) pi/4; the short polynomials below cover d in [0, pi/4].
__device__ __forceinline__ void sincos_bin(int ia, float u, float& cs, float& sn)
{
    const float quarter_pi = (float)(0.78539816339744830962);
    const bool even = (ia & 1) == 0;
    const float d = even ? u * quarter_pi : (1.0f - u) * quarter_pi;
    const int m = even ? (ia >> 1) : ((ia + 1) >> 1);
    const float d2 = d * d;
    // Horner steps as single-rounding fused multiply-adds (v_fma_f32)
    float sp = (float)(1.0 / 362880.0);
    sp = __builtin_fmaf(sp, d2, (float)(-1.0 / 5040.0));
    sp = __builtin_fmaf(sp, d2, (float)(1.0 / 120.0));
    sp = __builtin_fmaf(sp, d2, (float)(-1.0 / 6.0));
    sp = __builtin_fmaf(sp, d2, 1.0f);
    const float s0 = d * sp;
    float cp = (float)(-1.0 / 3628800.0);
    cp = __builtin_fmaf(cp, d2, (float)(1.0 / 40320.0));
    cp = __builtin_fmaf(cp, d2, (float)(-1.0 / 720.0));
    cp = __builtin_fmaf(cp, d2, (float)(1.0 / 24.0));
    cp = __builtin_fmaf(cp, d2, -0.5f);
    cp = __builtin_fmaf(cp, d2, 1.0f);
    const float c0 = cp;
    // quadrant table: even bins  m=0:(c,s) 1:(-s,c) 2:(-c,-s) 3:(s,-c)
    //                 odd bins   m=1:(s,c) 2:(-c,s) 3:(-s,-c) 4:(c,-s)
    // i.e. a rotation by q = m mod 4 quarter turns of (c0, +-s0), with the
    // sine negated for odd bins.  Selected without branches: a swap for odd
    // q, then sign flips (exact) for the negated entries.
    const int q = m & 3;
    const float s1 = __int_as_float(__float_as_int(s0) ^ ((ia & 1) << 31));
    const bool swap = (q & 1) != 0;
    const float a = swap ? s1 : c0;
    const float b = swap ? c0 : s1;
    const float c = __int_as_float(__float_as_int(a) ^ (((q ^ (q >> 1)) & 1) << 31));
    const float s = __int_as_float(__float_as_int(b) ^ ((q & 2) << 30));
    cs = c;
    sn = s;
}

}  // namespace fcsk

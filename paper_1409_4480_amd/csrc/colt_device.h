// Device building blocks of the Lyman-alpha transport: counter-based random
// numbers, H(a,x), x_cw, and the scattering samplers, in FP64 or FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "colt_internal.h"

namespace colt {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products,
// a word swap and a xor with the round key; the key advances by the Weyl
// constants after every round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                              uint32_t &c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input xor in one instruction (bit function 0x96 of gfx950's bitop3)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Per-photon stream: uniform k of photon `id` under key `seed` comes from
// counter block (k / per_block) of the photon's counter space.  FP64 takes 53
// bits from a word pair (two draws per block); FP32 takes one word per draw
// (four per block).  The last block's unused words are cached in registers.
// The u_par sampler starts on a fresh block and addresses its blocks directly.
__device__ __forceinline__ double u53(uint32_t lo, uint32_t hi)
{
    const uint64_t m = ((((uint64_t)hi) << 32) | lo) >> 11;
    return ((double)m + 1.0) * 0x1.0p-53;
}

__device__ __forceinline__ float u32f(uint32_t w)
{
    // (0, 1]: w 2^-32 + 2^-33, rounded to float
    return __builtin_fmaf((float)w, 0x1.0p-32f, 0x1.0p-33f);
}

struct RngKey {
    uint32_t key0, key1, id0, id1;
    __device__ __forceinline__ void block(uint64_t b, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                          uint32_t &w3) const
    {
        uint32_t c0 = (uint32_t)b, c1 = (uint32_t)(b >> 32), c2 = id0, c3 = id1;
        philox4x32_10(c0, c1, c2, c3, key0, key1);
        w0 = c0; w1 = c1; w2 = c2; w3 = c3;
    }
    // blocks b and b + 1 as two independent chains, so that their rounds
    // overlap instead of following each other
    __device__ __forceinline__ void block2(uint64_t b, uint32_t a[4], uint32_t c[4]) const
    {
        const uint64_t b1 = b + 1;
        a[0] = (uint32_t)b; a[1] = (uint32_t)(b >> 32); a[2] = id0; a[3] = id1;
        c[0] = (uint32_t)b1; c[1] = (uint32_t)(b1 >> 32); c[2] = id0; c[3] = id1;
        uint32_t k0 = key0, k1 = key1;
#pragma unroll
        for (int i = 0; i < 10; ++i) {
            const uint64_t pa0 = (uint64_t)0xD2511F53u * a[0], pa1 = (uint64_t)0xCD9E8D57u * a[2];
            const uint64_t pc0 = (uint64_t)0xD2511F53u * c[0], pc1 = (uint64_t)0xCD9E8D57u * c[2];
            const uint32_t na0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa1 >> 32), a[1], k0, 0x96);
            const uint32_t na2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa0 >> 32), a[3], k1, 0x96);
            const uint32_t nc0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pc1 >> 32), c[1], k0, 0x96);
            const uint32_t nc2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pc0 >> 32), c[3], k1, 0x96);
            a[1] = (uint32_t)pa1; a[3] = (uint32_t)pa0; a[0] = na0; a[2] = na2;
            c[1] = (uint32_t)pc1; c[3] = (uint32_t)pc0; c[0] = nc0; c[2] = nc2;
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
    }
};

template <typename R>
struct Rng;

template <>
struct Rng<double> {
    static constexpr int kPerBlock = 2;
    RngKey key;
    uint64_t k;
    uint32_t w2, w3;
    __device__ void init(uint64_t seed, uint64_t id)
    {
        key.key0 = (uint32_t)seed; key.key1 = (uint32_t)(seed >> 32);
        key.id0 = (uint32_t)id; key.id1 = (uint32_t)(id >> 32);
        k = 0;
    }
    __device__ __forceinline__ double next()
    {
        uint32_t lo, hi;
        if ((k & 1) == 0) {
            key.block(k >> 1, lo, hi, w2, w3);
        } else {
            lo = w2; hi = w3;
        }
        ++k;
        return u53(lo, hi);
    }
    // moves to the start of the next unused block; returns that block
    __device__ __forceinline__ uint64_t align()
    {
        k = (k + 1) & ~(uint64_t)1;
        return k >> 1;
    }
    // continues the stream at draw index k0 (a suspended photon): the words of
    // a partly used block are recomputed
    __device__ __forceinline__ void restore(uint64_t k0)
    {
        k = k0;
        if (k & 1) {
            uint32_t lo, hi;
            key.block(k >> 1, lo, hi, w2, w3);
        }
    }
};

template <>
struct Rng<float> {
    static constexpr int kPerBlock = 4;
    RngKey key;
    uint64_t k;
    uint32_t w1, w2, w3;
    __device__ void init(uint64_t seed, uint64_t id)
    {
        key.key0 = (uint32_t)seed; key.key1 = (uint32_t)(seed >> 32);
        key.id0 = (uint32_t)id; key.id1 = (uint32_t)(id >> 32);
        k = 0;
    }
    // the unused words of the current block wait in w1, w2, w3 (oldest first);
    // shifting them keeps every access static so the state stays in registers
    __device__ __forceinline__ float next()
    {
        uint32_t w;
        if (((uint32_t)k & 3u) == 0) {
            key.block(k >> 2, w, w1, w2, w3);
        } else {
            w = w1;
            w1 = w2;
            w2 = w3;
        }
        ++k;
        return u32f(w);
    }
    // the next five draws; from a block boundary the two blocks they span are
    // generated together and the second one's last three words stay cached
    __device__ __forceinline__ void next5(float u[5])
    {
        if (((uint32_t)k & 3u) == 0) {
            uint32_t a[4], c[4];
            key.block2(k >> 2, a, c);
#pragma unroll
            for (int i = 0; i < 4; ++i) u[i] = u32f(a[i]);
            u[4] = u32f(c[0]);
            w1 = c[1]; w2 = c[2]; w3 = c[3];
            k += 5;
        } else {
#pragma unroll
            for (int i = 0; i < 5; ++i) u[i] = next();
        }
    }
    __device__ __forceinline__ uint64_t align()
    {
        k = (k + 3) & ~(uint64_t)3;
        return k >> 2;
    }
    // continues the stream at draw index k0: at position m = k0 mod 4 of a
    // block the cache holds its words m, m+1, m+2 (those that exist)
    __device__ __forceinline__ void restore(uint64_t k0)
    {
        k = k0;
        const uint32_t m = (uint32_t)k & 3u;
        if (m) {
            uint32_t w[4];
            key.block(k >> 2, w[0], w[1], w[2], w[3]);
            w1 = (m == 1) ? w[1] : ((m == 2) ? w[2] : w[3]);
            w2 = (m == 1) ? w[2] : w[3];
            w3 = w[3];
        }
    }
};

// ---------------------------------------------------------------------------
// Elementary functions per precision.  FP64 uses the correctly-behaved double
// library functions; FP32 uses the hardware transcendental units (exp2, log2,
// sin/cos of revolutions).
// ---------------------------------------------------------------------------
template <typename R>
struct Fn;

template <>
struct Fn<double> {
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
    static __device__ __forceinline__ double cbrt(double x) { return ::cbrt(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    static __device__ __forceinline__ double atan(double x) { return ::atan(x); }
    static __device__ __forceinline__ double tan(double x) { return ::tan(x); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    // cos and sin of 2 pi R
    static __device__ __forceinline__ void cossin2pi(double R, double &c, double &s)
    {
        const double ang = 2.0 * kPi * R;
        c = ::cos(ang);
        s = ::sin(ang);
    }
};

template <>
struct Fn<float> {
    static __device__ __forceinline__ float exp(float x)
    {
        return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
    }
    static __device__ __forceinline__ float log(float x)
    {
        return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
    }
    // the square-root unit alone (about 1 ulp; the correctly rounded sqrtf
    // wraps it in a scaling and two-sided correction, ~6x its latency)
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    // x >= 0: 2^(log2(x) / 3) on the transcendental unit (a few ulp)
    static __device__ __forceinline__ float cbrt(float x)
    {
        return __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
    }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float atan(float x) { return ::atanf(x); }
    static __device__ __forceinline__ float div(float a, float b)
    {
        return a * __builtin_amdgcn_rcpf(b);
    }
    static __device__ __forceinline__ void cossin2pi(float R, float &c, float &s)
    {
        c = __builtin_amdgcn_cosf(R);
        s = __builtin_amdgcn_sinf(R);
    }
};

// ---------------------------------------------------------------------------
// H(a, x) to first order in a, three regions in z = x^2 with the continued
// fractions and coefficients of the paper's appendix (eq. AB, table AB).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R voigt_H(R a, R x)
{
    using F = Fn<R>;
    const R z = x * x;
    if (z <= R(3)) {
        const R cf = F::div(R(286.9341762324778),
                            z - R(19.05706700907019) +
                                F::div(R(28.22644017233441),
                                       z - R(9.526399802414186) +
                                           F::div(R(35.29217026286130),
                                                  z - R(0.8681020834678775))));
        return F::exp(-z) * (R(1) - a * (R(15.75328153963877) + cf));
    } else if (z < R(25)) {
        const R cf = F::div(
            R(0.5403095364583999),
            z - R(2.676724102580895) +
                F::div(R(12.82026082606220),
                       z + R(3.21166435627278) +
                           F::div(R(32.032981933420),
                                  z - R(9.0328158696) +
                                      F::div(R(23.7489999060), z - R(1.82106170570)))));
        return F::exp(-z) + a * (R(0.0003300469163682737) + cf);
    } else {
        return F::div(F::div(a, R(kSqrtPi)),
                      z - R(1.5) - F::div(R(1.5), z - R(3.5) - F::div(R(5), z - R(5.5))));
    }
}

// ---------------------------------------------------------------------------
// Parallel atom velocity u_par from f(u) ~ exp(-u^2)/(a^2+(x-u)^2)
// (Sec. 3.2.3): Lorentzian proposal for |x| <= 1; two-part comparison
// function split at u0 for 1 < |x| < 9 (u0,core below x_cw, u0,wing above),
// redrawing the part after each rejection; Gaussian of mean 1/x for |x| >= 9.
//
// Draw layout: the sampler starts on a fresh counter block B0.  Candidate t
// uses block B0 + t (FP32: words part, theta, accept; FP64 |x| <= 1: theta,
// accept) or blocks B0 + 2t, B0 + 2t + 1 (FP64 two-part: part, theta, accept
// from the first three word pairs).  Because a candidate's draws depend only
// on (photon, t), candidates can be evaluated in any order or in parallel and
// the first accepted one in t-order is the sequential result.
//
// The FP64 form follows the paper's expressions literally; the FP32 form
// evaluates the same quantities through phi = theta + pi/2, which keeps the
// angles near -pi/2 accurate in single precision.
// ---------------------------------------------------------------------------
enum { UPAR_CORE = 0, UPAR_SPLIT = 1, UPAR_GAUSS = 2 };

template <typename R>
struct UparReq {
    R X;          // |x|
    R a;
    R u0;         // split point (two-part regime)
    R p;          // probability of the part below u0
    R th0;        // FP64: theta0; FP32: phi0 = theta0 + pi/2
    int regime;
    // FP32 only, fixed per request: the first word's split point p 2^32 and
    // the reciprocal widths of the two parts' word ranges (the core regime is
    // the lower part over all words, with phi0 = pi)
    uint32_t wp;
    float inv_lo, inv_hi;
};

template <typename R>
__device__ __forceinline__ UparReq<R> upar_setup(R a, R x, R xcw)
{
    using F = Fn<R>;
    UparReq<R> q;
    q.X = (x < R(0)) ? -x : x;
    q.a = a;
    q.u0 = R(0);
    q.p = R(0);
    q.th0 = R(0);
    q.wp = 0xFFFFFFFFu;
    q.inv_lo = 0x1.0p-32f;
    q.inv_hi = 1.0f;
    q.regime = (q.X <= R(1)) ? UPAR_CORE : ((q.X < R(9)) ? UPAR_SPLIT : UPAR_GAUSS);
    if constexpr (sizeof(R) == 4) {
        if (q.regime == UPAR_CORE) q.th0 = float(kPi);
    }
    if (q.regime == UPAR_SPLIT) {
        const R X = q.X;
        R u0;
        if (X < xcw)
            u0 = X - F::div(R(1), X + F::div(F::exp(R(1) - X * X), a));
        else
            u0 = xcw - F::div(R(1), xcw) + R(0.15) * (X - xcw);
        const R e0 = F::exp(-u0 * u0);
        q.u0 = u0;
        if constexpr (sizeof(R) == 8) {
            const double theta0 = ::atan((u0 - X) / a);
            q.th0 = theta0;
            q.p = (theta0 + kPi / 2.0) / ((1.0 - e0) * theta0 + (1.0 + e0) * kPi / 2.0);
        } else {
            const float phi0 = F::atan(F::div(a, X - u0));
            q.th0 = phi0;
            q.p = F::div(phi0, phi0 + e0 * (float(kPi) - phi0));
            q.wp = (q.p >= 1.0f) ? 0xFFFFFFFFu : (uint32_t)(q.p * 4294967296.0f);
            q.inv_lo = __builtin_amdgcn_rcpf((float)q.wp);
            q.inv_hi = __builtin_amdgcn_rcpf((float)(0u - q.wp));
        }
    }
    return q;
}

// Advance of the draw index once candidate t (counted from 0) is accepted.
// FP64: a core candidate takes one block (two draws), a two-part candidate
// two blocks (four draws, the last unused).  FP32: two candidates share a
// block (two words each) and the stream resumes at the next fresh block.
template <typename R>
__device__ __forceinline__ uint64_t upar_advance(int regime, uint32_t t)
{
    if constexpr (sizeof(R) == 8) return (uint64_t)((regime == UPAR_SPLIT) ? 4u : 2u) * (t + 1);
    return 4ull * (t / 2 + 1);
}

// FP32 candidate from two words.  Core: theta = pi (R - 1/2) from the first,
// acceptance draw from the second.  Two-part: the first word both picks the
// part (probability p for the lower one) and, rescaled within the chosen
// part's range of words, places theta in that part; the rescaled value is
// uniform and independent of the choice.  The rescaling is done on the
// integer word so that it keeps full precision however small either part's
// share is.  The second word is the acceptance draw.
__device__ __forceinline__ bool upar_eval_fp32(const UparReq<float> &q, uint32_t wa,
                                               uint32_t wb, float &u)
{
    using F = Fn<float>;
    // one branch-free form for both regimes: a core request is the lower part
    // over all words (wp = 2^32 - 1, width 2^-32, phi0 = pi), which gives
    // phi = pi (R - 1/2) + pi/2 with R = u32f(wa) exactly
    const bool lower = wa < q.wp;
    const float Rth = ((float)(lower ? wa : wa - q.wp) + 0.5f) * (lower ? q.inv_lo : q.inv_hi);
    const float phi = lower ? Rth * q.th0 : q.th0 + Rth * (float(kPi) - q.th0);
    const float bias = lower ? 0.0f : q.u0 * q.u0;
    float c, s;
    F::cossin2pi(phi * float(0.5 / kPi), c, s);
    u = q.X - q.a * F::div(c, s);               // a tan(phi - pi/2) = -a cot(phi)
    return u32f(wb) < F::exp(bias - u * u);
}

// FP32: both candidates 2b and 2b+1 of one block; returns whether either is
// accepted, with the first accepted one in u and its position (0, 1) in half.
__device__ __forceinline__ bool upar_pair_fp32(const UparReq<float> &q, const RngKey &key,
                                               uint64_t B0, uint32_t b, float &u,
                                               uint32_t &half)
{
    uint32_t w0, w1, w2, w3;
    key.block(B0 + b, w0, w1, w2, w3);
    float u0, u1;
    const bool a0 = upar_eval_fp32(q, w0, w1, u0);
    const bool a1 = upar_eval_fp32(q, w2, w3, u1);
    u = a0 ? u0 : u1;
    half = a0 ? 0u : 1u;
    return a0 || a1;
}

// Candidate t of request q (unsigned |u|) from the photon's blocks starting at B0.
template <typename R>
__device__ __forceinline__ bool upar_candidate(const UparReq<R> &q, const RngKey &key,
                                               uint64_t B0, uint32_t t, R &u)
{
    uint32_t w0, w1, w2, w3;
    if constexpr (sizeof(R) == 8) {
        if (q.regime == UPAR_CORE) {
            key.block(B0 + t, w0, w1, w2, w3);
            const double theta = kPi * (u53(w0, w1) - 0.5);
            u = q.a * ::tan(theta) + q.X;
            return u53(w2, w3) < ::exp(-u * u);
        }
        key.block(B0 + 2ull * t, w0, w1, w2, w3);
        const double Rp = u53(w0, w1), Rth = u53(w2, w3);
        key.block(B0 + 2ull * t + 1, w0, w1, w2, w3);
        const double Racc = u53(w0, w1);
        double acc;
        if (Rp <= q.p) {
            const double theta = -kPi / 2.0 + Rth * (q.th0 + kPi / 2.0);
            u = q.a * ::tan(theta) + q.X;
            acc = ::exp(-u * u);
        } else {
            const double theta = q.th0 + Rth * (kPi / 2.0 - q.th0);
            u = q.a * ::tan(theta) + q.X;
            acc = ::exp(q.u0 * q.u0 - u * u);
        }
        return Racc < acc;
    } else {
        key.block(B0 + t / 2, w0, w1, w2, w3);
        return (t & 1) ? upar_eval_fp32(q, w2, w3, u) : upar_eval_fp32(q, w0, w1, u);
    }
}

// |x| >= 9: Gaussian of mean 1/|x| (variance 1/2) from one block.
template <typename R>
__device__ __forceinline__ R upar_gauss(const UparReq<R> &q, const RngKey &key, uint64_t B0)
{
    using F = Fn<R>;
    uint32_t w0, w1, w2, w3;
    key.block(B0, w0, w1, w2, w3);
    R R1, R2;
    if constexpr (sizeof(R) == 8) {
        R1 = u53(w0, w1);
        R2 = u53(w2, w3);
    } else {
        R1 = u32f(w0);
        R2 = u32f(w1);
    }
    R c, s;
    F::cossin2pi(R2, c, s);
    return F::div(R(1), q.X) + F::sqrt(-F::log(R1)) * c;
}

// Sequential sampler (one lane): signed u_par; advances the stream past the
// accepted candidate and counts candidates in `tries`.
template <typename R>
__device__ __forceinline__ R draw_upar(R a, R x, R xcw, Rng<R> &rng, uint32_t &tries)
{
    const UparReq<R> q = upar_setup<R>(a, x, xcw);
    const R sgn = (x < R(0)) ? R(-1) : R(1);
    const uint64_t B0 = rng.align();
    R u;
    if (q.regime == UPAR_GAUSS) {
        u = upar_gauss<R>(q, rng.key, B0);
        rng.k += Rng<R>::kPerBlock;
        return sgn * u;
    }
    uint32_t t = 0;
    while (!upar_candidate<R>(q, rng.key, B0, t, u)) ++t;
    tries += t + 1;
    rng.k += upar_advance<R>(q.regime, t);
    return sgn * u;
}

// Perpendicular components: Box-Muller on exp(-u^2)/sqrt(pi), truncated below
// the core-skipping frequency (Sec. 3.2.4).
template <typename R>
__device__ __forceinline__ void draw_uperp_from(R xc, R R1, R R2, R &u1, R &u2)
{
    using F = Fn<R>;
    const R rho = F::sqrt(xc * xc - F::log(R1));
    R c, s;
    F::cossin2pi(R2, c, s);
    u1 = rho * c;
    u2 = rho * s;
}

template <typename R>
__device__ __forceinline__ void draw_uperp(R xc, Rng<R> &rng, R &u1, R &u2)
{
    const R R1 = rng.next();
    const R R2 = rng.next();
    draw_uperp_from<R>(xc, R1, R2, u1, u2);
}

// Cosine of the scattering angle for W(mu) ~ 1 + rW mu^2 (eq. phaseW) by
// inverting its cubic CDF with Cardano's formula.
template <typename R>
__device__ __forceinline__ R draw_mu_from(R rW, R Rm)
{
    using F = Fn<R>;
    if (rW == R(0)) return R(2) * Rm - R(1);
    const R p = F::div(R(3), rW);
    const R q = (R(1) + p) * (R(1) - R(2) * Rm);
    const R D = R(0.25) * q * q + F::div(p * p * p, R(27));
    const R aq = (q < R(0)) ? -q : q;
    R c = F::cbrt(R(0.5) * aq + F::sqrt(D));
    if (q > R(0)) c = -c;
    R mu = c - F::div(p, R(3) * c);
    mu = (mu > R(1)) ? R(1) : mu;
    mu = (mu < R(-1)) ? R(-1) : mu;
    return mu;
}

template <typename R>
__device__ __forceinline__ R draw_mu(R rW, Rng<R> &rng)
{
    const R Rm = rng.next();
    return draw_mu_from<R>(rW, Rm);
}

// Orthonormal e1, e2 perpendicular to unit k: e1 ~ k x z (k x x when |k_z| > 0.9).
template <typename R>
__device__ __forceinline__ void perp_basis(const R k[3], R e1[3], R e2[3])
{
    using F = Fn<R>;
    const R kz = (k[2] < R(0)) ? -k[2] : k[2];
    if constexpr (sizeof(R) == 4) {
        // without branches: e1 = (a, -b, 0) or (0, a, -b), scaled by 1/|(a, b)|
        const bool zax = kz <= R(0.9);
        const R a = zax ? k[1] : k[2], b = zax ? k[0] : k[1];
        const R inv = F::rsqrt(a * a + b * b);
        const R ea = a * inv, eb = -b * inv;
        e1[0] = zax ? ea : R(0);
        e1[1] = zax ? eb : ea;
        e1[2] = zax ? R(0) : eb;
    } else if (kz <= R(0.9)) {
        const R n = F::sqrt(k[0] * k[0] + k[1] * k[1]);
        e1[0] = F::div(k[1], n); e1[1] = F::div(-k[0], n); e1[2] = R(0);
    } else {
        const R n = F::sqrt(k[1] * k[1] + k[2] * k[2]);
        e1[0] = R(0); e1[1] = F::div(k[2], n); e1[2] = F::div(-k[1], n);
    }
    e2[0] = k[1] * e1[2] - k[2] * e1[1];
    e2[1] = k[2] * e1[0] - k[0] * e1[2];
    e2[2] = k[0] * e1[1] - k[1] * e1[0];
}

template <typename R>
__device__ __forceinline__ R xcrit_of(R atau0)
{
    return (atau0 < R(1)) ? R(0) : Fn<R>::div(Fn<R>::cbrt(atau0), R(5));
}

}  // namespace colt

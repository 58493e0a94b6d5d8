// Device helpers of librbsog: the counter-based generator and the elementary
// functions of the force kernels, written for gfx950.
//
// The functions here are specialised to the arguments the kernels produce:
// exponentials of non-positive arguments (Gaussians and the screened factor)
// and sines/cosines of phases given in revolutions.  Both use polynomials on
// a reduced range whose truncation error is well below half an ulp, and no
// special-case branches (no overflow is possible; a very negative argument
// underflows to zero through ldexp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rbsog {

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the published multipliers, Weyl-sequence key
// schedule (golden-ratio and sqrt(3)-1 increments) applied between rounds.
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                     uint64_t out[4])
{
    const uint64_t mA = 0xD2E7470EE14C6C93ull, mB = 0xCA5A826395121157ull;
    const uint64_t wA = 0x9E3779B97F4A7C15ull, wB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hA = __umul64hi(mA, c0), lA = mA * c0;
        uint64_t hB = __umul64hi(mB, c2), lB = mB * c2;
        uint64_t n0 = hB ^ c1 ^ k0, n2 = hA ^ c3 ^ k1;
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += wA;
        k1 += wB;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// ---------------------------------------------------------------------------
// Taylor coefficients.  They are built at compile time on the host and handed
// to the kernels in their argument blocks, so they sit in scalar registers and
// each Horner step is a single FMA with a scalar operand.
// ---------------------------------------------------------------------------

constexpr double kLn2 = 0.6931471805599453;     // ln 2 rounded to FP64
constexpr double kTwoPi = 6.283185307179586;    // 2 pi rounded to FP64
constexpr double kLog2e = 1.4426950408889634;   // 1 / ln 2 rounded to FP64

// a^k / k!
constexpr double taylor_coef(double a, int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * a / (double)i;
    return c;
}

// 2^f for |f| <= 1/2: the degree-11 Chebyshev economization of its Taylor
// series (gen_exp2_poly.py beside this file derives the coefficients in exact
// arithmetic; the dropped terms are below 3.2e-18 and the coefficients as
// rounded to FP64 are within 0.17 ulp of 2^f over the interval).
struct Exp2Poly {
    double c[12];
};
constexpr Exp2Poly make_exp2_poly()
{
    return Exp2Poly{{0x1.0000000000000p+0, 0x1.62e42fefa39efp-1, 0x1.ebfbdff82c5aep-3, 0x1.c6b08d704a0d1p-5,
                     0x1.3b2ab6fb9f1a3p-7, 0x1.5d87fe78a2292p-10, 0x1.430913112cb56p-13, 0x1.ffcbfc75f302dp-17,
                     0x1.62bfc2c7ae40ep-20, 0x1.b524db38fd1f9p-24, 0x1.e6228bff026d1p-28, 0x1.ea044321bc0aap-32}};
}

// sin(2 pi f) = f sum_k s[k] f^(2k), s[k] = (-1)^k (2 pi)^(2k+1)/(2k+1)!, k = 0..8
// cos(2 pi f) = sum_k c[k] f^(2k),    c[k] = (-1)^k (2 pi)^(2k)/(2k)!,     k = 0..8
// For |f| <= 1/8 (|2 pi f| <= pi/4) the first omitted terms are below 2.1e-18.
struct SinCosPoly {
    double s[9];
    double c[9];
};
constexpr SinCosPoly make_sincos_poly()
{
    SinCosPoly p{};
    for (int k = 0; k < 9; ++k) {
        double sg = (k % 2) ? -1.0 : 1.0;
        p.s[k] = sg * taylor_coef(kTwoPi, 2 * k + 1);
        p.c[k] = sg * taylor_coef(kTwoPi, 2 * k);
    }
    return p;
}

// 2^y for finite y <= 0 (FP64): 2^y = 2^n 2^f with n = rint(y), f = y - n exact.
__device__ inline double exp2_nonpos(double y, const Exp2Poly &P)
{
    double n = rint(y);
    double f = y - n;
    double p = P.c[11];
#pragma unroll
    for (int k = 10; k >= 0; --k) p = fma(p, f, P.c[k]);
    return ldexp(p, (int)n);
}

// sin(2 pi u), cos(2 pi u) for a phase u in revolutions (FP64).  The integer
// and quarter-turn parts are removed exactly (u - rint(u) and r - q/4 are
// exact in FP64), leaving f in [-1/8, 1/8]; the quarter turn q rotates the
// result.
__device__ inline void sincos_rev(double u, const SinCosPoly &P, double *s, double *c)
{
    double r = u - rint(u);
    double q = rint(4.0 * r);
    double f = fma(-0.25, q, r);
    double f2 = f * f;
    double sp = P.s[8], cp = P.c[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) {
        sp = fma(sp, f2, P.s[k]);
        cp = fma(cp, f2, P.c[k]);
    }
    double sn = sp * f;
    // rotate by q quarter turns, q in {-2, -1, 0, 1, 2}
    int qi = (int)q & 3;
    double s1 = (qi & 1) ? cp : sn;
    double c1 = (qi & 1) ? sn : cp;
    *s = (qi & 2) ? -s1 : s1;
    *c = ((qi + 1) & 2) ? -c1 : c1;
}

constexpr int kPhaseTab = 128;   // entries of the rotation table

// sin(2 pi f / 128), cos(2 pi f / 128) for |f| <= 1/2 (f in 1/128 revolutions)
// by their Taylor series to degree 7 and 6 (s[k] = (-1)^k a^(2k+1)/(2k+1)!,
// c[k] = (-1)^k a^(2k)/(2k)!, a = 2 pi / 128): the first omitted terms are below
// 4e-19 relative to sin and 4e-18 absolute.
struct SinCosShort {
    double s[4];
    double c[4];
};
constexpr SinCosShort make_sincos_short()
{
    SinCosShort p{};
    for (int k = 0; k < 4; ++k) {
        double sg = (k % 2) ? -1.0 : 1.0;
        p.s[k] = sg * taylor_coef(kTwoPi / kPhaseTab, 2 * k + 1);
        p.c[k] = sg * taylor_coef(kTwoPi / kPhaseTab, 2 * k);
    }
    return p;
}


// sin(2 pi w / 128), cos(2 pi w / 128) for a phase w in 1/128 revolutions
// (FP64; the callers scale positions by 128 / L, exactly) with a table of
// (sin, cos)(2 pi j / 128): w = m + f exactly with m = rint(w) and |f| <= 1/2
// (for |w| < 2^52 the difference is exact), the short series give the rotation
// by f and the table entry of m mod 128 (in LDS) the rest.
__device__ inline void sincos_rev_tab(double w, const double2 *tab, const SinCosShort &P, double *s, double *c)
{
    double jr = rint(w);
    double f = w - jr;
    double2 t = tab[(int)jr & (kPhaseTab - 1)];
    double f2 = f * f;
    double sp = fma(fma(fma(P.s[3], f2, P.s[2]), f2, P.s[1]), f2, P.s[0]) * f;
    double cp = fma(fma(fma(P.c[3], f2, P.c[2]), f2, P.c[1]), f2, P.c[0]);
    *s = fma(t.x, cp, t.y * sp);
    *c = fma(t.y, cp, -(t.x * sp));
}

// The far field's finer table: 1024 entries (16 KB of LDS, which only the far
// kernel carries), so that the remainder |f| <= 1/2 in 1/1024 revolutions is
// at most pi/1024 rad and degree-5/4 series suffice (first omitted terms below
// 6e-22 relative to sin and 2e-18 absolute for cos): two FMA fewer per
// (particle, mode) than the 128-entry form.
constexpr int kFarTab = 1024;
struct SinCosFar {
    double s[3];
    double c[3];
};
constexpr SinCosFar make_sincos_far()
{
    SinCosFar p{};
    for (int k = 0; k < 3; ++k) {
        double sg = (k % 2) ? -1.0 : 1.0;
        p.s[k] = sg * taylor_coef(kTwoPi / kFarTab, 2 * k + 1);
        p.c[k] = sg * taylor_coef(kTwoPi / kFarTab, 2 * k);
    }
    return p;
}

// sin and cos of 2 pi w / 1024 for a phase w in 1/1024 revolutions, as
// sincos_rev_tab with the far field's table
__device__ inline void sincos_rev_far(double w, const double2 *tab, const SinCosFar &P, double *s, double *c)
{
    double jr = rint(w);
    double f = w - jr;
    double2 t = tab[(int)jr & (kFarTab - 1)];
    double f2 = f * f;
    double sp = fma(fma(P.s[2], f2, P.s[1]), f2, P.s[0]) * f;
    double cp = fma(fma(P.c[2], f2, P.c[1]), f2, P.c[0]);
    *s = fma(t.x, cp, t.y * sp);
    *c = fma(t.y, cp, -(t.x * sp));
}

// The same in FP32 after the exact FP64 reduction to [-1/2, 1/2] revolutions:
// the hardware sine and cosine take their argument in revolutions.
__device__ inline void sincos_rev_f32(double u, float *s, float *c)
{
    float r = (float)(u - rint(u));
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}

// Workgroup index remapped so that consecutive logical indices run on the same
// XCD (the hardware deals workgroups to the 8 XCDs round-robin; each XCD has
// its own L2, so spatially adjacent work should share one).
__device__ inline int xcd_block(int b, int nb)
{
    const int nx = 8;
    int x = b % nx, k = b / nx;
    int q = nb / nx, r = nb % nx;
    return x * q + min(x, r) + k;
}

}  // namespace rbsog

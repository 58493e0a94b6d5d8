// The near-field pair function as one polynomial.
//
// Inside the cutoff, eq. (3.8), the pair force is q_i q_j [F_N1 + F_N2](r) d with
// F_N1 = exp(-r/lambda)(1 + r/lambda)/r^3 and F_N2 = -G(r^2), G(r^2) =
// sum_g 2 c_g s_g exp(-s_g r^2), and the pair energy q_i q_j (Y(r) - F(r)) with
// F(r) = sum_g c_g exp(-s_g r^2).  Multiplying out the singular factors leaves
//   H(r) = r^3 [F_N1 + F_N2] = exp(-r/lambda)(1 + r/lambda) - r^3 G(r^2),
//   K(r) = r (Y - F)         = exp(-r/lambda) - r F(r^2),
// (for a two-term kernel, the terms' a_t exp(-r/l_t)(1 + r/l_t) and
// a_t exp(-r/l_t) summed in place of the first parts),
// both entire in r with H(0) = K(0) = 1 and derivatives governed by
// r_c/lambda and s_max r_c^2 (a few units for the SOG of Algorithm 1 at eps =
// 1e-4).  On [0, r_c] each is matched by a single polynomial in y = 2 r / r_c
// - 1: Chebyshev interpolation at 64 nodes in long double, truncated to a
// degree of kNearPolyDegs, converted to powers of y.  A fit is accepted only if
// its error, measured against a long-double evaluation on a fine grid with the
// kernel's FP64 Horner, is below kNearPolyTol; the lowest degree at which both
// H and K pass is taken (each degree fewer is one FMA fewer per pair in the
// kernel); when none passes the kernels evaluate the exponentials one by one.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace rbsog {

namespace {

constexpr int kNodes = 64;
constexpr int kCheck = 512;   // validation intervals on [-1, 1]

// cos(pi k (j + 1/2) / kNodes), shared by every fit
struct CosTable {
    long double c[kNodes][kNodes];
    CosTable()
    {
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int k = 0; k < kNodes; ++k)
            for (int j = 0; j < kNodes; ++j) c[k][j] = std::cos(pi * k * (j + 0.5L) / kNodes);
    }
};
const CosTable &cos_table()
{
    static const CosTable t;
    return t;
}

// H(r) (force) or K(r) (energy) in extended precision.
long double hk(const rbsog_sog &s, long double r, bool force)
{
    const long double r2 = r * r;
    long double acc = 0.0L;
    for (int g = 0; g < s.n; ++g) {
        long double e = std::exp(-(long double)s.s[g] * r2);
        acc += force ? 2.0L * (long double)s.c[g] * (long double)s.s[g] * e : (long double)s.c[g] * e;
    }
    const KernelTerms K = kernel_terms(s);
    long double y = 0.0L;
    for (int t = 0; t < K.n; ++t) {
        const long double rl = r / (long double)K.l[t];
        const long double ey = std::exp(-rl);
        y += (long double)K.a[t] * (force ? ey * (1.0L + rl) : ey);
    }
    return force ? y - r2 * r * acc : y - r * acc;
}

// Chebyshev interpolant of degree < kNodes of H or K over r = (y + 1) r_c / 2,
// y in [-1, 1], truncated to degree deg <= kNearPolyDeg and written in powers
// of y (the powers above deg zero).
bool fit(const rbsog_sog &s, double rc, bool force, int deg, double out[kNearPolyDeg + 1])
{
    const CosTable &ct = cos_table();
    std::vector<long double> fx(kNodes), b(kNodes);
    for (int j = 0; j < kNodes; ++j) fx[j] = hk(s, 0.5L * (ct.c[1][j] + 1.0L) * (long double)rc, force);
    for (int k = 0; k < kNodes; ++k) {
        long double acc = 0.0L;
        for (int j = 0; j < kNodes; ++j) acc += fx[j] * ct.c[k][j];
        b[k] = acc * (k == 0 ? 1.0L : 2.0L) / kNodes;
    }
    // sum_k b_k T_k(x) -> sum_k a_k x^k (k <= deg), with T_{k+1} = 2x T_k - T_{k-1}
    std::vector<long double> a(deg + 1, 0.0L), t0(deg + 1, 0.0L), t1(deg + 1, 0.0L);
    t0[0] = 1.0L;
    t1[1] = 1.0L;
    a[0] += b[0];
    for (int i = 0; i <= deg; ++i) a[i] += b[1] * t1[i];
    for (int k = 2; k <= deg; ++k) {
        std::vector<long double> t2(deg + 1, 0.0L);
        for (int i = 0; i < deg; ++i) t2[i + 1] = 2.0L * t1[i];
        for (int i = 0; i <= deg; ++i) t2[i] -= t0[i];
        for (int i = 0; i <= deg; ++i) a[i] += b[k] * t2[i];
        t0.swap(t1);
        t1.swap(t2);
    }
    for (int i = 0; i <= kNearPolyDeg; ++i) out[i] = i <= deg ? (double)a[i] : 0.0;
    // accept only a fit within tolerance (FP64 Horner as the kernel runs it;
    // H(0) = K(0) = 1 sets the scale)
    long double worst = 0.0L;
    for (int j = 0; j <= kCheck; ++j) {
        double y = -1.0 + 2.0 * j / (double)kCheck;
        double p = out[deg];
        for (int i = deg - 1; i >= 0; --i) p = std::fma(p, y, out[i]);
        long double ref = hk(s, 0.5L * ((long double)y + 1.0L) * (long double)rc, force);
        worst = std::max(worst, std::fabs((long double)p - ref));
    }
    return worst <= (long double)kNearPolyTol;
}

}  // namespace

int near_poly(const rbsog_sog &s, double rc, double h_out[kNearPolyDeg + 1], double k_out[kNearPolyDeg + 1])
{
    if (s.n < 1 || !(s.lambda > 0.0)) return 0;
    for (int deg : kNearPolyDegs)
        if (fit(s, rc, true, deg, h_out) && fit(s, rc, false, deg, k_out)) return deg;
    return 0;
}

}  // namespace rbsog

extern "C" int rbsog_sog_near_poly(const rbsog_sog *sog, double *h, double *k)
{
    if (!sog || !h || !k) return rbsog::fail(RBSOG_EINVAL, "null argument");
    if (sog->n < 1 || sog->n > RBSOG_MAX_GAUSS || !(sog->r_c > 0.0) || !(sog->lambda > 0.0))
        return rbsog::fail(RBSOG_EINVAL, "not an expanded decomposition");
    return rbsog::near_poly(*sog, sog->r_c, h, k);
}

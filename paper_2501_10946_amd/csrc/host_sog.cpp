// Host side of Algorithm 1 (Section 3.2): the C1-continuous sum-of-Gaussians
// decomposition of the Yukawa kernel, and its C2-continuous form (Appendix C).  Built with -ffp-contract=off so that
// the coefficient expansion is a fixed sequence of IEEE FP64 operations.
#include <cfloat>
#include <cmath>

#include "internal.h"

namespace rbsog {
namespace {

constexpr double kPi = 3.141592653589793;

// The integrand of the integral representation Y(r) = int f(t, r) dt (eq. ftr).
double integrand(double t, double r, double lambda)
{
    return std::exp(-r * r * std::exp(t) - std::exp(-t) / (4.0 * lambda * lambda) + 0.5 * t) / std::sqrt(kPi);
}

// Sum over the fixed-weight Gaussians m = -M1 .. M2-1 of f and of d f / d r
// (d f/dr = -2 r e^t f), at r.
void partial_sums(double lambda, double h, double t0, int M1, int M2, double r, double *val, double *der)
{
    double v = 0.0, d = 0.0;
    for (int m = -M1; m < M2; ++m) {
        double t = t0 + m * h;
        double fv = integrand(t, r, lambda);
        v += fv;
        d += -2.0 * r * std::exp(t) * fv;
    }
    *val = v;
    *der = d;
}

struct C1Problem {
    double lambda, rc, h;
    int M1, M2;
    double y, yp;  // Y(rc), Y'(rc)

    // w from the C0 condition (eq. 2.42); NaN when the narrowest Gaussian
    // underflows at r_c and w is not determined in FP64.
    double weight(double t0) const
    {
        double v, d;
        partial_sums(lambda, h, t0, M1, M2, rc, &v, &d);
        double den = h * integrand(t0 + M2 * h, rc, lambda);
        if (!(den >= DBL_MIN / DBL_EPSILON)) return NAN;
        return (y - h * v) / den;
    }

    // C1 residual (eq. 1.25) with w eliminated: Y'(rc) - F'(rc; t0, w(t0)).
    double residual(double t0) const
    {
        double w = weight(t0);
        double v, d;
        partial_sums(lambda, h, t0, M1, M2, rc, &v, &d);
        double tm = t0 + M2 * h;
        double dn = -2.0 * rc * std::exp(tm) * integrand(tm, rc, lambda);
        return yp - h * (w * dn + d);
    }
};

// The C2 form (Appendix C, eq. c2): the narrowest Gaussian m = M2 has the
// exponent e^{t} sigma r^2, g(r) = pi^{-1/2} exp(-r^2 e^t sigma - e^{-t}/(4 lambda^2) + t/2).
// With S the fixed-weight sum (and S', S'' its r-derivatives), the value and
// slope conditions at r_c read w g = Y/h - S =: P0 and w g' = Y'/h - S' =: P1;
// since g'/g = -2 r e^t sigma they give b = e^t sigma = -P1 / (2 r_c P0) and
// w = P0 / g, and leave the curvature condition, with g'' = (4 r^2 b^2 - 2 b) g,
//   R(t0) = Y''/h - S'' - P0 (4 r_c^2 b^2 - 2 b) = 0.
struct C2Problem {
    double lambda, rc, h;
    int M1, M2;
    double y, yp, ypp;  // Y, Y', Y'' at rc

    // residual of the curvature condition; sigma and w through the pointers;
    // NaN where P0 or b is not positive or g underflows
    double solve(double t0, double *sigma, double *w) const
    {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int m = -M1; m < M2; ++m) {
            const double t = t0 + m * h, a = std::exp(t), f = integrand(t, rc, lambda);
            s0 += f;
            s1 += -2.0 * rc * a * f;
            s2 += (4.0 * rc * rc * a * a - 2.0 * a) * f;
        }
        const double p0 = y / h - s0, p1 = yp / h - s1;
        const double b = -p1 / (2.0 * rc * p0);
        if (!(p0 > 0.0) || !(b > 0.0) || !std::isfinite(b)) return NAN;
        const double tm = t0 + M2 * h;
        const double sg = b / std::exp(tm);
        const double g = std::exp(-rc * rc * std::exp(tm) * sg - std::exp(-tm) / (4.0 * lambda * lambda) + 0.5 * tm) /
                         std::sqrt(kPi);
        if (!(g >= DBL_MIN / DBL_EPSILON)) return NAN;
        if (sigma) *sigma = sg;
        if (w) *w = p0 / g;
        return ypp / h - s2 - p0 * (4.0 * rc * rc * b * b - 2.0 * b);
    }
};

}  // namespace

double step_size(double eps, double delta)
{
    // eq. (2.30) with equality: the aliasing error is then at most eps/3 on [delta, R].
    double a = 6.0 * std::sqrt(2.0 * kPi) * std::exp(1.0 / 6.0);
    return kPi * kPi / (std::log(eps + a / delta) + std::log(1.0 / eps));
}

// Smallest t0 in [0, h) satisfying C1 with a positive weight.  The interval is
// scanned in 400 equal pieces; each sign change is refined by bisection until
// the bracket no longer shrinks in FP64.
int c1_start(double lambda, double rc, double h, int M1, int M2, double *t0_out, double *w_out)
{
    C1Problem pb{lambda, rc, h, M1, M2, std::exp(-rc / lambda) / rc,
                 -std::exp(-rc / lambda) * (1.0 / (lambda * rc) + 1.0 / (rc * rc))};
    const int pieces = 400;
    double a = 0.0, ra = pb.residual(a);
    for (int k = 1; k <= pieces; ++k) {
        double b = (double)k * h / (double)pieces;
        double rb = pb.residual(b);
        double root = NAN;
        if (ra == 0.0) {
            root = a;
        } else if ((ra < 0.0 && rb > 0.0) || (ra > 0.0 && rb < 0.0)) {
            double lo = a, hi = b, rlo = ra;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double rm = pb.residual(mid);
                if (rm == 0.0) { lo = hi = mid; break; }
                if ((rm < 0.0) == (rlo < 0.0)) { lo = mid; rlo = rm; } else { hi = mid; }
            }
            root = 0.5 * (lo + hi);
            // a sign change across a jump of an undetermined weight is not a root
            if (!(std::fabs(pb.residual(root)) <= 1e-8 * std::fabs(pb.yp))) root = NAN;
        }
        if (!std::isnan(root) && root < h) {
            double w = pb.weight(root);
            if (w > 0.0 && std::isfinite(w)) {
                *t0_out = root;
                *w_out = w;
                return 0;
            }
        }
        a = b;
        ra = rb;
    }
    return -1;
}

// Smallest t0 in [0, h) where the C2 conditions hold with w > 0 and sigma >
// e^{-h} (the adjusted Gaussian stays narrower than its neighbour m = M2 - 1):
// 400 equal pieces, each sign change bisected to the resolution of FP64.
int c2_start(double lambda, double rc, double h, int M1, int M2, double *t0_out, double *w_out, double *sigma_out)
{
    const double e = std::exp(-rc / lambda);
    C2Problem pb{lambda, rc, h, M1, M2, e / rc, -e * (1.0 / (lambda * rc) + 1.0 / (rc * rc)),
                 e * (1.0 / (lambda * lambda * rc) + 2.0 / (lambda * rc * rc) + 2.0 / (rc * rc * rc))};
    const int pieces = 400;
    double a = 0.0, ra = pb.solve(a, nullptr, nullptr);
    for (int k = 1; k <= pieces; ++k) {
        double b = (double)k * h / (double)pieces;
        double rb = pb.solve(b, nullptr, nullptr);
        double root = NAN;
        if (ra == 0.0) {
            root = a;
        } else if ((ra < 0.0 && rb > 0.0) || (ra > 0.0 && rb < 0.0)) {
            double lo = a, hi = b, rlo = ra;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double rm = pb.solve(mid, nullptr, nullptr);
                if (std::isnan(rm)) break;
                if (rm == 0.0) { lo = hi = mid; break; }
                if ((rm < 0.0) == (rlo < 0.0)) { lo = mid; rlo = rm; } else { hi = mid; }
            }
            root = 0.5 * (lo + hi);
            if (!(std::fabs(pb.solve(root, nullptr, nullptr)) <= 1e-8 * std::fabs(pb.ypp / h))) root = NAN;
        }
        if (!std::isnan(root) && root < h) {
            double sg = NAN, w = NAN;
            pb.solve(root, &sg, &w);
            if (w > 0.0 && std::isfinite(w) && sg > std::exp(-h) && std::isfinite(sg)) {
                *t0_out = root;
                *w_out = w;
                *sigma_out = sg;
                return 0;
            }
        }
        a = b;
        ra = rb;
    }
    return -1;
}

void expand(rbsog_sog *s)
{
    const double pi = kPi;
    const double pi32 = pi * std::sqrt(pi);
    const double inv4l2 = 1.0 / (4.0 * s->lambda * s->lambda);
    s->n = s->M1 + s->M2 + 1;
    double F0 = 0.0, Fh0 = 0.0;
    for (int j = 0; j < s->n; ++j) {
        int m = j - s->M1;
        double t = s->t0 + (double)m * s->h;
        double sj = std::exp(t);
        double cj = (s->h / std::sqrt(pi)) * std::exp(0.5 * t - std::exp(-t) * inv4l2);
        if (m == s->M2) {
            cj = cj * s->w;
            if (s->smooth == 2) sj = sj * s->sigma;
        }
        s->c[j] = cj;
        s->s[j] = sj;
        s->A[j] = pi32 * cj / (sj * std::sqrt(sj));
        s->B[j] = 1.0 / (4.0 * sj);
        F0 += cj;
        Fh0 += s->A[j];
    }
    for (int j = s->n; j < RBSOG_MAX_GAUSS; ++j) s->c[j] = s->s[j] = s->A[j] = s->B[j] = 0.0;
    s->F0 = F0;
    s->Fhat0 = Fh0;
}

// max |Y - F| over r = r_c + (33 l - r_c) u^2, u = j/1600, j = 0..1600, with l
// the kernel's longest length (lambda for the Yukawa kernel).
double sog_max_error(const rbsog_sog &s)
{
    const KernelTerms K = kernel_terms(s);
    double R = 33.0 * K.l[0], worst = 0.0;
    for (int j = 0; j <= 1600; ++j) {
        double u = (double)j / 1600.0;
        double r = s.r_c + (R - s.r_c) * u * u;
        double F = 0.0;
        for (int g = 0; g < s.n; ++g) F += s.c[g] * std::exp(-s.s[g] * r * r);
        double Y = 0.0;
        for (int t = 0; t < K.n; ++t) Y += K.a[t] * std::exp(-r / K.l[t]) / r;
        double e = std::fabs(Y - F);
        if (e > worst) worst = e;
    }
    return worst;
}

}  // namespace rbsog

using namespace rbsog;

extern "C" int rbsog_sog_init(double lambda, double r_c, double eps, int smooth, int M1, int M2, rbsog_sog *out)
{
    if (!out) return fail(RBSOG_EINVAL, "rbsog_sog_init: out is null");
    if (!(lambda > 0.0) || !std::isfinite(lambda) || !(r_c > 0.0) || !std::isfinite(r_c))
        return fail(RBSOG_EINVAL, "rbsog_sog_init: lambda and r_c must be positive and finite");
    if (!(eps > 0.0 && eps < 1.0)) return fail(RBSOG_EINVAL, "rbsog_sog_init: eps must lie in (0, 1)");
    if (!(r_c < 33.0 * lambda)) return fail(RBSOG_EINVAL, "rbsog_sog_init: r_c must be below 33 lambda");
    if (smooth != 1 && smooth != 2) return fail(RBSOG_EINVAL, "rbsog_sog_init: smooth must be 1 or 2");
    bool autom = (M1 == RBSOG_AUTO && M2 == RBSOG_AUTO);
    if (!autom && (M1 < 0 || M1 + M2 + 1 < 1 || M1 + M2 + 1 > RBSOG_MAX_GAUSS))
        return fail(RBSOG_EINVAL, "rbsog_sog_init: need M1 >= 0 and 1 <= M1+M2+1 <= %d", RBSOG_MAX_GAUSS);
    rbsog_sog s{};
    s.lambda = lambda;
    s.r_c = r_c;
    s.eps = eps;
    s.h = step_size(eps, r_c);
    s.smooth = smooth;
    s.sigma = 1.0;
    auto start = [&](int m1, int m2) {
        return smooth == 2 ? c2_start(lambda, r_c, s.h, m1, m2, &s.t0, &s.w, &s.sigma)
                           : c1_start(lambda, r_c, s.h, m1, m2, &s.t0, &s.w);
    };
    if (!autom) {
        s.M1 = M1;
        s.M2 = M2;
        if (start(M1, M2) != 0)
            return fail(RBSOG_ENOROOT, "rbsog_sog_init: no C%d starting point with w > 0 for M1=%d M2=%d", smooth, M1,
                        M2);
        expand(&s);
        s.max_err = sog_max_error(s);
        *out = s;
        return RBSOG_OK;
    }
    for (int total = 1; total <= RBSOG_MAX_GAUSS; ++total) {
        for (int m2 = -12; m2 <= total - 1; ++m2) {
            int m1 = total - 1 - m2;
            if (m1 < 0) continue;
            if (start(m1, m2) != 0) continue;
            s.M1 = m1;
            s.M2 = m2;
            expand(&s);
            s.max_err = sog_max_error(s);
            if (s.max_err <= eps) {
                *out = s;
                return RBSOG_OK;
            }
        }
    }
    return fail(RBSOG_ENOROOT, "rbsog_sog_init: no decomposition with at most %d Gaussians meets eps", RBSOG_MAX_GAUSS);
}

// Two-term kernel: the partial fractions of 4 pi / (k^2 eps_EGS(k)).  With
// b = nu lambda^2 / 4 the potential is 4 pi (1 + b k^2) / (b k^4 + k^2 +
// lambda^{-2}); the denominator's roots in k^2 are -alpha_{1,2} =
// -(1 -+ sqrt(1 - nu)) / (2 b), the smaller written as 2 / (lambda^2 (1 +
// sqrt(1 - nu))) to avoid the cancellation, and the residues give the weights.
extern "C" int rbsog_sog_init_egs(double lambda, double nu, double r_c, double eps, int smooth, rbsog_sog *out)
{
    if (!out) return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: out is null");
    if (!(lambda > 0.0) || !std::isfinite(lambda) || !(r_c > 0.0) || !std::isfinite(r_c))
        return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: lambda and r_c must be positive and finite");
    if (!(nu > 0.0 && nu < 1.0)) return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: nu must lie in (0, 1)");
    if (!(eps > 0.0 && eps < 1.0)) return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: eps must lie in (0, 1)");
    if (smooth != 1 && smooth != 2) return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: smooth must be 1 or 2");
    const double root = std::sqrt(1.0 - nu);
    const double alpha[2] = {2.0 / (lambda * lambda * (1.0 + root)), 2.0 * (1.0 + root) / (nu * lambda * lambda)};
    const double gap = alpha[1] - alpha[0];
    rbsog_sog s{};
    s.nyuk = 2;
    s.nu = nu;
    s.ya[0] = alpha[1] / gap;
    s.ya[1] = -alpha[0] / gap;
    s.yl[0] = 1.0 / std::sqrt(alpha[0]);
    s.yl[1] = 1.0 / std::sqrt(alpha[1]);
    if (!(r_c < 33.0 * s.yl[0]))
        return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: r_c must be below 33 times the longer length %g", s.yl[0]);
    const double eps_term = eps / (std::fabs(s.ya[0]) + std::fabs(s.ya[1]));
    int n = 0;
    for (int j = 0; j < 2; ++j) {
        if (!(r_c < 33.0 * s.yl[j])) continue;   // wholly near: no Gaussians
        rbsog_sog t{};
        const int rc = rbsog_sog_init(s.yl[j], r_c, eps_term, smooth, RBSOG_AUTO, RBSOG_AUTO, &t);
        if (rc != RBSOG_OK) return rc;
        if (n + t.n > RBSOG_MAX_GAUSS)
            return fail(RBSOG_EINVAL, "rbsog_sog_init_egs: the two terms need %d Gaussians, more than %d", n + t.n,
                        RBSOG_MAX_GAUSS);
        if (j == 0) {
            s.h = t.h;
            s.t0 = t.t0;
            s.w = t.w;
            s.M1 = t.M1;
            s.M2 = t.M2;
            s.sigma = t.sigma;
        }
        for (int g = 0; g < t.n; ++g, ++n) {
            s.c[n] = s.ya[j] * t.c[g];
            s.s[n] = t.s[g];
            s.A[n] = s.ya[j] * t.A[g];
            s.B[n] = t.B[g];
        }
    }
    s.n = n;
    s.lambda = lambda;
    s.r_c = r_c;
    s.eps = eps;
    s.smooth = smooth;
    s.F0 = 0.0;
    s.Fhat0 = 0.0;
    for (int g = 0; g < n; ++g) {
        s.F0 += s.c[g];
        s.Fhat0 += s.A[g];
    }
    s.max_err = sog_max_error(s);
    if (!(s.max_err <= eps))
        return fail(RBSOG_ENOROOT, "rbsog_sog_init_egs: the combined error %g exceeds eps", s.max_err);
    *out = s;
    return RBSOG_OK;
}

extern "C" int rbsog_sog_expand(rbsog_sog *sog)
{
    if (!sog) return fail(RBSOG_EINVAL, "rbsog_sog_expand: null");
    if (sog->nyuk == 2)
        return fail(RBSOG_EINVAL, "rbsog_sog_expand: a two-term kernel is built by rbsog_sog_init_egs only");
    int n = sog->M1 + sog->M2 + 1;
    if (sog->M1 < 0 || n < 1 || n > RBSOG_MAX_GAUSS)
        return fail(RBSOG_EINVAL, "rbsog_sog_expand: need M1 >= 0 and 1 <= M1+M2+1 <= %d", RBSOG_MAX_GAUSS);
    if (!(sog->lambda > 0.0) || !(sog->h > 0.0) || !(sog->r_c > 0.0) || !std::isfinite(sog->t0) ||
        !std::isfinite(sog->w))
        return fail(RBSOG_EINVAL, "rbsog_sog_expand: lambda, h, r_c must be positive and t0, w finite");
    if (sog->smooth == 2 && !(sog->sigma > 0.0 && std::isfinite(sog->sigma)))
        return fail(RBSOG_EINVAL, "rbsog_sog_expand: the C2 form needs a positive, finite sigma");
    expand(sog);
    sog->max_err = sog_max_error(*sog);
    return RBSOG_OK;
}

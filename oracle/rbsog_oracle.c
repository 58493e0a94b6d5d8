/*
 * rbsog_oracle.c -- plain FP64 CPU oracle for the random batch sum-of-Gaussians
 * (RBSOG) force evaluation and velocity-Verlet step for 3-D periodic Yukawa
 * systems (Chen, Liang & Xu, "Random batch sum-of-Gaussians algorithm for
 * molecular dynamics simulations of Yukawa systems in three dimensions").
 *
 * TEST INFRASTRUCTURE.  This file is the slow, obviously-correct reference that
 * the GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Conventions (all FP64, IEEE round-to-nearest, compiled without fast-math and
 * with -ffp-contract=off):
 *   positions are SoA x[3*N] = {x_0..x_{N-1}, y_0.., z_0..}, cubic box [0,L)^3;
 *   the SOG far field is F(r) = sum_j c_j exp(-s_j r^2), j ascending in m;
 *   its 3-D Fourier transform is Fhat(k) = sum_j A_j exp(-B_j k^2).
 *
 * Every function names the part of the paper it follows.  Where the paper is
 * silent or ambiguous, the reading taken is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.141592653589793

/* ------------------------------------------------------------------------- */
/* Section 1 and 3.1: the kernel and its integral representation             */
/* ------------------------------------------------------------------------- */

/* Yukawa kernel Y(r) = exp(-r/lambda)/r (Section 1). */
double orc_yukawa(double r, double lambda) { return exp(-r / lambda) / r; }

/* dY/dr = -exp(-r/lambda) (1/(lambda r) + 1/r^2). */
double orc_yukawa_dr(double r, double lambda)
{
    return -exp(-r / lambda) * (1.0 / (lambda * r) + 1.0 / (r * r));
}

/* The screened kernels, as sums of Yukawa terms Y(r) = sum_j a_j e^{-r/l_j}/r
 * (1 <= n <= 2): the Yukawa kernel of eq. (epsilon) is n = 1, a = 1,
 * l = lambda; the exact gradient-corrected screening (EGS) kernel of Section 1
 * is the two-term partial-fraction form of orc_egs_split.  Fourier transform:
 * Yhat(k) = sum_j a_j 4 pi l_j^2 / (1 + l_j^2 k^2). */
typedef struct { int n; double a[2], l[2]; } orc_kern;

static orc_kern kern_yukawa(double lambda)
{
    orc_kern K = {1, {1.0, 0.0}, {lambda, 1.0}};
    return K;
}

/* 0 if n is 1 or 2 and every l_j is positive and finite. */
static int kern_make(int n, const double *a, const double *l, orc_kern *K)
{
    if (n < 1 || n > 2) return -1;
    K->n = n;
    K->a[1] = 0.0;
    K->l[1] = 1.0;
    for (int j = 0; j < n; ++j) {
        if (!(l[j] > 0.0) || !isfinite(l[j]) || !isfinite(a[j])) return -1;
        K->a[j] = a[j];
        K->l[j] = l[j];
    }
    return 0;
}

/* sum_j a_j l_j^2: the kernel's integral over space is 4 pi times this
 * (Yhat(0)/(4 pi)); lambda^2 for both the Yukawa and the EGS kernel. */
static double kern_l2(const orc_kern *K)
{
    double acc = 0.0;
    for (int j = 0; j < K->n; ++j) acc += K->a[j] * K->l[j] * K->l[j];
    return acc;
}

/* Y(r) of a kernel given by its terms. */
double orc_kernel_Y(int n, const double *a, const double *l, double r)
{
    orc_kern K;
    if (kern_make(n, a, l, &K) != 0) return NAN;
    double acc = 0.0;
    for (int j = 0; j < K.n; ++j) acc += K.a[j] * exp(-r / K.l[j]) / r;
    return acc;
}

/* The EGS dielectric of Section 1, eps(k) = 1 + (lambda k)^{-2} (1 + nu
 * lambda^2 k^2 / 4)^{-1}, gives the potential 4 pi / (k^2 eps(k)) =
 * 4 pi (1 + b k^2) / (b k^4 + k^2 + lambda^{-2}) with b = nu lambda^2 / 4.  The
 * denominator is b (k^2 + alpha_1)(k^2 + alpha_2) with
 *   alpha_1 = 2 / (lambda^2 (1 + sqrt(1 - nu))),
 *   alpha_2 = 2 (1 + sqrt(1 - nu)) / (nu lambda^2)
 * (alpha_1 written without the cancellation of (1 - sqrt(1 - nu))), and partial
 * fractions give 4 pi / (k^2 eps) = sum_j a_j 4 pi / (k^2 + alpha_j) with
 * a_1 = alpha_2 / (alpha_2 - alpha_1), a_2 = -alpha_1 / (alpha_2 - alpha_1):
 * the difference of two Yukawa kernels of lengths l_j = alpha_j^{-1/2}.
 * a_1 + a_2 = 1 (Coulomb at short range) and a_1 l_1^2 + a_2 l_2^2 = lambda^2.
 * Needs 0 < nu < 1 (nu = 1 is a double root, nu > 1 complex lengths).
 * Returns 0, or -1 outside that range. */
int orc_egs_split(double lambda, double nu, double *a_out, double *l_out)
{
    if (!(lambda > 0.0) || !isfinite(lambda) || !(nu > 0.0) || !(nu < 1.0)) return -1;
    double sq = sqrt(1.0 - nu);
    double al1 = 2.0 / (lambda * lambda * (1.0 + sq));
    double al2 = 2.0 * (1.0 + sq) / (nu * lambda * lambda);
    a_out[0] = al2 / (al2 - al1);
    a_out[1] = -al1 / (al2 - al1);
    l_out[0] = 1.0 / sqrt(al1);
    l_out[1] = 1.0 / sqrt(al2);
    return 0;
}

/* max_{r in G} |Y(r) - F(r)| for a kernel given by its terms and any Gaussian
 * list, on G = { rc + (R - rc) u^2 : u = j/1600, j = 0..1600 } (the grid of
 * orc_sog_maxerr). */
double orc_kernel_maxerr(int n, const double *a, const double *l, double rc, double R, int nG, const double *c,
                         const double *s)
{
    double emax = 0.0;
    for (int j = 0; j <= 1600; ++j) {
        double u = j / 1600.0;
        double r = rc + (R - rc) * u * u;
        double F = 0.0;
        for (int g = 0; g < nG; ++g) F += c[g] * exp(-s[g] * r * r);
        double e = fabs(orc_kernel_Y(n, a, l, r) - F);
        if (e > emax) emax = e;
    }
    return emax;
}

/* Integrand of the integral representation Y(r) = int f(t,r) dt (eq. ftr):
 * f(t,r) = pi^{-1/2} exp(-r^2 e^t - e^{-t}/(4 lambda^2) + t/2). */
double orc_f(double t, double r, double lambda)
{
    return exp(-r * r * exp(t) - exp(-t) / (4.0 * lambda * lambda) + 0.5 * t) / sqrt(ORC_PI);
}

/* d f(t,r)/dr = -2 r e^t f(t,r). */
static double orc_f_dr(double t, double r, double lambda)
{
    return -2.0 * r * exp(t) * orc_f(t, r, lambda);
}

/* ------------------------------------------------------------------------- */
/* Section 3.1-3.2, Algorithm 1: the C1-continuous SOG decomposition          */
/* ------------------------------------------------------------------------- */

/* Step size from the aliasing bound, eq. (2.30), taken with equality:
 * h = pi^2 / ( log(eps + 6 sqrt(2 pi) e^{1/6} / delta) + log(1/eps) ). */
double orc_h_star(double eps, double delta)
{
    return ORC_PI * ORC_PI /
           (log(eps + 6.0 * sqrt(2.0 * ORC_PI) * exp(1.0 / 6.0) / delta) + log(1.0 / eps));
}

/* Weight of the narrowest Gaussian from the C0 condition, eq. (2.42):
 * w = [ Y(rc) - h sum_{m=-M1}^{M2-1} f(t_m, rc) ] / ( h f(t_{M2}, rc) ). */
double orc_sog_w(double lambda, double rc, double h, double t0, int M1, int M2)
{
    double acc = 0.0;
    for (int m = -M1; m <= M2 - 1; ++m) acc += orc_f(t0 + m * h, rc, lambda);
    double den = h * orc_f(t0 + M2 * h, rc, lambda);
    /* The narrowest Gaussian must be representable at r_c with full FP64
     * precision, otherwise w is not determined (it would be a quotient by an
     * underflowed number). */
    if (!(den >= DBL_MIN / DBL_EPSILON)) return NAN;
    return (orc_yukawa(rc, lambda) - h * acc) / den;
}

/* The far-field SOG in the paper's own form, eq. (2.41):
 * F(r) = h [ w f(t_{M2}, r) + sum_{m=-M1}^{M2-1} f(t_m, r) ]. */
double orc_sog_far(double lambda, double h, double t0, double w, int M1, int M2, double r)
{
    double acc = 0.0;
    for (int m = -M1; m <= M2 - 1; ++m) acc += orc_f(t0 + m * h, r, lambda);
    return h * (w * orc_f(t0 + M2 * h, r, lambda) + acc);
}

static double orc_sog_far_dr(double lambda, double h, double t0, double w, int M1, int M2, double r)
{
    double acc = 0.0;
    for (int m = -M1; m <= M2 - 1; ++m) acc += orc_f_dr(t0 + m * h, r, lambda);
    return h * (w * orc_f_dr(t0 + M2 * h, r, lambda) + acc);
}

typedef struct { double lambda, rc, h; int M1, M2; } c1_ctx;

/* Residual of the force-continuity (C1) condition, eq. (1.25), with w_{M2}
 * eliminated through eq. (2.42): R(t0) = Y'(rc) - F'(rc; t0, w(t0)). */
static double c1_residual(double t0, void *vctx)
{
    const c1_ctx *c = (const c1_ctx *)vctx;
    double w = orc_sog_w(c->lambda, c->rc, c->h, t0, c->M1, c->M2);
    return orc_yukawa_dr(c->rc, c->lambda) - orc_sog_far_dr(c->lambda, c->h, t0, w, c->M1, c->M2, c->rc);
}

double orc_sog_c1_residual(double lambda, double rc, double h, double t0, int M1, int M2)
{
    c1_ctx c = {lambda, rc, h, M1, M2};
    return c1_residual(t0, &c);
}

/* Brent's root finder (bisection safeguarded by secant and inverse quadratic
 * interpolation; R. P. Brent, "Algorithms for Minimization without
 * Derivatives", 1973).  Requires fa*fb < 0. */
static double brent(double (*fn)(double, void *), void *ctx, double a, double b, double fa, double fb,
                    double xtol)
{
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0.0 && fc > 0.0) || (fb < 0.0 && fc < 0.0)) {
            c = a; fc = fa; d = b - a; e = d;
        }
        if (fabs(fc) < fabs(fb)) {
            a = b; b = c; c = a;
            fa = fb; fb = fc; fc = fa;
        }
        double tol = 2.0 * DBL_EPSILON * fabs(b) + 0.5 * xtol;
        double mid = 0.5 * (c - b);
        if (fabs(mid) <= tol || fb == 0.0) return b;
        if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
            double s = fb / fa, p, q;
            if (a == c) {
                p = 2.0 * mid * s;
                q = 1.0 - s;
            } else {
                double qq = fa / fc, r = fb / fc;
                p = s * (2.0 * mid * qq * (qq - r) - (b - a) * (r - 1.0));
                q = (qq - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0.0) q = -q; else p = -p;
            double lim1 = 3.0 * mid * q - fabs(tol * q), lim2 = fabs(e * q);
            if (2.0 * p < (lim1 < lim2 ? lim1 : lim2)) { e = d; d = p / q; }
            else { d = mid; e = mid; }
        } else {
            d = mid; e = mid;
        }
        a = b; fa = fb;
        b += (fabs(d) > tol) ? d : (mid > 0.0 ? tol : -tol);
        fb = fn(b, ctx);
    }
    return b;
}

/* Algorithm 1 step 6 for fixed (h, M1, M2): the starting point t0 in [0,h)
 * that satisfies C1 (eq. 1.25) with w from C0 (eq. 2.42).  The paper allows
 * several roots; the reading taken is the smallest root in [0,h) whose weight
 * w is positive (this is the root printed in Table 1 for every row).
 * Roots are bracketed by a scan of [0,h) in 400 equal subintervals and refined
 * with Brent's method.  Returns 0 and sets *t0,*w on success, -1 if no root. */
int orc_sog_c1_root(double lambda, double rc, double h, int M1, int M2, double *t0_out, double *w_out)
{
    c1_ctx c = {lambda, rc, h, M1, M2};
    const int nscan = 400;
    double a = 0.0, fa = c1_residual(a, &c);
    for (int k = 0; k < nscan; ++k) {
        double b = (double)(k + 1) * h / (double)nscan;
        double fb = c1_residual(b, &c);
        double root = NAN;
        if (fa == 0.0) root = a;
        else if ((fa < 0.0 && fb > 0.0) || (fa > 0.0 && fb < 0.0)) root = brent(c1_residual, &c, a, b, fa, fb, 1e-15);
        /* accept only a genuine zero of the residual (a sign change across a
         * jump of an undetermined w is not a root) */
        if (!isnan(root) && !(fabs(c1_residual(root, &c)) <= 1e-8 * fabs(orc_yukawa_dr(rc, lambda)))) root = NAN;
        if (!isnan(root) && root < h) {
            double w = orc_sog_w(lambda, rc, h, root, M1, M2);
            if (w > 0.0 && isfinite(w)) {
                *t0_out = root;
                *w_out = w;
                return 0;
            }
        }
        a = b; fa = fb;
    }
    return -1;
}

/* max_{r in G} |Y(r) - F(r)| on the grid G = { rc + (33 lambda - rc) u^2 : u = j/1600,
 * j = 0..1600 }, the approximation range [delta, R] = [rc, 33 lambda] of
 * Section 3.2 sampled densely near rc. */
double orc_sog_maxerr(double lambda, double rc, double h, double t0, double w, int M1, int M2)
{
    double R = 33.0 * lambda, emax = 0.0;
    for (int j = 0; j <= 1600; ++j) {
        double u = (double)j / 1600.0;
        double r = rc + (R - rc) * u * u;
        double e = fabs(orc_yukawa(r, lambda) - orc_sog_far(lambda, h, t0, w, M1, M2, r));
        if (e > emax) emax = e;
    }
    return emax;
}

/* Algorithm 1 with the numbers of Gaussians chosen automatically.  The
 * paper's truncation criteria (eqs. 2.33-2.34) need t0, which in turn needs
 * M1, M2; the reading taken is the smallest total M_tot = M1 + M2 + 1 for which
 * a C1 root with w > 0 exists and the pointwise error on [rc, 33 lambda] is at
 * most eps.  For each M_tot the candidates are M2 = -12 .. M_tot-1 in that
 * order (M1 = M_tot - 1 - M2 >= 0); the first one accepted is returned. */
int orc_sog_auto(double lambda, double rc, double eps, int *M1_out, int *M2_out, double *h_out,
                 double *t0_out, double *w_out, double *err_out)
{
    double h = orc_h_star(eps, rc);
    for (int Mtot = 1; Mtot <= 48; ++Mtot) {
        for (int M2 = -12; M2 <= Mtot - 1; ++M2) {
            int M1 = Mtot - 1 - M2;
            if (M1 < 0) continue;
            double t0, w;
            if (orc_sog_c1_root(lambda, rc, h, M1, M2, &t0, &w) != 0) continue;
            double err = orc_sog_maxerr(lambda, rc, h, t0, w, M1, M2);
            if (err <= eps) {
                *M1_out = M1; *M2_out = M2; *h_out = h; *t0_out = t0; *w_out = w; *err_out = err;
                return 0;
            }
        }
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Appendix C: the C2-continuous decomposition                                */
/* ------------------------------------------------------------------------- */

/* Narrowest Gaussian of eq. (c2), its bandwidth scaled by sigma:
 * g(r) = pi^{-1/2} exp(-r^2 e^{t} sigma - e^{-t}/(4 lambda^2) + t/2), t = t_M2. */
static double orc_g2(double t, double sigma, double r, double lambda)
{
    return exp(-r * r * exp(t) * sigma - exp(-t) / (4.0 * lambda * lambda) + 0.5 * t) / sqrt(ORC_PI);
}

/* d^2 Y / dr^2 = exp(-r/lambda) (1/(lambda^2 r) + 2/(lambda r^2) + 2/r^3). */
double orc_yukawa_dr2(double r, double lambda)
{
    return exp(-r / lambda) * (1.0 / (lambda * lambda * r) + 2.0 / (lambda * r * r) + 2.0 / (r * r * r));
}

/* F(r) of eq. (c2): h [ w g(r) + sum_{m=-M1}^{M2-1} f(t_m, r) ]. */
double orc_sog_far2(double lambda, double h, double t0, double w, double sigma, int M1, int M2, double r)
{
    double acc = 0.0;
    for (int m = -M1; m <= M2 - 1; ++m) acc += orc_f(t0 + m * h, r, lambda);
    return h * (w * orc_g2(t0 + M2 * h, sigma, r, lambda) + acc);
}

typedef struct { double lambda, rc, h; int M1, M2; } c2_ctx;

/* For a given t0 the potential and force conditions at rc fix the narrowest
 * Gaussian: with S the fixed-weight sum, P0 = Y(rc)/h - S(rc) = w g(rc) and
 * P1 = Y'(rc)/h - S'(rc) = w g'(rc), and g'/g = -2 r e^{t_M2} sigma, so
 * b := e^{t_M2} sigma = -P1 / (2 rc P0) and w = P0 / g(rc).  Returns the
 * curvature residual Y''(rc)/h - S''(rc) - w g''(rc), g'' = (4 r^2 b^2 - 2 b) g,
 * and (through the pointers, when given) sigma and w; NaN where b or P0 is
 * not positive. */
static double c2_solve(double t0, const c2_ctx *c, double *sigma_out, double *w_out)
{
    double S0 = 0.0, S1 = 0.0, S2 = 0.0, r = c->rc;
    for (int m = -c->M1; m <= c->M2 - 1; ++m) {
        double t = t0 + m * c->h, a = exp(t), fv = orc_f(t, r, c->lambda);
        S0 += fv;
        S1 += -2.0 * r * a * fv;
        S2 += (4.0 * r * r * a * a - 2.0 * a) * fv;
    }
    double P0 = orc_yukawa(r, c->lambda) / c->h - S0;
    double P1 = orc_yukawa_dr(r, c->lambda) / c->h - S1;
    double b = -P1 / (2.0 * r * P0);
    if (!(P0 > 0.0) || !(b > 0.0) || !isfinite(b)) return NAN;
    double tm = t0 + c->M2 * c->h;
    double sigma = b / exp(tm);
    double g = orc_g2(tm, sigma, r, c->lambda);
    if (!(g >= DBL_MIN / DBL_EPSILON)) return NAN;
    if (sigma_out) *sigma_out = sigma;
    if (w_out) *w_out = P0 / g;
    return orc_yukawa_dr2(r, c->lambda) / c->h - S2 - P0 * (4.0 * r * r * b * b - 2.0 * b);
}

static double c2_residual(double t0, void *vctx) { return c2_solve(t0, (const c2_ctx *)vctx, NULL, NULL); }

double orc_sog_c2_residual(double lambda, double rc, double h, double t0, int M1, int M2)
{
    c2_ctx c = {lambda, rc, h, M1, M2};
    return c2_residual(t0, &c);
}

/* Smallest t0 in [0, h) where C0, C1 and C2 hold together with w > 0 and
 * sigma > e^{-h} -- the adjusted Gaussian stays the narrowest, its exponent
 * e^{t_M2} sigma above its neighbour's e^{t_M2 - h}: the interval scanned in
 * 400 pieces, each sign change of the curvature residual refined by Brent's
 * method. */
int orc_sog_c2_root(double lambda, double rc, double h, int M1, int M2, double *t0_out, double *w_out,
                    double *sigma_out)
{
    c2_ctx c = {lambda, rc, h, M1, M2};
    const int nscan = 400;
    double a = 0.0, fa = c2_residual(a, &c);
    for (int k = 0; k < nscan; ++k) {
        double b = (double)(k + 1) * h / (double)nscan;
        double fb = c2_residual(b, &c);
        double root = NAN;
        if (fa == 0.0) root = a;
        else if ((fa < 0.0 && fb > 0.0) || (fa > 0.0 && fb < 0.0)) root = brent(c2_residual, &c, a, b, fa, fb, 1e-15);
        if (!isnan(root) && !(fabs(c2_residual(root, &c)) <= 1e-8 * fabs(orc_yukawa_dr2(rc, lambda) / h))) root = NAN;
        if (!isnan(root) && root < h) {
            double sg, w;
            c2_solve(root, &c, &sg, &w);
            if (w > 0.0 && isfinite(w) && sg > exp(-h) && isfinite(sg)) {
                *t0_out = root;
                *w_out = w;
                *sigma_out = sg;
                return 0;
            }
        }
        a = b; fa = fb;
    }
    return -1;
}

/* max |Y - F| of eq. (c2) on the grid of orc_sog_maxerr. */
double orc_sog_maxerr2(double lambda, double rc, double h, double t0, double w, double sigma, int M1, int M2)
{
    double R = 33.0 * lambda, emax = 0.0;
    for (int j = 0; j <= 1600; ++j) {
        double u = (double)j / 1600.0;
        double r = rc + (R - rc) * u * u;
        double e = fabs(orc_yukawa(r, lambda) - orc_sog_far2(lambda, h, t0, w, sigma, M1, M2, r));
        if (e > emax) emax = e;
    }
    return emax;
}

/* Automatic numbers of Gaussians for the C2 decomposition, by the rule of
 * orc_sog_auto (smallest M_tot, M2 from -12 up, first set meeting eps). */
int orc_sog_auto2(double lambda, double rc, double eps, int *M1_out, int *M2_out, double *h_out, double *t0_out,
                  double *w_out, double *sigma_out, double *err_out)
{
    double h = orc_h_star(eps, rc);
    for (int Mtot = 1; Mtot <= 48; ++Mtot) {
        for (int M2 = -12; M2 <= Mtot - 1; ++M2) {
            int M1 = Mtot - 1 - M2;
            if (M1 < 0) continue;
            double t0, w, sg;
            if (orc_sog_c2_root(lambda, rc, h, M1, M2, &t0, &w, &sg) != 0) continue;
            double err = orc_sog_maxerr2(lambda, rc, h, t0, w, sg, M1, M2);
            if (err <= eps) {
                *M1_out = M1; *M2_out = M2; *h_out = h; *t0_out = t0; *w_out = w; *sigma_out = sg;
                *err_out = err;
                return 0;
            }
        }
    }
    return -1;
}

/* Expansion of the SOG (eq. 2.41) into Gaussian coefficients, index
 * j = m + M1 for m = -M1..M2 (ascending m), and of its 3-D Fourier transform
 * (Section 4.1, the transform of F):
 *   t_m = t0 + m h,  s_j = e^{t_m},
 *   c_j = (h / sqrt(pi)) exp(t_m/2 - e^{-t_m}/(4 lambda^2))   (times w at m = M2),
 *   A_j = pi^{3/2} c_j / (s_j sqrt(s_j)),  B_j = 1 / (4 s_j),
 * so that F(r) = sum_j c_j exp(-s_j r^2) and Fhat(k) = sum_j A_j exp(-B_j k^2).
 * The evaluation order of every expression is part of the contract with the
 * sampler (the shell weights must be reproducible bit for bit). */
void orc_sog_expand_s(double lambda, double h, double t0, double w, double sigma, int M1, int M2, double *c,
                      double *s, double *A, double *B);

void orc_sog_expand(double lambda, double h, double t0, double w, int M1, int M2, double *c, double *s,
                    double *A, double *B)
{
    orc_sog_expand_s(lambda, h, t0, w, 1.0, M1, M2, c, s, A, B);
}

/* The same with the narrowest Gaussian's bandwidth scaled by sigma (the C2
 * form of Appendix C: s_j = e^{t_M2} sigma at m = M2; sigma = 1 is the C1 form). */
void orc_sog_expand_s(double lambda, double h, double t0, double w, double sigma, int M1, int M2, double *c,
                      double *s, double *A, double *B)
{
    const double pi = ORC_PI;
    const double pi32 = pi * sqrt(pi);
    const double inv4l2 = 1.0 / (4.0 * lambda * lambda);
    for (int m = -M1; m <= M2; ++m) {
        int j = m + M1;
        double t = t0 + (double)m * h;
        double sj = exp(t);
        double cj = (h / sqrt(pi)) * exp(0.5 * t - exp(-t) * inv4l2);
        if (m == M2) {
            cj = cj * w;
            sj = sj * sigma;
        }
        c[j] = cj;
        s[j] = sj;
        A[j] = pi32 * cj / (sj * sqrt(sj));
        B[j] = 1.0 / (4.0 * sj);
    }
}

/* F(r) and Fhat(k^2) from the expanded coefficients, summed in ascending j. */
double orc_F(int nG, const double *c, const double *s, double r)
{
    double acc = 0.0;
    for (int j = 0; j < nG; ++j) acc += c[j] * exp(-s[j] * r * r);
    return acc;
}

double orc_Fhat(int nG, const double *A, const double *B, double k2)
{
    double acc = 0.0;
    for (int j = 0; j < nG; ++j) acc += A[j] * exp(-B[j] * k2);
    return acc;
}

/* -dFhat/d(k^2) = sum_j A_j B_j exp(-B_j k^2): how the far-field kernel
 * changes when a scaling of the box moves every k = 2 pi n / L. */
double orc_Fhat_slope(int nG, const double *A, const double *B, double k2)
{
    double acc = 0.0;
    for (int j = 0; j < nG; ++j) acc += A[j] * B[j] * exp(-B[j] * k2);
    return acc;
}

/* ------------------------------------------------------------------------- */
/* Section 4.3: the adaptive importance-sampling density                      */
/* ------------------------------------------------------------------------- */

enum { ORC_ADAPTIVE = 0, ORC_FLAT = 1, ORC_K2 = 2, ORC_DH4PI = 3 };

/* Correction factor F(k) of the sampling measure P(k) = F(k) Fhat(k) / S
 * (eq. 3.124).  ADAPTIVE is the leading Debye-Hueckel term of eq. (3.22),
 * kTV / (kTV/sum q^2 + eps(k)^{-1}/k^2) with eps(k) = 1 + (lambda k)^{-2}
 * (eq. epsilon), so eps^{-1}/k^2 = lambda^2/(1 + lambda^2 k^2), taken literally
 * as printed.  FLAT (F = 1) and K2 (F = k^2) are the two earlier densities the
 * paper compares against in Section 4.2; DH4PI keeps the 4 pi that the
 * potential's own Fourier transform carries (4 pi lambda^2/(1 + lambda^2 k^2)). */
static double density_k(int kind, double kT, double V, double Q2, const orc_kern *K, double k2)
{
    /* eps(k)^{-1}/k^2 = Yhat(k)/(4 pi) = sum_j a_j l_j^2/(1 + l_j^2 k^2) */
    double g = 0.0;
    for (int j = 0; j < K->n; ++j) {
        double l2 = K->l[j] * K->l[j];
        g += K->a[j] * l2 / (1.0 + l2 * k2);
    }
    switch (kind) {
    case ORC_FLAT: return 1.0;
    case ORC_K2: return k2;
    case ORC_DH4PI: return (kT * V) / ((kT * V) / Q2 + 4.0 * ORC_PI * g);
    default: return (kT * V) / ((kT * V) / Q2 + g);
    }
}

double orc_density(int kind, double kT, double V, double Q2, double lambda, double k2)
{
    orc_kern K = kern_yukawa(lambda);
    return density_k(kind, kT, V, Q2, &K, k2);
}

/* The same for a kernel given by its terms (the first term of eq. (3.22) is
 * written for any dielectric eps(k): eps^{-1}/k^2 is the kernel's
 * Yhat(k)/(4 pi)).  NAN for a bad kernel. */
double orc_density_k(int kind, double kT, double V, double Q2, int n, const double *a, const double *l, double k2)
{
    orc_kern K;
    if (kern_make(n, a, l, &K) != 0) return NAN;
    return density_k(kind, kT, V, Q2, &K, k2);
}

/* Default lattice truncation: the largest m >= 1 with Fhat(tk2 m) >= 1e-16 Fhat(0),
 * tk2 = (2 pi / L)^2.  Fhat decreases monotonically in k^2, so the sum over
 * |n|^2 <= m_max holds every term above that level. */
int orc_mmax_default(int nG, const double *A, const double *B, double L)
{
    double t = (2.0 * ORC_PI) / L;
    double tk2 = t * t;
    double thr = 1e-16 * orc_Fhat(nG, A, B, 0.0);
    int m = 1;
    while (orc_Fhat(nG, A, B, tk2 * (double)(m + 1)) >= thr) ++m;
    return m;
}

/* The integer lattice {n in Z^3 : 1 <= |n|^2 <= mmax}, sorted by
 * (|n|^2, nx, ny, nz) ascending.  n3 holds [count][3]; start[m] is the first
 * index with |n|^2 = m, for m = 0..mmax+1 (start[mmax+1] = count).
 * A plain enumeration followed by a counting placement per shell. */
int64_t orc_lattice_count(int mmax)
{
    int R = (int)floor(sqrt((double)mmax)) + 1;
    int64_t cnt = 0;
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int c = -R; c <= R; ++c) {
                int64_t m = (int64_t)a * a + (int64_t)b * b + (int64_t)c * c;
                if (m >= 1 && m <= mmax) ++cnt;
            }
    return cnt;
}

void orc_lattice_build(int mmax, int32_t *n3, int64_t *start)
{
    int R = (int)floor(sqrt((double)mmax)) + 1;
    int64_t *fill = (int64_t *)calloc((size_t)mmax + 2, sizeof(int64_t));
    for (int m = 0; m <= mmax + 1; ++m) start[m] = 0;
    /* counts per shell */
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int c = -R; c <= R; ++c) {
                int64_t m = (int64_t)a * a + (int64_t)b * b + (int64_t)c * c;
                if (m >= 1 && m <= mmax) fill[m]++;
            }
    int64_t run = 0;
    for (int m = 0; m <= mmax; ++m) {
        start[m] = run;
        run += fill[m];
        fill[m] = 0;
    }
    start[mmax + 1] = run;
    /* enumeration in (nx, ny, nz) ascending order keeps each shell sorted */
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int c = -R; c <= R; ++c) {
                int64_t m = (int64_t)a * a + (int64_t)b * b + (int64_t)c * c;
                if (m >= 1 && m <= mmax) {
                    int64_t p = start[m] + fill[m]++;
                    n3[3 * p + 0] = a;
                    n3[3 * p + 1] = b;
                    n3[3 * p + 2] = c;
                }
            }
    free(fill);
}

/* Cumulative shell weights of P(k) = F(k) Fhat(k) / S restricted to the
 * lattice {1 <= |n|^2 <= mmax}, k = (2 pi / L) n.  In a cubic box both F and
 * Fhat depend on |n|^2 only, so the measure is a per-shell weight
 * W(m) = F(k^2) Fhat(k^2) times the shell size r3(m).  For the shells m with
 * r3(m) > 0 in ascending m: cdf_i = cdf_{i-1} + r3(m_i) W(m_i), S = cdf_last.
 * Also returns per shell the coefficient coef = S / (P V F(k^2)) of the
 * estimators of eq. (UF).  Returns the number of shells. */
static int shell_table_k(int mmax, const int64_t *start, int nG, const double *A, const double *B, double L,
                         int kind, double kT, double Q2, const orc_kern *K, int P, int32_t *shell_m, double *cdf,
                         double *coef);

int orc_shell_table(int mmax, const int64_t *start, int nG, const double *A, const double *B, double L,
                    int kind, double kT, double Q2, double lambda, int P, int32_t *shell_m, double *cdf,
                    double *coef)
{
    orc_kern K = kern_yukawa(lambda);
    return shell_table_k(mmax, start, nG, A, B, L, kind, kT, Q2, &K, P, shell_m, cdf, coef);
}

static int shell_table_k(int mmax, const int64_t *start, int nG, const double *A, const double *B, double L,
                         int kind, double kT, double Q2, const orc_kern *K, int P, int32_t *shell_m, double *cdf,
                         double *coef)
{
    double t = (2.0 * ORC_PI) / L;
    double tk2 = t * t;
    double V = L * L * L;
    int ns = 0;
    double run = 0.0;
    for (int m = 1; m <= mmax; ++m) {
        int64_t r3 = start[m + 1] - start[m];
        if (r3 <= 0) continue;
        double k2 = tk2 * (double)m;
        double Fk = density_k(kind, kT, V, Q2, K, k2);
        double W = Fk * orc_Fhat(nG, A, B, k2);
        run = run + (double)r3 * W;
        shell_m[ns] = m;
        cdf[ns] = run;
        ns++;
    }
    double S = run;
    for (int i = 0; i < ns; ++i) {
        double k2 = tk2 * (double)shell_m[i];
        double Fk = density_k(kind, kT, V, Q2, K, k2);
        coef[i] = S / ((double)P * V * Fk);
    }
    return ns;
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror & Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                     */
/* ------------------------------------------------------------------------- */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Algorithm 2, first step of each time step: draw P i.i.d. Fourier modes from
 * P(k).  The paper draws them with a Metropolis-Hastings chain whose details it
 * does not give; the reading taken here is exact inverse-CDF sampling of the
 * same measure, which is what the unbiasedness lemma assumes.
 * Sample l at force-evaluation index `step`:
 *   (w0,w1,w2,w3) = Philox4x64-10(counter = (l, step, 0, 0), key = (seed, replica));
 *   u = (w0 >> 11) 2^-53;  target = u S;
 *   i = first shell with cdf_i > target (the last shell if none);
 *   j = floor(w1 r3(m_i) / 2^64)  (high word of the 64x64 product);
 *   n_l = lattice[start[m_i] + j],  coef_l = coef of shell i. */
/* One draw from a shell CDF with two Philox words: the shell from w0, the
 * point within it from w1 (as above).  Sets the shell index and returns the
 * lattice index. */
static int64_t draw_point(uint64_t w0, uint64_t w1, int nshell, const int32_t *shell_m, const double *cdf,
                          const int64_t *start, int *shell_out)
{
    double S = cdf[nshell - 1];
    double u = (double)(w0 >> 11) * (1.0 / 9007199254740992.0);
    double target = u * S;
    int lo = 0, hi = nshell; /* first index with cdf > target */
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (cdf[mid] > target) hi = mid; else lo = mid + 1;
    }
    int i = lo < nshell ? lo : nshell - 1;
    int m = shell_m[i];
    uint64_t r3 = (uint64_t)(start[m + 1] - start[m]);
    uint64_t jhi, jlo;
    mulhilo64(w1, r3, &jhi, &jlo);
    *shell_out = i;
    return start[m] + (int64_t)jhi;
}

void orc_draw(int P, uint64_t step, uint64_t seed, uint32_t replica, int nshell, const int32_t *shell_m,
              const double *cdf, const double *shell_coef, const int64_t *start, const int32_t *n3,
              int32_t *n_out, double *coef_out)
{
    for (int l = 0; l < P; ++l) {
        uint64_t ctr[4] = {(uint64_t)l, step, 0, 0}, key[2] = {seed, (uint64_t)replica}, w[4];
        orc_philox4x64_10(ctr, key, w);
        int i;
        int64_t p = draw_point(w[0], w[1], nshell, shell_m, cdf, start, &i);
        n_out[3 * l + 0] = n3[3 * p + 0];
        n_out[3 * l + 1] = n3[3 * p + 1];
        n_out[3 * l + 2] = n3[3 * p + 2];
        coef_out[l] = shell_coef[i];
    }
}

/* The Metropolis-Hastings variant of the draws (Section 4.1 names the method
 * for sampling P(k) and gives no chain; the reading taken): an independence
 * chain on the lattice whose proposals come from the measure with F = 1,
 * P_q(k) proportional to Fhat(k), drawn exactly as above from its own shell
 * CDF cdf_q.  Against the target P(k) proportional to F(k) Fhat(k) the
 * Metropolis-Hastings ratio P(k') P_q(k) / (P(k) P_q(k')) is F(k') / F(k) =
 * coef(k) / coef(k'), the estimator coefficient S / (P V F) being inversely
 * proportional to F.  Step l at force-evaluation index `step`:
 *   (w0, w1, w2, w3) = Philox4x64-10(counter = (l, step, 2, 0), key = (seed, replica));
 *   proposal k' (shell i') from w0, w1 on cdf_q;  a = (w2 >> 11) 2^-53;
 *   the chain moves to k' iff it is empty or a coef(i') < coef(i);
 *   sample l = the chain's state after that decision.
 * state[2] = (lattice index, shell index) of the chain, shell index -1 for
 * an empty chain; it carries over from call to call. */
void orc_mh_draw(int P, uint64_t step, uint64_t seed, uint32_t replica, int nshell, const int32_t *shell_m,
                 const double *cdf_q, const double *shell_coef, const int64_t *start, const int32_t *n3,
                 int64_t *state, int32_t *n_out, double *coef_out)
{
    for (int l = 0; l < P; ++l) {
        uint64_t ctr[4] = {(uint64_t)l, step, 2, 0}, key[2] = {seed, (uint64_t)replica}, w[4];
        orc_philox4x64_10(ctr, key, w);
        int ip;
        int64_t pp = draw_point(w[0], w[1], nshell, shell_m, cdf_q, start, &ip);
        double a = (double)(w[2] >> 11) * (1.0 / 9007199254740992.0);
        if (state[1] < 0 || a * shell_coef[ip] < shell_coef[state[1]]) {
            state[0] = pp;
            state[1] = ip;
        }
        int64_t p = state[0];
        n_out[3 * l + 0] = n3[3 * p + 0];
        n_out[3 * l + 1] = n3[3 * p + 1];
        n_out[3 * l + 2] = n3[3 * p + 2];
        coef_out[l] = shell_coef[state[1]];
    }
}

/* ------------------------------------------------------------------------- */
/* Cell list (the neighbour set of eq. 3.8, built as cells of width >= rc)    */
/* ------------------------------------------------------------------------- */

/* Cells of a box with edges Lb[3]: nc_d = floor(L_d/rc) cells along axis d,
 * inv_d = nc_d/L_d, c_d = clamp(floor(x_d inv_d), 0, nc_d-1),
 * id = (c_z nc_y + c_y) nc_x + c_x.  cell_start[nc_x nc_y nc_z + 1] and
 * order[N] list the particles sorted by id, ties in ascending particle index
 * (a stable sort of the original order).  Writes nc_d to nc_out. */
void orc_cells_box(int64_t N, const double *x, const double *Lb, double rc, int32_t *cell_start, int32_t *order,
                   int *nc_out)
{
    int nc[3];
    double inv[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = (int)floor(Lb[d] / rc);
        inv[d] = (double)nc[d] / Lb[d];
        nc_out[d] = nc[d];
    }
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *id = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    int64_t *cnt = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    for (int64_t i = 0; i < N; ++i) {
        int cd[3];
        for (int d = 0; d < 3; ++d) {
            double f = floor(x[d * N + i] * inv[d]);
            int c = (int)f;
            if (f < 0.0) c = 0;
            if (c > nc[d] - 1) c = nc[d] - 1;
            cd[d] = c;
        }
        id[i] = (cd[2] * nc[1] + cd[1]) * nc[0] + cd[0];
        cnt[id[i]]++;
    }
    int64_t run = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        cell_start[c] = (int32_t)run;
        run += cnt[c];
        cnt[c] = 0;
    }
    cell_start[ncell] = (int32_t)run;
    for (int64_t i = 0; i < N; ++i) {
        int c = id[i];
        order[cell_start[c] + cnt[c]++] = (int32_t)i;
    }
    free(cnt);
    free(id);
}

/* The cubic box: nc = floor(L/rc) per axis.  Returns nc. */
int orc_cells(int64_t N, const double *x, double L, double rc, int32_t *cell_start, int32_t *order)
{
    const double Lb[3] = {L, L, L};
    int nc[3];
    orc_cells_box(N, x, Lb, rc, cell_start, order, nc);
    return nc[0];
}

/* ------------------------------------------------------------------------- */
/* Section 4.1, eq. (3.8): near field                                         */
/* ------------------------------------------------------------------------- */

/* Pair force factor and energy of the near part N(r) = Y(r) - F(r), r < rc
 * (eq. short):  F_N1(r) = e^{-r/lambda}(1 + r/lambda)/r^3 (summed over the
 * kernel's Yukawa terms, each weighted by a_j, for a two-term kernel),
 * F_N2(r) = -2 sum_j c_j s_j e^{-s_j r^2};  the force on i from j is
 * q_i q_j (F_N1 + F_N2) d with d = r_i - r_j (minimum image; eq. 3.8 is
 * written with r_ij, whose sign is read so that like charges repel). */
static void near_pair(double r2, const orc_kern *K, int nG, const double *c, const double *s, double *fac,
                      double *en)
{
    double r = sqrt(r2);
    double f1 = 0.0, y = 0.0;
    for (int j = 0; j < K->n; ++j) {
        double ey = exp(-r / K->l[j]);
        f1 += K->a[j] * ey * (1.0 + r / K->l[j]) / (r2 * r);
        y += K->a[j] * ey / r;
    }
    double f2 = 0.0, fr = 0.0;
    for (int j = 0; j < nG; ++j) {
        double g = exp(-s[j] * r2);
        f2 += c[j] * s[j] * g;
        fr += c[j] * g;
    }
    *fac = f1 - 2.0 * f2;
    *en = y - fr;
}

/* Near-field forces (written to f, SoA) and energy U_N = 1/2 sum over ordered
 * pairs and images of q_i q_j N(|d|) with 0 < |d| < rc, and (W_out, nullable)
 * its virial W_N = 1/2 sum over the same ordered pairs of d . F_ij: when the
 * configuration and the box are scaled together (d -> s d, V = L^3), a pair
 * potential gives -3V dU/dV = sum over pairs of d . F_ij, since N(r) and N'(r)
 * vanish at r_c (the C0 and C1 conditions of the SOG), so no pair crossing the
 * cutoff contributes.  With L >= 3 rc and
 * N > 2000 the pairs are found through the cell list; otherwise every image
 * shift that can reach within rc is looped over directly (tiny boxes). */
static void near_box(int64_t N, const double *x, const double *q, const double *Lb, orc_kern K, double rc,
                     int nG, const double *c, const double *s, double *f, double *U_out, double *W_out);

void orc_near(int64_t N, const double *x, const double *q, double L, double lambda, double rc, int nG,
              const double *c, const double *s, double *f, double *U_out, double *W_out)
{
    const double Lb[3] = {L, L, L};
    near_box(N, x, q, Lb, kern_yukawa(lambda), rc, nG, c, s, f, U_out, W_out);
}

/* orc_near for a kernel given by its terms.  Returns 0, or -1 for a bad kernel. */
int orc_near_k(int64_t N, const double *x, const double *q, double L, int nY, const double *ya, const double *yl,
               double rc, int nG, const double *c, const double *s, double *f, double *U_out, double *W_out)
{
    const double Lb[3] = {L, L, L};
    orc_kern K;
    if (kern_make(nY, ya, yl, &K) != 0) return -1;
    near_box(N, x, q, Lb, K, rc, nG, c, s, f, U_out, W_out);
    return 0;
}

/* orc_near_k in a box of edges Lb[3] (a cuboid; every pair within rc, over
 * all images). */
int orc_near_box(int64_t N, const double *x, const double *q, const double *Lb, int nY, const double *ya,
                 const double *yl, double rc, int nG, const double *c, const double *s, double *f, double *U_out,
                 double *W_out)
{
    orc_kern K;
    if (kern_make(nY, ya, yl, &K) != 0) return -1;
    near_box(N, x, q, Lb, K, rc, nG, c, s, f, U_out, W_out);
    return 0;
}

static void near_box(int64_t N, const double *x, const double *q, const double *Lb, orc_kern K, double rc,
                     int nG, const double *c, const double *s, double *f, double *U_out, double *W_out)
{
    double rc2 = rc * rc;
    double *ei = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    double *wi = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = (int)floor(Lb[d] / rc);
    if (nc[0] >= 3 && nc[1] >= 3 && nc[2] >= 3 && N > 2000) {
        int32_t *cs = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc[0] * nc[1] * nc[2] + 1));
        int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        int ncb[3];
        orc_cells_box(N, x, Lb, rc, cs, ord, ncb);
        double inv[3];
        for (int d = 0; d < 3; ++d) inv[d] = (double)nc[d] / Lb[d];
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i) {
            double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
            int ci[3];
            for (int d = 0; d < 3; ++d) {
                double fl = floor(x[d * N + i] * inv[d]);
                int cc = (int)fl;
                if (fl < 0.0) cc = 0;
                if (cc > nc[d] - 1) cc = nc[d] - 1;
                ci[d] = cc;
            }
            double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cx = ci[0] + dx, cy = ci[1] + dy, cz = ci[2] + dz;
                        double sx = 0, sy = 0, sz = 0; /* image shift of the neighbour cell */
                        if (cx < 0) { cx += nc[0]; sx = -Lb[0]; } else if (cx >= nc[0]) { cx -= nc[0]; sx = Lb[0]; }
                        if (cy < 0) { cy += nc[1]; sy = -Lb[1]; } else if (cy >= nc[1]) { cy -= nc[1]; sy = Lb[1]; }
                        if (cz < 0) { cz += nc[2]; sz = -Lb[2]; } else if (cz >= nc[2]) { cz -= nc[2]; sz = Lb[2]; }
                        int cell = (cz * nc[1] + cy) * nc[0] + cx;
                        for (int32_t p = cs[cell]; p < cs[cell + 1]; ++p) {
                            int64_t j = ord[p];
                            if (j == i) continue;
                            double dx_ = xi - (x[j] + sx), dy_ = yi - (x[N + j] + sy), dz_ = zi - (x[2 * N + j] + sz);
                            double r2 = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
                            if (r2 >= rc2) continue;
                            double fac, en;
                            near_pair(r2, &K, nG, c, s, &fac, &en);
                            double qq = q[i] * q[j];
                            fx += qq * fac * dx_; fy += qq * fac * dy_; fz += qq * fac * dz_;
                            e += 0.5 * qq * en;
                            w += 0.5 * qq * fac * r2;
                        }
                    }
            f[i] = fx; f[N + i] = fy; f[2 * N + i] = fz;
            ei[i] = e;
            wi[i] = w;
        }
        free(cs);
        free(ord);
    } else {
        int ni[3];
        for (int d = 0; d < 3; ++d) ni[d] = (int)ceil(rc / Lb[d]);
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < N; ++i) {
            double fx = 0, fy = 0, fz = 0, e = 0, w = 0;
            for (int64_t j = 0; j < N; ++j) {
                for (int a = -ni[0]; a <= ni[0]; ++a)
                    for (int b = -ni[1]; b <= ni[1]; ++b)
                        for (int cc = -ni[2]; cc <= ni[2]; ++cc) {
                            if (j == i && a == 0 && b == 0 && cc == 0) continue;
                            double dx_ = x[i] - x[j] - a * Lb[0];
                            double dy_ = x[N + i] - x[N + j] - b * Lb[1];
                            double dz_ = x[2 * N + i] - x[2 * N + j] - cc * Lb[2];
                            double r2 = dx_ * dx_ + dy_ * dy_ + dz_ * dz_;
                            if (r2 >= rc2 || r2 == 0.0) continue;
                            double fac, en;
                            near_pair(r2, &K, nG, c, s, &fac, &en);
                            double qq = q[i] * q[j];
                            fx += qq * fac * dx_; fy += qq * fac * dy_; fz += qq * fac * dz_;
                            e += 0.5 * qq * en;
                            w += 0.5 * qq * fac * r2;
                        }
            }
            f[i] = fx; f[N + i] = fy; f[2 * N + i] = fz;
            ei[i] = e;
            wi[i] = w;
        }
    }
    double U = 0.0, W = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        U += ei[i];
        W += wi[i];
    }
    *U_out = U;
    if (W_out) *W_out = W;
    free(ei);
    free(wi);
}

/* Near-field force on a subset of particles idx[0..nsub) (for checks at sizes
 * where the whole near field is too slow on the CPU): the same pair sum of
 * eq. (3.8) over every j != i and every image with |d| < rc, found by a cell
 * list when L >= 3 rc and by looping over every image shift that can reach
 * within rc otherwise (boxes smaller than three cutoffs).  f_out is
 * [3][nsub].  Returns 0, or -1 for an index outside [0, N). */
static int near_subset_box(int64_t N, const double *x, const double *q, const double *Lb, orc_kern K, double rc,
                           int nG, const double *c, const double *s, int64_t nsub, const int64_t *idx,
                           double *f_out);

int orc_near_subset(int64_t N, const double *x, const double *q, double L, double lambda, double rc, int nG,
                    const double *c, const double *s, int64_t nsub, const int64_t *idx, double *f_out)
{
    const double Lb[3] = {L, L, L};
    return near_subset_box(N, x, q, Lb, kern_yukawa(lambda), rc, nG, c, s, nsub, idx, f_out);
}

/* orc_near_subset for a kernel given by its terms (-1 also for a bad kernel). */
int orc_near_subset_k(int64_t N, const double *x, const double *q, double L, int nY, const double *ya,
                      const double *yl, double rc, int nG, const double *c, const double *s, int64_t nsub,
                      const int64_t *idx, double *f_out)
{
    const double Lb[3] = {L, L, L};
    orc_kern K;
    if (kern_make(nY, ya, yl, &K) != 0) return -1;
    return near_subset_box(N, x, q, Lb, K, rc, nG, c, s, nsub, idx, f_out);
}

/* orc_near_subset_k in a box of edges Lb[3]. */
int orc_near_subset_box(int64_t N, const double *x, const double *q, const double *Lb, int nY, const double *ya,
                        const double *yl, double rc, int nG, const double *c, const double *s, int64_t nsub,
                        const int64_t *idx, double *f_out)
{
    orc_kern K;
    if (kern_make(nY, ya, yl, &K) != 0) return -1;
    return near_subset_box(N, x, q, Lb, K, rc, nG, c, s, nsub, idx, f_out);
}

static int near_subset_box(int64_t N, const double *x, const double *q, const double *Lb, orc_kern K, double rc,
                           int nG, const double *c, const double *s, int64_t nsub, const int64_t *idx,
                           double *f_out)
{
    double rc2 = rc * rc;
    int nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = (int)floor(Lb[d] / rc);
    for (int64_t k = 0; k < nsub; ++k)
        if (idx[k] < 0 || idx[k] >= N) return -1;
    if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) {
        int ni[3];
        for (int d = 0; d < 3; ++d) ni[d] = (int)ceil(rc / Lb[d]);
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t k = 0; k < nsub; ++k) {
            int64_t i = idx[k];
            double fx = 0, fy = 0, fz = 0;
            for (int64_t j = 0; j < N; ++j)
                for (int a = -ni[0]; a <= ni[0]; ++a)
                    for (int b = -ni[1]; b <= ni[1]; ++b)
                        for (int cc = -ni[2]; cc <= ni[2]; ++cc) {
                            if (j == i && a == 0 && b == 0 && cc == 0) continue;
                            double ddx = x[i] - x[j] - a * Lb[0];
                            double ddy = x[N + i] - x[N + j] - b * Lb[1];
                            double ddz = x[2 * N + i] - x[2 * N + j] - cc * Lb[2];
                            double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                            if (r2 >= rc2 || r2 == 0.0) continue;
                            double fac, en;
                            near_pair(r2, &K, nG, c, s, &fac, &en);
                            double qq = q[i] * q[j];
                            fx += qq * fac * ddx; fy += qq * fac * ddy; fz += qq * fac * ddz;
                        }
            f_out[k] = fx; f_out[nsub + k] = fy; f_out[2 * nsub + k] = fz;
        }
        return 0;
    }
    int32_t *cs = (int32_t *)malloc(sizeof(int32_t) * ((size_t)nc[0] * nc[1] * nc[2] + 1));
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int ncb[3];
    orc_cells_box(N, x, Lb, rc, cs, ord, ncb);
    double inv[3];
    for (int d = 0; d < 3; ++d) inv[d] = (double)nc[d] / Lb[d];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nsub; ++k) {
        int64_t i = idx[k];
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            double fl = floor(x[d * N + i] * inv[d]);
            int cc = (int)fl;
            if (fl < 0.0) cc = 0;
            if (cc > nc[d] - 1) cc = nc[d] - 1;
            ci[d] = cc;
        }
        double fx = 0, fy = 0, fz = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int cx = ci[0] + dx, cy = ci[1] + dy, cz = ci[2] + dz;
                    double sx = 0, sy = 0, sz = 0;
                    if (cx < 0) { cx += nc[0]; sx = -Lb[0]; } else if (cx >= nc[0]) { cx -= nc[0]; sx = Lb[0]; }
                    if (cy < 0) { cy += nc[1]; sy = -Lb[1]; } else if (cy >= nc[1]) { cy -= nc[1]; sy = Lb[1]; }
                    if (cz < 0) { cz += nc[2]; sz = -Lb[2]; } else if (cz >= nc[2]) { cz -= nc[2]; sz = Lb[2]; }
                    int cell = (cz * nc[1] + cy) * nc[0] + cx;
                    for (int32_t p = cs[cell]; p < cs[cell + 1]; ++p) {
                        int64_t j = ord[p];
                        if (j == i) continue;
                        double ddx = x[i] - (x[j] + sx), ddy = x[N + i] - (x[N + j] + sy), ddz = x[2 * N + i] - (x[2 * N + j] + sz);
                        double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                        if (r2 >= rc2) continue;
                        double fac, en;
                        near_pair(r2, &K, nG, c, s, &fac, &en);
                        double qq = q[i] * q[j];
                        fx += qq * fac * ddx; fy += qq * fac * ddy; fz += qq * fac * ddz;
                    }
                }
        f_out[k] = fx; f_out[nsub + k] = fy; f_out[2 * nsub + k] = fz;
    }
    free(cs);
    free(ord);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Section 2 and 4.1: structure factors and the far field                     */
/* ------------------------------------------------------------------------- */

/* rho(k_l) = sum_j q_j e^{i k_l . r_j} with k_l = 2 pi (n_x/L_x, n_y/L_y, n_z/L_z)
 * (Section 2; a box of edges Lb[3]).  rho is [P][2] = (re, im).  The phase
 * is formed literally as k . r. */
void orc_rho_box(int64_t N, const double *x, const double *q, const double *Lb, int P, const int32_t *n3,
                 double *rho)
{
    double tx = (2.0 * ORC_PI) / Lb[0], ty = (2.0 * ORC_PI) / Lb[1], tz = (2.0 * ORC_PI) / Lb[2];
#pragma omp parallel for schedule(static)
    for (int l = 0; l < P; ++l) {
        double kx = tx * n3[3 * l], ky = ty * n3[3 * l + 1], kz = tz * n3[3 * l + 2];
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double th = kx * x[j] + ky * x[N + j] + kz * x[2 * N + j];
            re += q[j] * cos(th);
            im += q[j] * sin(th);
        }
        rho[2 * l] = re;
        rho[2 * l + 1] = im;
    }
}

/* The cubic box: k = (2 pi / L) n. */
void orc_rho(int64_t N, const double *x, const double *q, double L, int P, const int32_t *n3, double *rho)
{
    const double Lb[3] = {L, L, L};
    orc_rho_box(N, x, q, Lb, P, n3, rho);
}

/* Random-batch far force, eq. (UF):  F*_i = -(S/(2PV)) sum_l grad_i |rho_l|^2 / F(k_l)
 * with grad_i |rho|^2 = 2 q_i k Im(e^{-i k.r_i} rho), i.e.
 * F*_i = -q_i sum_l coef_l k_l (rho_im cos th - rho_re sin th),  coef = S/(P V F(k)).
 * Adds into f (SoA). */
void orc_far_rb_box(int64_t N, const double *x, const double *q, const double *Lb, int P, const int32_t *n3,
                    const double *coef, const double *rho, double *f)
{
    double tx = (2.0 * ORC_PI) / Lb[0], ty = (2.0 * ORC_PI) / Lb[1], tz = (2.0 * ORC_PI) / Lb[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double fx = 0, fy = 0, fz = 0;
        for (int l = 0; l < P; ++l) {
            double kx = tx * n3[3 * l], ky = ty * n3[3 * l + 1], kz = tz * n3[3 * l + 2];
            double th = kx * x[i] + ky * x[N + i] + kz * x[2 * N + i];
            double im = rho[2 * l + 1] * cos(th) - rho[2 * l] * sin(th);
            double g = coef[l] * im;
            fx += g * kx; fy += g * ky; fz += g * kz;
        }
        f[i] -= q[i] * fx;
        f[N + i] -= q[i] * fy;
        f[2 * N + i] -= q[i] * fz;
    }
}

void orc_far_rb(int64_t N, const double *x, const double *q, double L, int P, const int32_t *n3,
                const double *coef, const double *rho, double *f)
{
    const double Lb[3] = {L, L, L};
    orc_far_rb_box(N, x, q, Lb, P, n3, coef, rho, f);
}

/* Estimator of the far energy, eq. (UF): U*_F = S/(2PV) sum_l |rho_l|^2 / F(k_l)
 * = 1/2 sum_l coef_l |rho_l|^2. */
double orc_far_rb_energy(int P, const double *coef, const double *rho)
{
    double U = 0.0;
    for (int l = 0; l < P; ++l) U += coef[l] * (rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1]);
    return 0.5 * U;
}

/* Virial of the far field, W_F = -3V dU_F/dV with the configuration scaled
 * with the box (all edges by one factor): U_F = (1/2V) sum_k Fhat(k^2) |rho(k)|^2
 * has rho unchanged (k . r is invariant) while 1/V and k^2 (each k_d = 2 pi
 * n_d / L_d, so k^2 is prop. to V^(-2/3))
 * change, so W_F = 3 U_F - (1/V) sum_k k^2 G(k^2) |rho(k)|^2 with
 * G = -dFhat/d(k^2).  Its random-batch estimator over the modes of eq. (UF)
 * (the same importance weights as the energy, coef_l = S / (P V F(k_l))):
 *   W*_F = sum_l coef_l |rho_l|^2 (3/2 - k_l^2 G(k_l^2) / Fhat(k_l^2)). */
static double box_k2(const double *Lb, const int32_t *n)
{
    if (Lb[0] == Lb[1] && Lb[1] == Lb[2]) { /* cubic: (2 pi/L)^2 |n|^2, as the shell tables form it */
        double t = (2.0 * ORC_PI) / Lb[0];
        double m = (double)n[0] * n[0] + (double)n[1] * n[1] + (double)n[2] * n[2];
        return t * t * m;
    }
    double kx = (2.0 * ORC_PI) * n[0] / Lb[0], ky = (2.0 * ORC_PI) * n[1] / Lb[1], kz = (2.0 * ORC_PI) * n[2] / Lb[2];
    return kx * kx + ky * ky + kz * kz;
}

double orc_far_rb_virial_box(int P, const int32_t *n3, const double *coef, const double *rho, const double *Lb,
                             int nG, const double *A, const double *B)
{
    double W = 0.0;
    for (int l = 0; l < P; ++l) {
        double k2 = box_k2(Lb, n3 + 3 * l);
        double r2 = rho[2 * l] * rho[2 * l] + rho[2 * l + 1] * rho[2 * l + 1];
        W += coef[l] * r2 * (1.5 - k2 * orc_Fhat_slope(nG, A, B, k2) / orc_Fhat(nG, A, B, k2));
    }
    return W;
}

double orc_far_rb_virial(int P, const int32_t *n3, const double *coef, const double *rho, double L, int nG,
                         const double *A, const double *B)
{
    const double Lb[3] = {L, L, L};
    return orc_far_rb_virial_box(P, n3, coef, rho, Lb, nG, A, B);
}

/* Deterministic far field summed over the lattice modes n3[0..cnt) of a box
 * of edges Lb[3] (eqs. 3.5 and 3.8, k = 0 excluded; its energy is added
 * separately):
 *   U_F = (1/2V) sum_k Fhat(k) |rho(k)|^2,
 *   F_i += -(q_i/V) sum_k k Fhat(k) Im(e^{-ik.r_i} rho(k)),
 * and (W_out, nullable) the virial W_F = 3 U_F - (1/V) sum_k k^2 G(k^2) |rho|^2
 * (see orc_far_rb_virial).  Adds into f; returns U_F. */
static double far_full_list(int64_t N, const double *x, const double *q, const double *Lb, int nG, const double *A,
                            const double *B, int64_t cnt, const int32_t *n3, double *f, double *W_out)
{
    double tx = (2.0 * ORC_PI) / Lb[0], ty = (2.0 * ORC_PI) / Lb[1], tz = (2.0 * ORC_PI) / Lb[2];
    double V = Lb[0] * Lb[1] * Lb[2];
    double *rho = (double *)malloc(sizeof(double) * 2 * (size_t)(cnt > 0 ? cnt : 1));
    double *fh = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
    for (int64_t p = 0; p < cnt; ++p) fh[p] = orc_Fhat(nG, A, B, box_k2(Lb, n3 + 3 * p));
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < cnt; ++p) {
        double kx = tx * n3[3 * p], ky = ty * n3[3 * p + 1], kz = tz * n3[3 * p + 2];
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double th = kx * x[j] + ky * x[N + j] + kz * x[2 * N + j];
            re += q[j] * cos(th);
            im += q[j] * sin(th);
        }
        rho[2 * p] = re;
        rho[2 * p + 1] = im;
    }
    double U = 0.0, Wk = 0.0;
    for (int64_t p = 0; p < cnt; ++p) {
        double k2 = box_k2(Lb, n3 + 3 * p);
        double r2 = rho[2 * p] * rho[2 * p] + rho[2 * p + 1] * rho[2 * p + 1];
        U += fh[p] * r2;
        Wk += k2 * orc_Fhat_slope(nG, A, B, k2) * r2;
    }
    U = U / (2.0 * V);
    if (W_out) *W_out = 3.0 * U - Wk / V;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double fx = 0, fy = 0, fz = 0;
        for (int64_t p = 0; p < cnt; ++p) {
            double kx = tx * n3[3 * p], ky = ty * n3[3 * p + 1], kz = tz * n3[3 * p + 2];
            double th = kx * x[i] + ky * x[N + i] + kz * x[2 * N + i];
            double im = rho[2 * p + 1] * cos(th) - rho[2 * p] * sin(th);
            double g = fh[p] * im;
            fx += g * kx; fy += g * ky; fz += g * kz;
        }
        f[i] -= q[i] * fx / V;
        f[N + i] -= q[i] * fy / V;
        f[2 * N + i] -= q[i] * fz / V;
    }
    free(rho); free(fh);
    return U;
}

/* The cubic box over every mode 1 <= |n|^2 <= mmax. */
double orc_far_full(int64_t N, const double *x, const double *q, double L, int nG, const double *A,
                    const double *B, int mmax, double *f, double *W_out)
{
    int64_t cnt = orc_lattice_count(mmax);
    int32_t *n3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)cnt);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)mmax + 2));
    orc_lattice_build(mmax, n3, start);
    const double Lb[3] = {L, L, L};
    double U = far_full_list(N, x, q, Lb, nG, A, B, cnt, n3, f, W_out);
    free(n3); free(start);
    return U;
}

/* ------------------------------------------------------------------------- */
/* Cuboid boxes: the lattice and the sampling measure point by point         */
/* ------------------------------------------------------------------------- */

typedef struct { double k2; int32_t n[3]; } box_point;

static int box_point_cmp(const void *a, const void *b)
{
    const box_point *p = (const box_point *)a, *r = (const box_point *)b;
    if (p->k2 < r->k2) return -1;
    if (p->k2 > r->k2) return 1;
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < r->n[d]) return -1;
        if (p->n[d] > r->n[d]) return 1;
    }
    return 0;
}

/* The Fourier lattice of a box of edges Lb[3] (k = 2 pi (n_x/L_x, n_y/L_y,
 * n_z/L_z)): every n != 0 with Fhat(k^2) >= 1e-16 Fhat(0) (the truncation of
 * the cubic default, Fhat decreasing in k^2), sorted by (k^2, n_x, n_y, n_z).
 * In a cubic box this is the lattice 1 <= |n|^2 <= m_max of the default
 * m_max.  Writes n3_out[count][3] and k2_out[count] when not null; returns the
 * count, or -1 when some |n_d| would exceed 511. */
int64_t orc_box_lattice(const double *Lb, int nG, const double *A, const double *B, int32_t *n3_out,
                        double *k2_out)
{
    double thr = 1e-16 * orc_Fhat(nG, A, B, 0.0);
    double lo = 0.0, hi = 1.0;
    while (orc_Fhat(nG, A, B, hi) >= thr) hi *= 2.0;
    for (int it = 0; it < 200; ++it) { /* the k^2 where Fhat crosses thr */
        double mid = 0.5 * (lo + hi);
        if (orc_Fhat(nG, A, B, mid) >= thr) lo = mid; else hi = mid;
    }
    int nm[3];
    for (int d = 0; d < 3; ++d) {
        nm[d] = (int)floor(Lb[d] * sqrt(hi) / (2.0 * ORC_PI)) + 1;
        if (nm[d] > 511) return -1;
    }
    int64_t cap = (int64_t)(2 * nm[0] + 1) * (2 * nm[1] + 1) * (2 * nm[2] + 1);
    box_point *pts = (box_point *)malloc(sizeof(box_point) * (size_t)cap);
    int64_t cnt = 0;
    for (int a = -nm[0]; a <= nm[0]; ++a)
        for (int b = -nm[1]; b <= nm[1]; ++b)
            for (int c = -nm[2]; c <= nm[2]; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                int32_t n[3] = {a, b, c};
                double k2 = box_k2(Lb, n);
                if (!(orc_Fhat(nG, A, B, k2) >= thr)) continue;
                pts[cnt].k2 = k2;
                pts[cnt].n[0] = a; pts[cnt].n[1] = b; pts[cnt].n[2] = c;
                cnt++;
            }
    qsort(pts, (size_t)cnt, sizeof(box_point), box_point_cmp);
    for (int64_t i = 0; i < cnt; ++i) {
        if (n3_out) for (int d = 0; d < 3; ++d) n3_out[3 * i + d] = pts[i].n[d];
        if (k2_out) k2_out[i] = pts[i].k2;
    }
    free(pts);
    return cnt;
}

/* The far field of orc_far_full over the lattice of orc_box_lattice. */
double orc_far_full_box(int64_t N, const double *x, const double *q, const double *Lb, int nG, const double *A,
                        const double *B, double *f, double *W_out)
{
    int64_t cnt = orc_box_lattice(Lb, nG, A, B, NULL, NULL);
    if (cnt < 0) return NAN;
    int32_t *n3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(cnt > 0 ? cnt : 1));
    orc_box_lattice(Lb, nG, A, B, n3, NULL);
    double U = far_full_list(N, x, q, Lb, nG, A, B, cnt, n3, f, W_out);
    free(n3);
    return U;
}

/* Point-by-point measure of a cuboid box, eq. (3.124) without the shell
 * grouping (the measure depends on k^2, which no longer groups by |n|^2):
 * cdf_i = cdf_{i-1} + F(k_i^2) Fhat(k_i^2) over the lattice in its order,
 * S = cdf_last, coef_i = S / (P V F(k_i^2)). */
static void box_tables(int64_t cnt, const double *k2, int nG, const double *A, const double *B, double V, int kind,
                       double kT, double Q2, const orc_kern *K, int P, double *cdf, double *coef)
{
    double run = 0.0;
    for (int64_t i = 0; i < cnt; ++i) {
        double Fk = density_k(kind, kT, V, Q2, K, k2[i]);
        run = run + Fk * orc_Fhat(nG, A, B, k2[i]);
        cdf[i] = run;
    }
    for (int64_t i = 0; i < cnt; ++i) coef[i] = run / ((double)P * V * density_k(kind, kT, V, Q2, K, k2[i]));
}

/* Draws of a cuboid box: sample l at force-evaluation index `step` takes
 * (w0, ...) = Philox4x64-10(counter = (l, step, 0, 0), key = (seed, replica)),
 * u = (w0 >> 11) 2^-53, and the first point with cdf_i > u S (the last if
 * none). */
void orc_box_draw(int P, uint64_t step, uint64_t seed, uint32_t replica, int64_t cnt, const double *cdf,
                  const double *coef, const int32_t *n3, int32_t *n_out, double *coef_out)
{
    double S = cdf[cnt - 1];
    for (int l = 0; l < P; ++l) {
        uint64_t ctr[4] = {(uint64_t)l, step, 0, 0}, key[2] = {seed, (uint64_t)replica}, w[4];
        orc_philox4x64_10(ctr, key, w);
        double target = (double)(w[0] >> 11) * (1.0 / 9007199254740992.0) * S;
        int64_t lo = 0, hi = cnt;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        int64_t i = lo < cnt ? lo : cnt - 1;
        for (int d = 0; d < 3; ++d) n_out[3 * l + d] = n3[3 * i + d];
        coef_out[l] = coef[i];
    }
}

/* ------------------------------------------------------------------------- */
/* A whole system: tables, one force evaluation, Algorithm 2's time loop      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t N;
    double L, V, lambda, rc, kT, Q1, Q2;
    double Lb[3];  /* edges; a cuboid (cuboid = 1) samples point by point */
    int cuboid;
    orc_kern kern; /* the kernel's Yukawa terms */
    int P, mmax, density, full_k, nG;
    double friction, bath_kT; /* Langevin thermostat (friction 0: plain velocity-Verlet) */
    int bath;                 /* 0 none / Langevin (friction), 2 Nose-Hoover, 3 Berendsen */
    double bath_rate;         /* 1/tau of the global baths                                */
    double xi, eta;           /* Nose-Hoover friction variable and its time integral      */
    uint64_t seed;
    uint32_t replica;
    double c[64], s[64], A[64], B[64];
    double F0, Fhat0;
    const double *q, *m; /* caller-owned, length N */
    /* sampling tables */
    int64_t nlat;
    int32_t *n3;
    int64_t *start;
    int nshell;
    int32_t *shell_m;
    double *cdf, *shell_coef;
    /* Metropolis-Hastings draws (sampler 1): the proposal CDF and the chain */
    int sampler;
    double *cdf_q;
    int64_t mh_state[2];
} orc_sys;

/* Builds the sampling tables of a system.  q and m must outlive the system. */
orc_sys *orc_sys_create_k(int64_t N, double L, int nY, const double *ya, const double *yl, double rc, double kT,
                          int P, int mmax, uint64_t seed, uint32_t replica, int density, int full_k, int nG,
                          const double *c, const double *s, const double *A, const double *B, const double *q,
                          const double *m);

orc_sys *orc_sys_create(int64_t N, double L, double lambda, double rc, double kT, int P, int mmax,
                        uint64_t seed, uint32_t replica, int density, int full_k, int nG, const double *c,
                        const double *s, const double *A, const double *B, const double *q, const double *m)
{
    double one = 1.0;
    return orc_sys_create_k(N, L, 1, &one, &lambda, rc, kT, P, mmax, seed, replica, density, full_k, nG, c, s, A,
                            B, q, m);
}

/* orc_sys_create for a kernel given by its Yukawa terms (ya, yl; nY <= 2). */
orc_sys *orc_sys_create_k(int64_t N, double L, int nY, const double *ya, const double *yl, double rc, double kT,
                          int P, int mmax, uint64_t seed, uint32_t replica, int density, int full_k, int nG,
                          const double *c, const double *s, const double *A, const double *B, const double *q,
                          const double *m)
{
    orc_kern K;
    if (nG < 1 || nG > 64 || kern_make(nY, ya, yl, &K) != 0) return NULL;
    orc_sys *S = (orc_sys *)calloc(1, sizeof(orc_sys));
    S->N = N; S->L = L; S->V = L * L * L; S->lambda = yl[0]; S->kern = K; S->rc = rc; S->kT = kT;
    S->Lb[0] = S->Lb[1] = S->Lb[2] = L;
    S->P = P; S->density = density; S->full_k = full_k; S->nG = nG;
    S->seed = seed; S->replica = replica; S->q = q; S->m = m;
    memcpy(S->c, c, sizeof(double) * nG); memcpy(S->s, s, sizeof(double) * nG);
    memcpy(S->A, A, sizeof(double) * nG); memcpy(S->B, B, sizeof(double) * nG);
    double q1 = 0.0, q2 = 0.0;
    for (int64_t i = 0; i < N; ++i) { q1 += q[i]; q2 += q[i] * q[i]; }
    S->Q1 = q1; S->Q2 = q2;
    S->F0 = 0.0; for (int j = 0; j < nG; ++j) S->F0 += c[j];
    S->Fhat0 = orc_Fhat(nG, A, B, 0.0);
    S->mmax = mmax > 0 ? mmax : orc_mmax_default(nG, A, B, L);
    S->nlat = orc_lattice_count(S->mmax);
    S->n3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)S->nlat);
    S->start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)S->mmax + 2));
    orc_lattice_build(S->mmax, S->n3, S->start);
    S->shell_m = (int32_t *)malloc(sizeof(int32_t) * ((size_t)S->mmax + 1));
    S->cdf = (double *)malloc(sizeof(double) * ((size_t)S->mmax + 1));
    S->shell_coef = (double *)malloc(sizeof(double) * ((size_t)S->mmax + 1));
    S->nshell = shell_table_k(S->mmax, S->start, nG, A, B, L, density, kT, q2, &S->kern, P, S->shell_m,
                              S->cdf, S->shell_coef);
    return S;
}

/* A system in a box of edges Lb[3].  Equal edges give orc_sys_create_k's
 * system; a cuboid samples point by point (orc_box_lattice, the point
 * tables, orc_box_draw) and requires mmax = 0 (the default truncation).
 * NULL for bad arguments or a lattice beyond |n_d| = 511. */
orc_sys *orc_sys_create_box(int64_t N, const double *Lb, int nY, const double *ya, const double *yl, double rc,
                            double kT, int P, int mmax, uint64_t seed, uint32_t replica, int density, int full_k,
                            int nG, const double *c, const double *s, const double *A, const double *B,
                            const double *q, const double *m)
{
    if (Lb[0] == Lb[1] && Lb[1] == Lb[2])
        return orc_sys_create_k(N, Lb[0], nY, ya, yl, rc, kT, P, mmax, seed, replica, density, full_k, nG, c, s, A,
                                B, q, m);
    orc_kern K;
    if (nG < 1 || nG > 64 || mmax != 0 || kern_make(nY, ya, yl, &K) != 0) return NULL;
    for (int d = 0; d < 3; ++d)
        if (!(Lb[d] > 0.0)) return NULL;
    int64_t cnt = orc_box_lattice(Lb, nG, A, B, NULL, NULL);
    if (cnt < 1) return NULL;
    orc_sys *S = (orc_sys *)calloc(1, sizeof(orc_sys));
    S->N = N; S->L = Lb[0]; S->V = Lb[0] * Lb[1] * Lb[2]; S->lambda = yl[0]; S->kern = K; S->rc = rc; S->kT = kT;
    S->Lb[0] = Lb[0]; S->Lb[1] = Lb[1]; S->Lb[2] = Lb[2];
    S->cuboid = 1;
    S->P = P; S->density = density; S->full_k = full_k; S->nG = nG;
    S->seed = seed; S->replica = replica; S->q = q; S->m = m;
    memcpy(S->c, c, sizeof(double) * nG); memcpy(S->s, s, sizeof(double) * nG);
    memcpy(S->A, A, sizeof(double) * nG); memcpy(S->B, B, sizeof(double) * nG);
    double q1 = 0.0, q2 = 0.0;
    for (int64_t i = 0; i < N; ++i) { q1 += q[i]; q2 += q[i] * q[i]; }
    S->Q1 = q1; S->Q2 = q2;
    S->F0 = 0.0; for (int j = 0; j < nG; ++j) S->F0 += c[j];
    S->Fhat0 = orc_Fhat(nG, A, B, 0.0);
    S->mmax = 0;
    S->nlat = cnt;
    S->nshell = (int)cnt;
    S->n3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)cnt);
    double *k2 = (double *)malloc(sizeof(double) * (size_t)cnt);
    orc_box_lattice(Lb, nG, A, B, S->n3, k2);
    S->cdf = (double *)malloc(sizeof(double) * (size_t)cnt);
    S->shell_coef = (double *)malloc(sizeof(double) * (size_t)cnt);
    box_tables(cnt, k2, nG, A, B, S->V, density, kT, q2, &K, P, S->cdf, S->shell_coef);
    free(k2);
    return S;
}

void orc_sys_destroy(orc_sys *S)
{
    if (!S) return;
    free(S->n3); free(S->start); free(S->shell_m); free(S->cdf); free(S->shell_coef); free(S->cdf_q);
    free(S);
}

int orc_sys_mmax(const orc_sys *S) { return S->mmax; }
int orc_sys_nshell(const orc_sys *S) { return S->nshell; }
int64_t orc_sys_nlat(const orc_sys *S) { return S->nlat; }
void orc_sys_tables(const orc_sys *S, int32_t *shell_m, double *cdf, double *coef)
{
    if (S->shell_m) memcpy(shell_m, S->shell_m, sizeof(int32_t) * S->nshell);
    else memset(shell_m, 0, sizeof(int32_t) * S->nshell); /* a cuboid: one entry per lattice point */
    memcpy(cdf, S->cdf, sizeof(double) * S->nshell);
    memcpy(coef, S->shell_coef, sizeof(double) * S->nshell);
}
void orc_sys_lattice(const orc_sys *S, int32_t *n3, int64_t *start)
{
    memcpy(n3, S->n3, sizeof(int32_t) * 3 * (size_t)S->nlat);
    if (S->start) memcpy(start, S->start, sizeof(int64_t) * ((size_t)S->mmax + 2));
}

/* The draws of force-evaluation index `step`: i.i.d. (sampler 0) or the next P
 * states of the Metropolis-Hastings chain (sampler 1, which advances it). */
void orc_sys_draw(orc_sys *S, uint64_t step, int32_t *n_out, double *coef_out)
{
    if (S->cuboid)
        orc_box_draw(S->P, step, S->seed, S->replica, S->nlat, S->cdf, S->shell_coef, S->n3, n_out, coef_out);
    else if (S->sampler == 1)
        orc_mh_draw(S->P, step, S->seed, S->replica, S->nshell, S->shell_m, S->cdf_q, S->shell_coef, S->start,
                    S->n3, S->mh_state, n_out, coef_out);
    else
        orc_draw(S->P, step, S->seed, S->replica, S->nshell, S->shell_m, S->cdf, S->shell_coef, S->start, S->n3,
                 n_out, coef_out);
}

/* Selects the sampler: 0 i.i.d. inverse-CDF draws, 1 the Metropolis-Hastings
 * chain of orc_mh_draw (its proposal table is built here and the chain
 * emptied).  Returns 0, or -1 for another value. */
int orc_sys_set_sampler(orc_sys *S, int sampler)
{
    if (sampler != 0 && sampler != 1) return -1;
    if (sampler == 1 && S->cuboid) return -1; /* the chain's proposals are drawn by shell */
    S->sampler = sampler;
    S->mh_state[0] = 0;
    S->mh_state[1] = -1;
    if (sampler == 1 && !S->cdf_q) {
        S->cdf_q = (double *)malloc(sizeof(double) * ((size_t)S->mmax + 1));
        int32_t *m_tmp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)S->mmax + 1));
        double *c_tmp = (double *)malloc(sizeof(double) * ((size_t)S->mmax + 1));
        shell_table_k(S->mmax, S->start, S->nG, S->A, S->B, S->L, ORC_FLAT, S->kT, S->Q2, &S->kern, S->P, m_tmp,
                      S->cdf_q, c_tmp);
        free(m_tmp);
        free(c_tmp);
    }
    return 0;
}

/* One force evaluation at force-evaluation index `step` (the force step of
 * Algorithm 2).  f (SoA) receives near + far forces; f_near (nullable) the near part
 * alone.  energy[8] (nullable) = { U_N, U_F (estimator, or the full sum in
 * full-k mode), U_k0, U_self, U_bg, 0, W_N, W_F (estimator, or the full
 * sum) }, where
 *   U_k0   = Fhat(0) (sum q)^2 / (2V)  -- the k = 0 mode of eq. (3.5), excluded
 *            from sampling and added deterministically;
 *   U_self = -1/2 sum q_i^2 F(0)       -- Section 4.1;
 *   U_bg   = -(sum q)^2 4 pi lambda^2 / (2V) -- the uniform neutralising
 *            background's interaction energy (constant, no force; 4 pi
 *            lambda^2 is the kernel's integral over space, the same for the
 *            Yukawa and the EGS kernel);
 *   W_N, W_F = the virials -3V dU/dV of the near and far parts (orc_near,
 *            orc_far_rb_virial); U_k0 and U_bg scale as 1/V, so their
 *            virials are 3 U_k0 and 3 U_bg, and U_self has none. */
void orc_sys_force(orc_sys *S, uint64_t step, const double *x, double *f, double *f_near, double *energy)
{
    int64_t N = S->N;
    double UN = 0.0, UF = 0.0, WN = 0.0, WF = 0.0;
    near_box(N, x, S->q, S->Lb, S->kern, S->rc, S->nG, S->c, S->s, f, &UN, &WN);
    if (f_near) memcpy(f_near, f, sizeof(double) * 3 * (size_t)N);
    if (S->full_k) {
        if (S->cuboid) UF = orc_far_full_box(N, x, S->q, S->Lb, S->nG, S->A, S->B, f, &WF);
        else UF = orc_far_full(N, x, S->q, S->L, S->nG, S->A, S->B, S->mmax, f, &WF);
    } else {
        int32_t *n = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)S->P);
        double *coef = (double *)malloc(sizeof(double) * (size_t)S->P);
        double *rho = (double *)malloc(sizeof(double) * 2 * (size_t)S->P);
        orc_sys_draw(S, step, n, coef);
        orc_rho_box(N, x, S->q, S->Lb, S->P, n, rho);
        orc_far_rb_box(N, x, S->q, S->Lb, S->P, n, coef, rho, f);
        UF = orc_far_rb_energy(S->P, coef, rho);
        WF = orc_far_rb_virial_box(S->P, n, coef, rho, S->Lb, S->nG, S->A, S->B);
        free(n); free(coef); free(rho);
    }
    if (energy) {
        energy[0] = UN;
        energy[1] = UF;
        energy[2] = S->Fhat0 * S->Q1 * S->Q1 / (2.0 * S->V);
        energy[3] = -0.5 * S->Q2 * S->F0;
        energy[4] = -(S->Q1 * S->Q1) * (4.0 * ORC_PI * kern_l2(&S->kern)) / (2.0 * S->V);
        energy[5] = 0.0;
        energy[6] = WN;
        energy[7] = WF;
    }
}

static double kinetic(const orc_sys *S, const double *v)
{
    int64_t N = S->N;
    double ke = 0.0;
    for (int64_t i = 0; i < N; ++i)
        ke += 0.5 * S->m[i] * (v[i] * v[i] + v[N + i] * v[N + i] + v[2 * N + i] * v[2 * N + i]);
    return ke;
}

/* Velocity-Verlet (Algorithm 2, last line; Section 5.1), with f = F(x, step0)
 * on entry.  For each of nsteps steps n = 0..nsteps-1:
 *   v += (dt/2) f / m;   x += dt v;   wrap x into [0, L);
 *   f = F(x, step0 + n + 1);   v += (dt/2) f / m.
 * With a Langevin thermostat (friction g > 0, bath k_B T) the drift becomes the
 * BAOAB splitting's A-O-A: x += (dt/2) v;  v = c v + sqrt((1 - c^2) k_B T / m) z
 * with c = exp(-g dt) and z the particle's normals for force index
 * step0 + n + 1 (orc_langevin_normals);  x += (dt/2) v. 
 * ehist (nullable) receives [nsteps][8] energy rows of the new state
 * (orc_sys_force's, with KE in slot 5).  Returns 0, or -1 if a particle moved a full box length. */
/* The three normal deviates of particle i (caller index) for the thermostat
 * step into force index `step`: Philox4x64-10(counter = (i, step, 1, 0), key
 * = (seed, replica)) gives four uniforms u_k = ((w_k >> 11) + 1) 2^-53 in
 * (0, 1], and the Box-Muller transform z0 + i z1 = sqrt(-2 ln u0) e^{2 pi i u1},
 * z2 = sqrt(-2 ln u2) cos(2 pi u3) (counter word 2 = 1 keeps these apart from
 * the mode draws, whose word 2 is 0). */
void orc_langevin_normals(uint64_t i, uint64_t step, uint64_t seed, uint32_t replica, double z[3])
{
    uint64_t ctr[4] = {i, step, 1, 0}, key[2] = {seed, (uint64_t)replica}, w[4];
    orc_philox4x64_10(ctr, key, w);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = (double)((w[k] >> 11) + 1) * 0x1p-53;
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(2.0 * ORC_PI * u[1]);
    z[1] = r0 * sin(2.0 * ORC_PI * u[1]);
    z[2] = r1 * cos(2.0 * ORC_PI * u[3]);
}

/* Langevin thermostat for Algorithm 2's time loop: friction (per unit time)
 * and bath temperature; friction 0 turns it off (and any global bath). */
void orc_sys_set_langevin(orc_sys *S, double friction, double bath_kT)
{
    S->friction = friction;
    S->bath_kT = bath_kT;
    S->bath = 0;
}

/* The global baths of the time loop (Section 5.1 equilibrates in the NVT
 * ensemble with Nose-Hoover dynamics; Berendsen's weak coupling is the other
 * global scheme), each applied as a half-step operator T(dt/2) before and
 * after every velocity-Verlet step (a symmetric Trotter splitting of the
 * thermostatted equations), with g = 3N degrees of freedom and tau = 1/rate:
 *   Nose-Hoover (one thermostat, mass Q = g kT tau^2):
 *     xi += (dt/4)(2K - g kT)/Q;  v *= e^{-xi dt/2} (K *= e^{-xi dt});
 *     eta += (dt/2) xi;  xi += (dt/4)(2K - g kT)/Q;
 *     the extended energy K + U + Q xi^2/2 + g kT eta is conserved;
 *   Berendsen: lambda^2 = 1 + (dt/(2 tau))(g kT/(2K) - 1), v *= lambda
 *     (K *= lambda^2; lambda = 1 when K = 0), relaxing K to g kT/2 at rate
 *     1/tau.
 * K is the kinetic energy.  kind 2 or 3 (0 switches every bath off); rate and
 * bath_kT positive.  xi and eta restart at 0.  Returns 0, or -1. */
int orc_sys_set_bath(orc_sys *S, int kind, double rate, double bath_kT)
{
    if (kind == 0) {
        S->bath = 0;
        S->friction = 0.0;
        return 0;
    }
    if ((kind != 2 && kind != 3) || !(rate > 0.0) || !(bath_kT > 0.0)) return -1;
    S->bath = kind;
    S->bath_rate = rate;
    S->bath_kT = bath_kT;
    S->friction = 0.0;
    S->xi = 0.0;
    S->eta = 0.0;
    return 0;
}

void orc_sys_bath_state(const orc_sys *S, double out[2])
{
    out[0] = S->xi;
    out[1] = S->eta;
}

/* One half-step operator T(dt/2) of a global bath on kinetic energy *K;
 * returns the factor the velocities are scaled by and updates *K. */
static double bath_half(orc_sys *S, double dt, double *K)
{
    double g = 3.0 * (double)S->N, gkT = g * S->bath_kT;
    if (S->bath == 2) {
        double tau = 1.0 / S->bath_rate, Q = gkT * tau * tau;
        S->xi += 0.25 * dt * (2.0 * *K - gkT) / Q;
        double sc = exp(-0.5 * dt * S->xi);
        *K = *K * (sc * sc);
        S->eta += 0.5 * dt * S->xi;
        S->xi += 0.25 * dt * (2.0 * *K - gkT) / Q;
        return sc;
    }
    if (!(*K > 0.0)) return 1.0;
    double lam2 = 1.0 + 0.5 * dt * S->bath_rate * (gkT / (2.0 * *K) - 1.0);
    if (lam2 < 0.0) lam2 = 0.0;
    *K = *K * lam2;
    return sqrt(lam2);
}

static void scale_v(const orc_sys *S, double *v, double sc)
{
    for (int64_t k = 0; k < 3 * S->N; ++k) v[k] *= sc;
}

int orc_sys_run(orc_sys *S, double *x, double *v, double *f, uint64_t step0, int nsteps, double dt,
                double *ehist)
{
    int64_t N = S->N;
    int bad = 0;
    const double c1 = exp(-S->friction * dt);
    const int global = S->bath == 2 || S->bath == 3;
    double K = 0.0;
    if (global && nsteps > 0) { /* the first step's opening half-step */
        K = kinetic(S, v);
        scale_v(S, v, bath_half(S, dt, &K));
    }
    for (int n = 0; n < nsteps; ++n) {
        for (int64_t i = 0; i < N; ++i) {
            double hm = (0.5 * dt) / S->m[i];
            double z[3] = {0.0, 0.0, 0.0}, sig = 0.0;
            if (S->friction > 0.0) {
                orc_langevin_normals((uint64_t)i, step0 + (uint64_t)n + 1, S->seed, S->replica, z);
                sig = sqrt((1.0 - c1 * c1) * S->bath_kT / S->m[i]);
            }
            for (int d = 0; d < 3; ++d) {
                double vv = v[d * N + i] + hm * f[d * N + i];
                double dx;
                if (S->friction > 0.0) {
                    /* BAOAB: half drift, Ornstein-Uhlenbeck velocity update, half drift */
                    double v2 = c1 * vv + sig * z[d];
                    dx = 0.5 * dt * vv + 0.5 * dt * v2;
                    vv = v2;
                } else {
                    dx = dt * vv;
                }
                const double Ld = S->Lb[d];
                if (fabs(dx) >= Ld) bad = 1;
                double xx = x[d * N + i] + dx;
                if (xx >= Ld) xx -= Ld;
                if (xx < 0.0) xx += Ld;
                if (xx >= Ld) xx = 0.0;
                v[d * N + i] = vv;
                x[d * N + i] = xx;
            }
        }
        double e[8];
        orc_sys_force(S, step0 + (uint64_t)n + 1, x, f, NULL, e);
        for (int64_t i = 0; i < N; ++i) {
            double hm = (0.5 * dt) / S->m[i];
            for (int d = 0; d < 3; ++d) v[d * N + i] = v[d * N + i] + hm * f[d * N + i];
        }
        if (global) { /* closing half-step, then the next step's opening one */
            K = kinetic(S, v);
            scale_v(S, v, bath_half(S, dt, &K));
            if (ehist) e[5] = K;
            if (n + 1 < nsteps) scale_v(S, v, bath_half(S, dt, &K));
        } else if (ehist) {
            e[5] = kinetic(S, v);
        }
        if (ehist) memcpy(ehist + 8 * (size_t)n, e, sizeof(e));
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Observables of Section 5.1: static structure factor and pair distribution  */
/* ------------------------------------------------------------------------- */

/* Shell means of the weighted structure factor over every lattice mode with
 * 1 <= |n|^2 <= mmax:  s_out[m] = (1/cnt_m) sum_{|n|^2 = m} |sum_j w_j e^{ik.r_j}|^2,
 * k = 2 pi n / L, cnt_m the modes of shell m (s_out[m] = 0 where there are
 * none, and for m = 0).  With unit weights S(k) = s_out / N, the static
 * structure factor <rho(k) rho(-k)> / N. */
void orc_ssf(int64_t N, const double *x, const double *w, double L, int mmax, double *s_out)
{
    int64_t cnt = orc_lattice_count(mmax);
    int32_t *n3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(cnt > 0 ? cnt : 1));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)mmax + 2));
    orc_lattice_build(mmax, n3, start);
    double t = (2.0 * ORC_PI) / L;
    double *r2 = (double *)malloc(sizeof(double) * (size_t)(cnt > 0 ? cnt : 1));
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < cnt; ++p) {
        double kx = t * n3[3 * p], ky = t * n3[3 * p + 1], kz = t * n3[3 * p + 2];
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double th = kx * x[j] + ky * x[N + j] + kz * x[2 * N + j];
            re += w[j] * cos(th);
            im += w[j] * sin(th);
        }
        r2[p] = re * re + im * im;
    }
    for (int m = 0; m <= mmax; ++m) {
        double acc = 0.0;
        for (int64_t p = start[m]; p < start[m + 1]; ++p) acc += r2[p];
        s_out[m] = start[m + 1] > start[m] ? acc / (double)(start[m + 1] - start[m]) : 0.0;
    }
    free(n3); free(start); free(r2);
}

/* Histogram of ordered pairs (i, j), i != j, by minimum-image distance r <
 * r_max (r_max <= L/2, so at most one image counts): bin floor(r / dr), dr =
 * r_max / nbins, added into counts[nbins].  g(r) of bin b is counts[b] /
 * (N (N/V) 4/3 pi ((b+1)^3 - b^3) dr^3).  A pair whose r / dr lies within
 * 1e-9 of a bin edge could fall on either side under another rounding of the
 * same arithmetic: it is also counted into amb[] of both adjacent bins. */
void orc_rdf_box(int64_t N, const double *x, const double *Lb, double r_max, int nbins, int64_t *counts,
                 int64_t *amb);

void orc_rdf(int64_t N, const double *x, double L, double r_max, int nbins, int64_t *counts, int64_t *amb)
{
    const double Lb[3] = {L, L, L};
    orc_rdf_box(N, x, Lb, r_max, nbins, counts, amb);
}

/* orc_rdf in a box of edges Lb[3] (r_max <= L_d/2 on every axis). */
void orc_rdf_box(int64_t N, const double *x, const double *Lb, double r_max, int nbins, int64_t *counts,
                 int64_t *amb)
{
    double dr = r_max / nbins;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double r2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                double u = x[d * N + i] - x[d * N + j];
                u -= Lb[d] * floor(u / Lb[d] + 0.5);
                r2 += u * u;
            }
            double r = sqrt(r2);
            if (!(r < r_max)) continue;
            double y = r / dr;
            int b = (int)floor(y);
            if (b >= nbins) b = nbins - 1;
            counts[b] += 1;
            double e = floor(y + 0.5);
            if (fabs(y - e) < 1e-9) {
                int hi = (int)e;
                if (hi - 1 >= 0 && hi - 1 < nbins) amb[hi - 1] += 1;
                if (hi >= 0 && hi < nbins) amb[hi] += 1;
            }
        }
}

/* Unwrapped displacement between two snapshots of the wrapped positions:
 * disp += (x - x_last) - L rint((x - x_last)/L), the minimum image (each
 * particle must have moved less than L/2 in between), then x_last = x. */
void orc_track(int64_t N, double L, const double *x, double *x_last, double *disp)
{
    for (int64_t k = 0; k < 3 * N; ++k) {
        double d = x[k] - x_last[k];
        d = d - L * rint(d / L);
        disp[k] += d;
        x_last[k] = x[k];
    }
}

/* orc_track in a cuboid box of edges Lb[3]: the minimum image along each
 * axis with that axis's edge. */
void orc_track_box(int64_t N, const double *Lb, const double *x, double *x_last, double *disp)
{
    for (int a = 0; a < 3; ++a)
        for (int64_t i = 0; i < N; ++i) {
            const int64_t k = a * N + i;
            double d = x[k] - x_last[k];
            d = d - Lb[a] * rint(d / Lb[a]);
            disp[k] += d;
            x_last[k] = x[k];
        }
}

/* Mean squared displacement (1/N) sum_i |disp_i|^2 and velocity
 * autocorrelation (1/N) sum_i v0_i . v_i (Section 5.1's MSD and VACF at one
 * time lag), in particle order. */
void orc_msd_vacf(int64_t N, const double *disp, const double *v0, const double *v, double out[2])
{
    double msd = 0.0, vacf = 0.0;
    for (int64_t i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            msd += disp[d * N + i] * disp[d * N + i];
            vacf += v0[d * N + i] * v[d * N + i];
        }
    out[0] = msd / (double)N;
    out[1] = vacf / (double)N;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

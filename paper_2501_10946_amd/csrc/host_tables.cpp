// Host side of the importance-sampling measure (Section 4.3, eq. 3.124):
// the Fourier lattice and the per-shell cumulative weights of
// P(k) = F(k) Fhat(k) / S.  Built with -ffp-contract=off: the cumulative
// weights are a fixed sequence of IEEE FP64 operations, so two conforming
// implementations produce the same bits and therefore the same samples.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace rbsog {
namespace {

constexpr double kPi = 3.141592653589793;

}  // namespace

// Fhat(k^2) = sum_j A_j exp(-B_j k^2), ascending j.
double fhat(const rbsog_sog &s, double k2)
{
    double acc = 0.0;
    for (int j = 0; j < s.n; ++j) acc += s.A[j] * std::exp(-s.B[j] * k2);
    return acc;
}

// The virial -3V dU/dV of the far part scales the configuration with the box:
// rho(k) is unchanged, 1/V gives 3 U_F, and each k^2 = (2 pi / L)^2 m moves as
// V^(-2/3), which adds -(1/V) sum_k k^2 G(k^2) |rho|^2 with G = -dFhat/d(k^2)
// = sum_j A_j B_j exp(-B_j k^2).  A mode's term is therefore its energy term
// times 2 (3/2 - vm), vm = k^2 G / Fhat; vm depends on |n|^2 = m only.
void virial_table(const rbsog_sog &s, double L, int mmax, double *vm)
{
    const double t = (2.0 * kPi) / L;
    for (int m = 0; m <= mmax; ++m) {
        const double k2 = t * t * (double)m;
        double F = 0.0, G = 0.0;
        for (int j = 0; j < s.n; ++j) {
            const double e = std::exp(-s.B[j] * k2);
            F += s.A[j] * e;
            G += s.A[j] * s.B[j] * e;
        }
        vm[m] = F > 0.0 ? k2 * G / F : 0.0;
    }
}

// Correction factor of the measure.  ADAPTIVE is the leading Debye-Hueckel
// term of eq. (3.22) as printed, with eps(k)^{-1}/k^2 the kernel's Yhat(k) /
// (4 pi): lambda^2/(1 + lambda^2 k^2) for the Yukawa dielectric eps(k) = 1 +
// (lambda k)^{-2}, the sum of its two terms' for the EGS dielectric.
double density(int kind, double kT, double V, double Q2, const KernelTerms &K, double k2)
{
    if (kind == RBSOG_FLAT) return 1.0;
    if (kind == RBSOG_K2) return k2;
    double g = 0.0;
    for (int t = 0; t < K.n; ++t) {
        const double l2 = K.l[t] * K.l[t];
        g += K.a[t] * l2 / (1.0 + l2 * k2);
    }
    if (kind == RBSOG_DH4PI) return (kT * V) / ((kT * V) / Q2 + 4.0 * kPi * g);
    return (kT * V) / ((kT * V) / Q2 + g);
}

// Largest m >= 1 with Fhat((2 pi/L)^2 m) >= 1e-16 Fhat(0).
int default_mmax(const rbsog_sog &s, double L)
{
    double t = (2.0 * kPi) / L;
    double tk2 = t * t;
    double floor_val = 1e-16 * fhat(s, 0.0);
    int m = 1;
    while (m < kMaxLatticeM && fhat(s, tk2 * (double)(m + 1)) >= floor_val) ++m;
    return m;
}

namespace {

// Process-wide cache of the packed lattice for the largest m_max built so far:
// all n with 1 <= |n|^2 <= m_max sorted by (|n|^2, nx, ny, nz), and the shell
// sizes r3(m).  The list of a smaller m_max is a prefix of this one, so every
// system (and every replica of an ensemble) reads the same table.
struct LatticeCache {
    std::mutex mu;
    int mmax = 0;
    std::vector<int32_t> packed;
    std::vector<int64_t> size;    // [mmax + 1]
    std::vector<int64_t> first;   // [mmax + 1] index of the shell's first point
};
LatticeCache g_lat;

void grow_cache(int mmax)
{
    LatticeCache &c = g_lat;
    int R = (int)std::sqrt((double)mmax) + 1;
    std::vector<int64_t> size(mmax + 1, 0);
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int cc = -R; cc <= R; ++cc) {
                int64_t m = (int64_t)a * a + (int64_t)b * b + (int64_t)cc * cc;
                if (m >= 1 && m <= mmax) ++size[m];
            }
    std::vector<int64_t> first(mmax + 1, 0);
    int64_t run = 0;
    for (int m = 1; m <= mmax; ++m) {
        first[m] = run;
        run += size[m];
    }
    std::vector<int32_t> packed((size_t)run, 0);
    // lexicographic (nx, ny, nz) enumeration fills each shell in sorted order
    std::vector<int64_t> fill(first);
    for (int a = -R; a <= R; ++a)
        for (int b = -R; b <= R; ++b)
            for (int cc = -R; cc <= R; ++cc) {
                int64_t m = (int64_t)a * a + (int64_t)b * b + (int64_t)cc * cc;
                if (m < 1 || m > mmax) continue;
                packed[(size_t)fill[m]++] = (int32_t)((uint32_t)(a + kLatticeBias) |
                                                      ((uint32_t)(b + kLatticeBias) << 10) |
                                                      ((uint32_t)(cc + kLatticeBias) << 20));
            }
    c.mmax = mmax;
    c.packed.swap(packed);
    c.size.swap(size);
    c.first.swap(first);
}

}  // namespace

int64_t lattice_points(int mmax)
{
    std::lock_guard<std::mutex> lock(g_lat.mu);
    if (g_lat.mmax < mmax) grow_cache(mmax);
    return g_lat.first[mmax] + g_lat.size[mmax];
}

void lattice_copy(int mmax, int32_t *out)
{
    std::lock_guard<std::mutex> lock(g_lat.mu);
    if (g_lat.mmax < mmax) grow_cache(mmax);
    int64_t n = g_lat.first[mmax] + g_lat.size[mmax];
    std::copy(g_lat.packed.begin(), g_lat.packed.begin() + n, out);
}

// k^2 of lattice point n in a box of edges Lb: (2 pi / L)^2 |n|^2 in a cube (as
// the shell tables form it), else the sum over the axes of (2 pi n_d / L_d)^2.
double box_k2(const double Lb[3], int nx, int ny, int nz)
{
    if (Lb[0] == Lb[1] && Lb[1] == Lb[2]) {
        const double t = (2.0 * kPi) / Lb[0];
        const double m = (double)nx * nx + (double)ny * ny + (double)nz * nz;
        return t * t * m;
    }
    const double kx = (2.0 * kPi) * nx / Lb[0], ky = (2.0 * kPi) * ny / Lb[1], kz = (2.0 * kPi) * nz / Lb[2];
    return kx * kx + ky * ky + kz * kz;
}

namespace {

struct BoxPoint {
    double k2;
    int n[3];
};

// The lattice of a cuboid: every n != 0 with Fhat(k^2) >= 1e-16 Fhat(0), sorted
// by (k^2, nx, ny, nz).  False when some |n_d| would exceed 511 (the packing).
bool box_points(const rbsog_sog &s, const double Lb[3], std::vector<BoxPoint> *out)
{
    const double thr = 1e-16 * fhat(s, 0.0);
    double lo = 0.0, hi = 1.0;
    while (fhat(s, hi) >= thr) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {   // the k^2 where Fhat crosses the threshold
        const double mid = 0.5 * (lo + hi);
        if (fhat(s, mid) >= thr) lo = mid; else hi = mid;
    }
    int nm[3];
    for (int d = 0; d < 3; ++d) {
        nm[d] = (int)std::floor(Lb[d] * std::sqrt(hi) / (2.0 * kPi)) + 1;
        if (nm[d] > 511) return false;
    }
    out->clear();
    for (int a = -nm[0]; a <= nm[0]; ++a)
        for (int b = -nm[1]; b <= nm[1]; ++b)
            for (int c = -nm[2]; c <= nm[2]; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const double k2 = box_k2(Lb, a, b, c);
                if (!(fhat(s, k2) >= thr)) continue;
                out->push_back(BoxPoint{k2, {a, b, c}});
            }
    std::sort(out->begin(), out->end(), [](const BoxPoint &x, const BoxPoint &y) {
        if (x.k2 != y.k2) return x.k2 < y.k2;
        if (x.n[0] != y.n[0]) return x.n[0] < y.n[0];
        if (x.n[1] != y.n[1]) return x.n[1] < y.n[1];
        return x.n[2] < y.n[2];
    });
    return true;
}

}  // namespace

int64_t box_lattice_points(const rbsog_sog &s, const double Lb[3])
{
    std::vector<BoxPoint> pts;
    if (!box_points(s, Lb, &pts)) return -1;
    return (int64_t)pts.size();
}

void build_tables(const rbsog_sog &s, const rbsog_params &p, double Q2, int mmax, Tables *t, bool with_lattice)
{
    double Lb[3];
    box_edges(&p, Lb);
    if (!(Lb[0] == Lb[1] && Lb[1] == Lb[2])) {
        // a cuboid: every lattice point its own shell (the measure depends on
        // k^2, which no longer groups by |n|^2)
        std::vector<BoxPoint> pts;
        box_points(s, Lb, &pts);
        const double V = Lb[0] * Lb[1] * Lb[2];
        t->mmax = 0;
        t->nlat = (int64_t)pts.size();
        t->packed.clear();
        t->cdf.clear();
        t->coef.clear();
        t->shell_first.clear();
        t->shell_size.clear();
        std::vector<double> Fk_of;
        double acc = 0.0;
        for (size_t i = 0; i < pts.size(); ++i) {
            const BoxPoint &q = pts[i];
            if (with_lattice)
                t->packed.push_back((int32_t)((uint32_t)(q.n[0] + kLatticeBias) |
                                              ((uint32_t)(q.n[1] + kLatticeBias) << 10) |
                                              ((uint32_t)(q.n[2] + kLatticeBias) << 20)));
            const double Fk = density(p.density, p.kT, V, Q2, kernel_terms(s), q.k2);
            acc = acc + Fk * fhat(s, q.k2);
            t->cdf.push_back(acc);
            t->shell_first.push_back((int32_t)i);
            t->shell_size.push_back(1);
            Fk_of.push_back(Fk);
        }
        t->nshell = (int)t->cdf.size();
        t->S = acc;
        for (int i = 0; i < t->nshell; ++i) t->coef.push_back(t->S / ((double)p.P * V * Fk_of[i]));
        return;
    }
    t->mmax = mmax;
    std::vector<int64_t> size, first;
    {
        std::lock_guard<std::mutex> lock(g_lat.mu);
        if (g_lat.mmax < mmax) grow_cache(mmax);
        size.assign(g_lat.size.begin(), g_lat.size.begin() + mmax + 1);
        first.assign(g_lat.first.begin(), g_lat.first.begin() + mmax + 1);
        t->nlat = first[mmax] + size[mmax];
        if (with_lattice) t->packed.assign(g_lat.packed.begin(), g_lat.packed.begin() + t->nlat);
        else t->packed.clear();
    }
    // cumulative shell weights
    double tt = (2.0 * kPi) / p.L;
    double tk2 = tt * tt;
    double V = p.L * p.L * p.L;
    t->cdf.clear();
    t->coef.clear();
    t->shell_first.clear();
    t->shell_size.clear();
    std::vector<double> Fk_of;
    double acc = 0.0;
    for (int m = 1; m <= mmax; ++m) {
        if (size[m] == 0) continue;
        double k2 = tk2 * (double)m;
        double Fk = density(p.density, p.kT, V, Q2, kernel_terms(s), k2);
        double W = Fk * fhat(s, k2);
        acc = acc + (double)size[m] * W;
        t->cdf.push_back(acc);
        t->shell_first.push_back((int32_t)first[m]);
        t->shell_size.push_back((int32_t)size[m]);
        Fk_of.push_back(Fk);
    }
    t->nshell = (int)t->cdf.size();
    t->S = acc;
    for (int i = 0; i < t->nshell; ++i) t->coef.push_back(t->S / ((double)p.P * V * Fk_of[i]));
}

// (sin, cos)(2 pi j / n), j < n: 2 pi j / n is within an ulp of the exact
// angle; the quarter turns are set exactly so that they carry no rounding
static void rotation_table(double *out, int n)
{
    const double two_pi = 6.283185307179586;
    for (int j = 0; j < n; ++j) {
        double a = two_pi * (double)j / (double)n;
        double s = std::sin(a), c = std::cos(a);
        if (j == n / 4) { s = 1.0; c = 0.0; }
        if (j == n / 2) { s = 0.0; c = -1.0; }
        if (j == 3 * n / 4) { s = -1.0; c = 0.0; }
        out[2 * j] = s;
        out[2 * j + 1] = c;
    }
}

void phase_table(double out[2 * kPhaseTable]) { rotation_table(out, kPhaseTable); }

void far_table(double out[2 * kFarTable]) { rotation_table(out, kFarTable); }

void charge_sums(const double *q, int64_t N, double *q1, double *q2)
{
    double a = 0.0, b = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        a += q[i];
        b += q[i] * q[i];
    }
    *q1 = a;
    *q2 = b;
}

}  // namespace rbsog

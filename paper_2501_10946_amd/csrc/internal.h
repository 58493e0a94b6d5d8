// Internal declarations shared by the host code and the kernel launchers of
// librbsog.  Nothing here is part of the C-ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rbsog.h"

namespace rbsog {

// thread-local error message behind rbsog_last_error()
int fail(int code, const char *fmt, ...);

// ---- host: the kernel's Yukawa terms ----------------------------------------
// Y(r) = sum_{t < n} a[t] e^{-r/l[t]}/r: the Yukawa kernel (n = 1, a = 1,
// l = lambda) or the two terms of the EGS kernel (nyuk = 2), longest first.
struct KernelTerms {
    int n;
    double a[2], l[2];
};
inline KernelTerms kernel_terms(const rbsog_sog &s)
{
    if (s.nyuk == 2) return KernelTerms{2, {s.ya[0], s.ya[1]}, {s.yl[0], s.yl[1]}};
    return KernelTerms{1, {1.0, 0.0}, {s.lambda, 1.0}};
}

// ---- host: Algorithm 1 (host_sog.cpp) --------------------------------------
double step_size(double eps, double delta);
int c1_start(double lambda, double rc, double h, int M1, int M2, double *t0, double *w);
void expand(rbsog_sog *s);
double sog_max_error(const rbsog_sog &s);

// ---- host: the near-field pair function as a polynomial (host_near.cpp) ----
// H(r) = r^3 [F_N1 + F_N2](r) and K(r) = r (Y(r) - F(r)) on [0, r_c] as
// polynomials in y = 2 r / r_c - 1 (ascending powers, kNearPolyDeg + 1 of
// them) of the lowest degree of kNearPolyDegs at which both are within
// kNearPolyTol (absolute; H(0) = K(0) = 1), the powers above it zero; returns
// that degree, 0 when none is accurate enough.
constexpr int kNearPolyDeg = 28;
constexpr int kNearPolyDegs[3] = {24, 26, 28};
constexpr double kNearPolyTol = 1e-15;
int near_poly(const rbsog_sog &s, double rc, double h_out[kNearPolyDeg + 1], double k_out[kNearPolyDeg + 1]);

// ---- host: Fourier lattice and sampling tables (host_tables.cpp) -----------
// Lattice vectors are packed into one int32: (nx+512) | (ny+512)<<10 | (nz+512)<<20.
constexpr int kLatticeBias = 512;
constexpr int kMaxLatticeM = 511 * 511;

struct Tables {
    int mmax = 0;
    int64_t nlat = 0;
    int nshell = 0;
    double S = 0.0;
    std::vector<int32_t> packed;       // [nlat], sorted by (|n|^2, nx, ny, nz)
    std::vector<double> cdf;           // [nshell] running sum of shell weights
    std::vector<double> coef;          // [nshell] S / (P V F(k^2))
    std::vector<int32_t> shell_first;  // [nshell] index of the shell's first point
    std::vector<int32_t> shell_size;   // [nshell] points in the shell, r3(m)
};

int default_mmax(const rbsog_sog &s, double L);
// points of the lattice up to m_max, and a copy of its packed list (both from
// a process-wide cache that grows to the largest m_max asked for)
int64_t lattice_points(int mmax);
void lattice_copy(int mmax, int32_t *out);
// the correction factor of the sampling measure (eq. 3.124) for the kernel's
// terms (the first term of eq. 3.22 with eps(k)^{-1}/k^2 = sum_t a_t l_t^2 /
// (1 + l_t^2 k^2))
double density(int kind, double kT, double V, double Q2, const KernelTerms &K, double k2);
// Fhat(k^2) = sum_m A_m exp(-B_m k^2) in ascending m
double fhat(const rbsog_sog &s, double k2);
// vm[m] = k^2 G(k^2) / Fhat(k^2) at k^2 = (2 pi / L)^2 m, m = 0 .. mmax, with
// G = -dFhat/d(k^2): the factor a mode's term of the far-field virial carries
// beside 3/2 of its energy term
void virial_table(const rbsog_sog &s, double L, int mmax, double *vm);
// shell CDF, coefficients and shell ranges; the packed lattice too when asked
// (a cuboid box, see box_edges, gets one entry per lattice point and ignores mmax)
void build_tables(const rbsog_sog &s, const rbsog_params &p, double Q2, int mmax, Tables *t, bool with_lattice);
// k^2 of lattice point n in a box of edges Lb
double box_k2(const double Lb[3], int nx, int ny, int nz);
// points of a cuboid's lattice (every n != 0 with Fhat(k^2) >= 1e-16 Fhat(0)), or -1 beyond |n_d| = 511
int64_t box_lattice_points(const rbsog_sog &s, const double Lb[3]);
// the box edges of the parameters (Ly, Lz of 0 take L)
void box_edges(const rbsog_params *p, double Lb[3]);
// (sin, cos)(2 pi j / kPhaseTable), j = 0 .. kPhaseTable - 1, interleaved, from
// the host's libm: the rotation table of the FP64 phase kernels
constexpr int kPhaseTable = 128;
void phase_table(double out[2 * kPhaseTable]);
// the far field's finer table, (sin, cos)(2 pi j / 1024)
constexpr int kFarTable = 1024;
void far_table(double out[2 * kFarTable]);
// sum q and sum q^2 in particle order (plain FP64 additions, no contraction)
void charge_sums(const double *q, int64_t N, double *q1, double *q2);

}  // namespace rbsog

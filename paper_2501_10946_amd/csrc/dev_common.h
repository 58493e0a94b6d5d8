// Device helpers shared by the kernels of librbsog.
#pragma once

#include <hip/hip_runtime.h>

#include "dev_math.h"
#include "launch.h"

namespace rbsog {

// Cell coordinate of a position: clamp(floor(x nc / L), 0, nc - 1); a NaN maps to 0.
__device__ inline int cell_coord(double x, double inv_cell, int nc)
{
    double f = floor(x * inv_cell);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(nc - 1)) return nc - 1;
    return (int)f;
}

// Raises *flag when cond holds in any active lane of the wave: one atomic per
// wave (the lowest such lane), not one per lane.  Every lane of a step may
// raise the same rebuild gate (a hot system with no skin), and same-address
// atomics from every lane serialise in the L2.
__device__ inline void raise_any(int32_t *flag, bool cond)
{
    const uint64_t m = __ballot(cond);
    if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) atomicOr(flag, 1);
}

// Raises a rebuild gate when some particle of the wave has moved more than half
// the skin since the last build (d2: its squared displacement).  With no skin
// any motion leaves the lists stale, so the gate is raised by the system's
// first particle alone: one atomic per launch instead of one per wave (at 1e6
// particles the 15 625 same-address atomics of the waves serialise for
// ~0.15 ms).
__device__ inline void raise_gate(int32_t *gate, double d2, double half_skin2, int p)
{
    raise_any(gate, half_skin2 > 0.0 ? !(d2 <= half_skin2) : p == 0);
}

// Fixed-order sum over a 256-thread block; valid in thread 0.
__device__ inline double block_sum_256(double v, double *red)
{
    int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
#pragma unroll
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    return red[0];
}

// The thermostat's three normal deviates of particle i (caller index) for the
// drift into force index `step`: four uniforms ((w >> 11) + 1) 2^-53 in (0, 1]
// from Philox4x64-10(counter (i, step, 1, 0), key (seed, replica)) -- word 2 =
// 1 keeps them apart from the mode draws -- through the Box-Muller transform.
__device__ inline void langevin_normals(uint64_t i, const Thermo &th, double z[3])
{
    uint64_t w[4];
    philox4x64_10(i, th.step, 1, 0, th.seed, (uint64_t)th.replica, w);
    double u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = (double)((w[k] >> 11) + 1) * 0x1p-53;
    const double twopi = 6.283185307179586;
    const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(twopi * u[1]);
    z[1] = r0 * sin(twopi * u[1]);
    z[2] = r1 * cos(twopi * u[3]);
}

// First half-kick and drift of one particle (cell position p): v += hm f,
// x += dt v, wrapped into [0, L); returns the squared minimum-image distance
// from the build position xb and sets *bad on a step of a box length or more.
// The drift kernel and the far kernel's fused form both run this, so that
// their trajectories agree bit for bit.  hm = dt / (2 m); with a thermostat
// on, ci is the particle's caller index and m its mass.
__device__ inline double kick_drift_row(double x[3], double v[3], const double f[3], double hm, double dt,
                                        const double Lb[3], const double inv_Lb[3], const double *xb, int N, int p,
                                        bool *bad, const Thermo &th, uint64_t ci, double m)
{
    double d2 = 0.0;
    double z[3] = {0.0, 0.0, 0.0}, sig = 0.0;
    if (th.on) {
        langevin_normals(ci, th, z);
        sig = sqrt(th.c2kT / m);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double vv = v[d] + hm * f[d];
        double dx;
        if (th.on) {   // half drift, Ornstein-Uhlenbeck update, half drift
            const double v2 = th.c1 * vv + sig * z[d];
            dx = 0.5 * dt * vv + 0.5 * dt * v2;
            vv = v2;
        } else {
            dx = dt * vv;
        }
        const double L = Lb[d];
        *bad |= !(fabs(dx) < L);
        double xx = x[d] + dx;
        if (xx >= L) xx -= L;
        if (xx < 0.0) xx += L;
        if (xx >= L) xx = 0.0;
        v[d] = vv;
        x[d] = xx;
        double s = xx - xb[d * N + p];
        s = fma(-L, rint(s * inv_Lb[d]), s);
        d2 = fma(s, s, d2);
    }
    return d2;
}

// ---------------------------------------------------------------------------
// structure factors.  Particles are cut into groups of C (the "chunk") and the
// lanes of the grid are laid out flat over (group s, sample l), lane s P + l,
// so every lane of every wave has work whatever P is.  A workgroup stages the
// particles of the groups its lanes touch in LDS; each lane sums its group in
// two interleaved streams and writes one partial per (group, sample); a second
// kernel adds the partials of each sample in a fixed order.
// ---------------------------------------------------------------------------

// One particle's term q exp(i k.r) of a mode; p holds (r/L, q) (mixed) or
// (T r/L, q) (FP64, T the entries of the rotation table: kPhaseTab, or
// kFarTab with FINE), so that k.p is the phase in the unit that the
// precision's sine and cosine take.
template <bool CELL, bool MIXED, bool FINE = false>
__device__ inline void rho_term(const RhoArgs &a, const double2 *tab, const double4 &k, const double4 &p,
                                double &re, double &im)
{
    double u = k.x * p.x + k.y * p.y + k.z * p.z;
    if (MIXED) {
        float sn, cs;
        sincos_rev_f32(u, &sn, &cs);
        re = fma(p.w, (double)cs, re);
        im = fma(p.w, (double)sn, im);
    } else {
        double sn, cs;
        if (FINE) sincos_rev_far(u, tab, a.sf, &sn, &cs);
        else sincos_rev_tab(u, tab, a.ss, &sn, &cs);
        re = fma(p.w, cs, re);
        im = fma(p.w, sn, im);
    }
}

template <bool CELL, bool MIXED, bool FINE>
__device__ inline void rho_partial_body(const RhoArgs &a, int b)
{
    // dynamic LDS: the rotation table (FP64), then the staged particles
    constexpr int T = FINE ? kFarTab : kPhaseTab;
    extern __shared__ double4 lds[];
    double2 *tab = (double2 *)lds;
    double4 *sp = lds + (MIXED ? 0 : T / 2);
    const int t = threadIdx.x;
    const int64_t g0 = (int64_t)b * kBlock;
    const int s_lo = (int)(g0 / a.P);
    const int s_hi = (int)min((int64_t)a.nchunk - 1, (g0 + kBlock - 1) / a.P);
    const int j_lo = s_lo * a.chunk;
    const int j_hi = min(a.N, (s_hi + 1) * a.chunk);
    // phase units of the precision, per axis
    const double phx = MIXED ? a.inv_L[0] : a.inv_L[0] * T;
    const double phy = MIXED ? a.inv_L[1] : a.inv_L[1] * T;
    const double phz = MIXED ? a.inv_L[2] : a.inv_L[2] * T;
    for (int k = t; k < j_hi - j_lo; k += kBlock) {
        int j = j_lo + k;
        double4 v;
        if (CELL) v = a.xs[j];
        else v = make_double4(a.x[j], a.x[a.N + j], a.x[2 * a.N + j], a.q[j]);
        sp[k] = make_double4(v.x * phx, v.y * phy, v.z * phz, v.w);
    }
    if (!MIXED) {
        const double2 *src = FINE ? a.tab_fine : a.tab;
        for (int k = t; k < T; k += kBlock) tab[k] = src[k];
    }
    __syncthreads();
    const int64_t g = g0 + t;
    if (g >= (int64_t)a.nchunk * a.P) return;
    const int s = (int)(g / a.P), l = (int)(g - (int64_t)s * a.P);
    const double4 k = a.samp[l];
    const int ib = s * a.chunk - j_lo, e = min(a.N, (s + 1) * a.chunk) - j_lo;
    double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
    int i = ib;
    for (; i + 1 < e; i += 2) {
        rho_term<CELL, MIXED, FINE>(a, tab, k, sp[i], re0, im0);
        rho_term<CELL, MIXED, FINE>(a, tab, k, sp[i + 1], re1, im1);
    }
    if (i < e) rho_term<CELL, MIXED, FINE>(a, tab, k, sp[i], re0, im0);
    a.part[g] = make_double2(re0 + re1, im0 + im1);
}

// k^2 G / Fhat of a mode (G = -dFhat/d(k^2)): from the table by |n|^2 in a
// cube, from the Fourier coefficients in a cuboid.
__device__ inline double mode_vm(const RhoArgs &a, const double4 &sl)
{
    if (a.vm) {   // |n|^2 from the mode's integer components (exact in FP64)
        const int m = (int)(sl.x * sl.x + sl.y * sl.y + sl.z * sl.z);
        return a.vm[m];
    }
    const double tp = 6.283185307179586;
    const double kx = tp * sl.x * a.inv_L[0], ky = tp * sl.y * a.inv_L[1], kz = tp * sl.z * a.inv_L[2];
    const double k2 = kx * kx + ky * ky + kz * kz;
    double F = 0.0, G = 0.0;
    for (int g = 0; g < a.nG; ++g) {
        const double e = exp(-a.fb[g] * k2);
        F += a.fa[g] * e;
        G += a.fa[g] * a.fb[g] * e;
    }
    return F > 0.0 ? k2 * G / F : 0.0;
}

// Fixed-order sum of the chunk partials, one workgroup per kRedModes adjacent
// samples so that each partial row is read as one contiguous segment.  Thread
// t takes sample l = kRedModes b + (t mod kRedModes) and adds the partials of
// groups c, c + 64, c + 128, ... (c = t / kRedModes, four loads in flight); the
// 16 threads of a wave that share a sample are added by a fixed butterfly and
// the four waves in order.
__device__ inline void rho_reduce_body(const RhoArgs &a, int b)
{
    constexpr int kLanes = kBlock / kRedModes;   // group streams per sample
    __shared__ double2 red[kBlock / 64][kRedModes];
    const int t = threadIdx.x, m = t % kRedModes, c0 = t / kRedModes;
    const int l = b * kRedModes + m;
    const bool live = l < a.P;
    const double2 *col = a.part + (live ? l : 0);
    const size_t P = (size_t)a.P;
    const int nch = live ? a.nchunk : 0;
    double re = 0.0, im = 0.0;
    int c = c0;
    for (; c + 3 * kLanes < nch; c += 4 * kLanes) {
        double2 v0 = col[(size_t)c * P], v1 = col[(size_t)(c + kLanes) * P];
        double2 v2 = col[(size_t)(c + 2 * kLanes) * P], v3 = col[(size_t)(c + 3 * kLanes) * P];
        re += v0.x;
        im += v0.y;
        re += v1.x;
        im += v1.y;
        re += v2.x;
        im += v2.y;
        re += v3.x;
        im += v3.y;
    }
    for (; c < nch; c += kLanes) {
        double2 v = col[(size_t)c * P];
        re += v.x;
        im += v.y;
    }
#pragma unroll
    for (int off = 32; off >= kRedModes; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if ((t & 63) < kRedModes) red[t >> 6][m] = make_double2(re, im);
    __syncthreads();
    if (t < kRedModes && live) {
        re = 0.0;
        im = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            re += red[w][t].x;
            im += red[w][t].y;
        }
        double cf = a.samp[l].w;
        a.rho[l] = make_double2(re, im);
        a.gk[l] = make_double2(cf * re, cf * im);
        a.eF[l] = 0.5 * cf * (re * re + im * im);
        if (a.eW) a.eW[l] = cf * (re * re + im * im) * (1.5 - mode_vm(a, a.samp[l]));
        if (a.rho_out) {
            a.rho_out[2 * l] = re;
            a.rho_out[2 * l + 1] = im;
        }
    }
}

}  // namespace rbsog

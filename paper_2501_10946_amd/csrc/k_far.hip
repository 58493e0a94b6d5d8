// gfx950 kernels of librbsog: far field, force assembly, second half-kick, energies.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace rbsog {

// ---------------------------------------------------------------------------
// far field of the random batch (eq. UF):
//   f_i += -q_i (2 pi / L) sum_l coef_l n_l Im(exp(-i k_l . r_i) rho_l).
// A workgroup owns 64 consecutive particles (cell order) and has 4 waves; wave
// g takes the samples l = g mod 4 of each LDS tile of 256 samples, so every
// particle's sum is spread over 4 lanes (4x the waves of one lane per particle,
// which the latency of the dependent FP64 chains needs).  The 4 partial sums are
// added in a fixed order, then near + far is written (in cell order, and/or
// in the caller's order) and the second half-kick applied in cell order; in a
// run of steps the next step's first half-kick and drift follow at once.
// ---------------------------------------------------------------------------

constexpr int kFarGroups = 4;
constexpr int kFarThreads = 64 * kFarGroups;
constexpr int kFarTile = 256;

// Im(exp(-i k.r) coef rho) of one mode (kv: n, gv: coef rho); (sx, sy, sz) is
// r/L (mixed) or 1024 r/L (FP64), so that n.s is the phase in the unit that the
// precision's sine and cosine take.
template <bool MIXED>
__device__ inline double far_term(const FarArgs &a, const double2 *tab, const double4 &kv, const double2 &gv,
                                  double sx, double sy, double sz)
{
    double u = kv.x * sx + kv.y * sy + kv.z * sz;
    if (MIXED) {
        float sn, cs;
        sincos_rev_f32(u, &sn, &cs);
        return gv.y * (double)cs - gv.x * (double)sn;
    } else {
        double sn, cs;
        sincos_rev_far(u, tab, a.ss, &sn, &cs);
        return gv.y * cs - gv.x * sn;
    }
}

template <bool MIXED, bool DRIFT>
__device__ inline void far_body(const FarArgs &a, int b)
{
    __shared__ double4 sk[kFarTile];
    __shared__ double2 sg[kFarTile];
    __shared__ double2 tab[kFarTab];
    __shared__ double red[64];
    static_assert(sizeof(sk) >= 3 * kFarThreads * sizeof(double), "partials reuse the sample tile");
    double(*part)[kFarThreads] = (double(*)[kFarThreads])sk;
    const int t = threadIdx.x;
    const int g = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;   // g is uniform per wave
    const int p = b * 64 + lane;
    if (a.gate_clear && b == 0 && t == 0) {
        if (a.rebuilds && *a.gate_clear) *a.rebuilds += 1;
        *a.gate_clear = 0;
    }
    const bool live = p < a.N;
    double4 pi = live ? a.xs[p] : make_double4(0.0, 0.0, 0.0, 0.0);
    // phases in revolutions (mixed) or 1/1024 revolutions (FP64 table path)
    const double phx = MIXED ? a.inv_L[0] : a.inv_L[0] * kFarTab;
    const double phy = MIXED ? a.inv_L[1] : a.inv_L[1] * kFarTab;
    const double phz = MIXED ? a.inv_L[2] : a.inv_L[2] * kFarTab;
    double sx = pi.x * phx, sy = pi.y * phy, sz = pi.z * phz;
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (!MIXED)
        for (int k = t; k < kFarTab; k += kFarThreads) tab[k] = a.tab[k];
    for (int l0 = 0; l0 < a.P; l0 += kFarTile) {
        __syncthreads();
        if (l0 + t < a.P) {
            sk[t] = a.samp[l0 + t];
            sg[t] = a.gk[l0 + t];
        }
        __syncthreads();
        int nl = min(kFarTile, a.P - l0);
        // two modes per pass (independent chains), added in mode order
        int k = g;
        for (; k + kFarGroups < nl; k += 2 * kFarGroups) {
            const double4 k0 = sk[k], k1 = sk[k + kFarGroups];
            const double im0 = far_term<MIXED>(a, tab, k0, sg[k], sx, sy, sz);
            const double im1 = far_term<MIXED>(a, tab, k1, sg[k + kFarGroups], sx, sy, sz);
            ax += im0 * k0.x;
            ay += im0 * k0.y;
            az += im0 * k0.z;
            ax += im1 * k1.x;
            ay += im1 * k1.y;
            az += im1 * k1.z;
        }
        if (k < nl) {
            const double4 k0 = sk[k];
            const double im0 = far_term<MIXED>(a, tab, k0, sg[k], sx, sy, sz);
            ax += im0 * k0.x;
            ay += im0 * k0.y;
            az += im0 * k0.z;
        }
    }
    __syncthreads();   // the sample tile is done with: it holds the partials next
    part[0][t] = ax;
    part[1][t] = ay;
    part[2][t] = az;
    __syncthreads();
    double ke = 0.0;
    if (t < 64 && live) {
        double bx = 0.0, by = 0.0, bz = 0.0;
#pragma unroll
        for (int k = 0; k < kFarGroups; ++k) {
            bx += part[0][k * 64 + t];
            by += part[1][k * 64 + t];
            bz += part[2][k * 64 + t];
        }
        const double scx = -pi.w * a.two_pi_over_L[0], scy = -pi.w * a.two_pi_over_L[1];
        const double scz = -pi.w * a.two_pi_over_L[2];
        // near field: the lane partials, added in lane order
        double fnx = 0.0, fny = 0.0, fnz = 0.0;
#pragma unroll
        for (int k = 0; k < kNearLanes; ++k) {
            const double *pl = a.fnear + (size_t)k * 3 * a.N + p;
            fnx += pl[0];
            fny += pl[a.N];
            fnz += pl[2 * (size_t)a.N];
        }
        double fx = fnx + scx * bx, fy = fny + scy * by, fz = fnz + scz * bz;
        if (a.fs) {
            a.fs[p] = fx;
            a.fs[a.N + p] = fy;
            a.fs[2 * a.N + p] = fz;
        }
        if (a.f || a.f_near_out) {
            int i = a.order[p];
            if (a.f) {
                a.f[i] = fx;
                a.f[a.N + i] = fy;
                a.f[2 * a.N + i] = fz;
            }
            if (a.f_near_out) {
                a.f_near_out[i] = fnx;
                a.f_near_out[a.N + i] = fny;
                a.f_near_out[2 * a.N + i] = fnz;
            }
        }
        raise_any(a.flag, !isfinite(fx + fy + fz));
        if (a.vs) {
            double mi = a.ms[p];
            double hm = a.half_dt / mi;
            double vx = a.vs[p] + hm * fx, vy = a.vs[a.N + p] + hm * fy, vz = a.vs[2 * a.N + p] + hm * fz;
            ke = 0.5 * mi * (vx * vx + vy * vy + vz * vz);
            if (DRIFT) {   // the next step's first half-kick and drift
                double x[3] = {pi.x, pi.y, pi.z}, v[3] = {vx, vy, vz};
                const double f[3] = {fx, fy, fz};
                bool bad = false;
                double d2 = kick_drift_row(x, v, f, hm, a.dt, a.L, a.inv_L, a.xb, a.N, p, &bad, a.th,
                                           a.th.on ? (uint64_t)a.order[p] : 0, mi);
                vx = v[0];
                vy = v[1];
                vz = v[2];
                a.xs_next[p] = make_double4(x[0], x[1], x[2], pi.w);
                raise_any(a.flag, bad);
                raise_gate(a.gate_raise, d2, a.half_skin2, p);
            }
            a.vs[p] = vx;
            a.vs[a.N + p] = vy;
            a.vs[2 * a.N + p] = vz;
        }
    }
    if (a.kepart) {
        if (t < 64) red[t] = ke;
        __syncthreads();
        for (int off = 32; off > 0; off >>= 1) {
            if (t < off) red[t] += red[t + off];
            __syncthreads();
        }
        if (t == 0) a.kepart[b] = red[0];
    }
}

template <bool MIXED, bool DRIFT>
__global__ __launch_bounds__(kFarThreads) void k_far(FarArgs a)
{
    far_body<MIXED, DRIFT>(a, (int)blockIdx.x);
}

template <bool MIXED>
__global__ __launch_bounds__(kFarThreads) void k_far_batch(const FarArgs *__restrict__ tab,
                                                           const EnsItem *__restrict__ items)
{
    const EnsItem e = items[blockIdx.x];
    far_body<MIXED, false>(tab[e.r], e.b);
}

hipError_t launch_far_batch(const FarArgs *tab, const EnsItem *items, int n, bool mixed, hipStream_t st)
{
    if (!tab || !items || n < 1) return hipErrorInvalidValue;
    if (mixed) hipLaunchKernelGGL(k_far_batch<true>, dim3(n), dim3(kFarThreads), 0, st, tab, items);
    else hipLaunchKernelGGL(k_far_batch<false>, dim3(n), dim3(kFarThreads), 0, st, tab, items);
    return hipGetLastError();
}

hipError_t launch_far(const FarArgs &a, hipStream_t st)
{
    if (a.N < 1 || a.P < 1 || !a.xs || !a.order || !a.samp || !a.gk || !a.fnear || (!a.f && !a.fs) || !a.flag ||
        (a.vs && (!a.ms || !a.kepart)) || (!a.mixed && !a.tab) ||
        (a.drift && (!a.vs || !a.xb || !a.xs_next || !a.gate_raise)))
        return hipErrorInvalidValue;
    dim3 grid(far_blocks(a.N));
    if (a.drift) {
        if (a.mixed) hipLaunchKernelGGL((k_far<true, true>), grid, dim3(kFarThreads), 0, st, a);
        else hipLaunchKernelGGL((k_far<false, true>), grid, dim3(kFarThreads), 0, st, a);
    } else {
        if (a.mixed) hipLaunchKernelGGL((k_far<true, false>), grid, dim3(kFarThreads), 0, st, a);
        else hipLaunchKernelGGL((k_far<false, false>), grid, dim3(kFarThreads), 0, st, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// energies: fixed-order sums of the block partials
// ---------------------------------------------------------------------------

// shift: rows of `out` to skip (the ensemble writes row shift + row0)
__device__ inline void energy_body(const EnergyArgs &a, uint64_t shift)
{
    __shared__ double red[kBlock];
    double un = 0.0, ke = 0.0, uf = 0.0, wn = 0.0, wf = 0.0;
    for (int b = threadIdx.x; b < a.nnear; b += kBlock) {
        un += a.epart[b];
        wn += a.epart[a.nnear + b];
    }
    for (int l = threadIdx.x; l < a.P; l += kBlock) {
        uf += a.eF[l];
        wf += a.eW[l];
    }
    if (a.kepart)
        for (int b = threadIdx.x; b < a.nfar; b += kBlock) ke += a.kepart[b];
    un = block_sum_256(un, red);
    __syncthreads();
    uf = block_sum_256(uf, red);
    __syncthreads();
    ke = block_sum_256(ke, red);
    __syncthreads();
    wn = block_sum_256(wn, red);
    __syncthreads();
    wf = block_sum_256(wf, red);
    if (threadIdx.x == 0) {
        double *o = a.out + kEnergyCols * (shift + a.row0);
        o[0] = un;
        o[1] = uf;
        o[2] = a.Uk0;
        o[3] = a.Uself;
        o[4] = a.Ubg;
        o[5] = a.ke_set ? *a.ke_set : ke;
        o[6] = wn;
        o[7] = wf;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a) { energy_body(a, 0); }

__global__ __launch_bounds__(kBlock) void k_energy_batch(const EnergyArgs *__restrict__ tab,
                                                         const EnsItem *__restrict__ items, const uint64_t *shift)
{
    energy_body(tab[items[blockIdx.x].r], *shift);
}

hipError_t launch_energy_batch(const EnergyArgs *tab, const EnsItem *items, int n, const uint64_t *shift,
                               hipStream_t st)
{
    if (!tab || !items || n < 1 || !shift) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_batch, dim3(n), dim3(kBlock), 0, st, tab, items, shift);
    return hipGetLastError();
}

hipError_t launch_energy(const EnergyArgs &a, hipStream_t st)
{
    if (!a.epart || !a.eF || !a.eW || !a.out) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}


}  // namespace rbsog

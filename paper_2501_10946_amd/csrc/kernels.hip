// gfx950 kernels of librbsog: cell list, sampling, structure factors, near
// field, far field with force assembly and the velocity-Verlet half steps.
//
// Data layout in HBM: the caller's particle arrays stay FP64 SoA in the
// caller's order; each evaluation builds a cell-ordered copy xs[N] of
// (x, y, z, q) as double4 (32-byte rows, one 128-bit-pair load per particle)
// that the pair and far-field kernels stream.
#include <hip/hip_runtime.h>

#include "dev_math.h"
#include "launch.h"

namespace rbsog {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Cell coordinate of a position: clamp(floor(x nc / L), 0, nc - 1); a NaN maps to 0.
__device__ inline int cell_coord(double x, double inv_cell, int nc)
{
    double f = floor(x * inv_cell);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(nc - 1)) return nc - 1;
    return (int)f;
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

__global__ void k_zero_int(int32_t *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_int(int32_t *p, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_int, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cell list: ids + counts, scan, scatter, stable rank + gather
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_cell_ids(CellArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    int nc = a.g.nc;
    int cx = cell_coord(a.x[i], a.g.inv_cell, nc);
    int cy = cell_coord(a.x[a.N + i], a.g.inv_cell, nc);
    int cz = cell_coord(a.x[2 * a.N + i], a.g.inv_cell, nc);
    int id = (cz * nc + cy) * nc + cx;
    a.cell_id[i] = id;
    atomicAdd(&a.count[id], 1);
}

// Exclusive scan of the cell counts by one workgroup; also clears the fill counters.
__global__ __launch_bounds__(1024) void k_scan(CellArgs a)
{
    __shared__ int32_t sums[1024];
    int t = threadIdx.x;
    int n = a.g.ncell;
    int per = (n + 1023) / 1024;
    int b = t * per, e = min(n, b + per);
    int32_t s = 0;
    for (int k = b; k < e; ++k) s += a.count[k];
    sums[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = (t >= off) ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int32_t run = (t == 0) ? 0 : sums[t - 1];
    for (int k = b; k < e; ++k) {
        a.cell_start[k] = run;
        run += a.count[k];
        a.fill[k] = 0;
    }
    if (t == 1023) a.cell_start[n] = sums[1023];
}

// Unordered placement into each cell's segment.
__global__ __launch_bounds__(kBlock) void k_scatter(CellArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    int c = a.cell_id[i];
    int slot = atomicAdd(&a.fill[c], 1);
    a.tmp[a.cell_start[c] + slot] = i;
}

// Stable position: a particle's rank within its cell is the number of cell
// members with a smaller index, so ties keep ascending particle index whatever
// order the scatter produced.  Gathers (x, y, z, q) into cell order.
__global__ __launch_bounds__(kBlock) void k_rank(CellArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    int c = a.cell_id[i];
    int b = a.cell_start[c], e = a.cell_start[c + 1];
    int r = 0;
    for (int k = b; k < e; ++k) r += (a.tmp[k] < i);
    int p = b + r;
    a.order[p] = i;
    a.xs[p] = make_double4(a.x[i], a.x[a.N + i], a.x[2 * a.N + i], a.q[i]);
}

hipError_t launch_cell_ids(const CellArgs &a, hipStream_t st)
{
    hipError_t e = launch_zero_int(a.count, a.g.ncell, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_ids, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_cells_finish(const CellArgs &a, hipStream_t st)
{
    int grid = (a.N + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_rank, dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// first half-kick + drift + wrap, fused with the cell ids of the new positions
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_kick_drift(KickDriftArgs a)
{
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    double L = a.g.L;
    double hm = (0.5 * a.dt) / a.m[i];
    int cc[3];
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double vv = a.v[d * a.N + i] + hm * a.f[d * a.N + i];
        double dx = a.dt * vv;
        bad |= !(fabs(dx) < L);
        double xx = a.x[d * a.N + i] + dx;
        if (xx >= L) xx -= L;
        if (xx < 0.0) xx += L;
        if (xx >= L) xx = 0.0;
        a.v[d * a.N + i] = vv;
        a.x[d * a.N + i] = xx;
        cc[d] = cell_coord(xx, a.g.inv_cell, a.g.nc);
    }
    if (bad) atomicOr(a.flag, 1);
    int id = (cc[2] * a.g.nc + cc[1]) * a.g.nc + cc[0];
    a.cell_id[i] = id;
    atomicAdd(&a.count[id], 1);
}

hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t st)
{
    hipError_t e = launch_zero_int(a.count, a.g.ncell, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sampling: P i.i.d. modes from the shell CDF (bit-exact integer/IEEE steps)
// ---------------------------------------------------------------------------

__global__ void k_sample(SampleArgs a)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.P) return;
    uint64_t w[4];
    philox4x64_10((uint64_t)l, a.step, 0, 0, a.seed, (uint64_t)a.replica, w);
    double u = (double)(w[0] >> 11) * 0x1p-53;
    double target = u * a.S;
    int lo = 0, hi = a.nshell;
    while (lo < hi) {
        int mid = lo + ((hi - lo) >> 1);
        if (a.cdf[mid] > target) hi = mid; else lo = mid + 1;
    }
    int i = lo < a.nshell ? lo : a.nshell - 1;
    uint64_t j = __umul64hi(w[1], (uint64_t)a.size[i]);
    uint32_t pk = (uint32_t)a.lattice[a.first[i] + (int64_t)j];
    int nx = (int)(pk & 1023u) - 512, ny = (int)((pk >> 10) & 1023u) - 512, nz = (int)((pk >> 20) & 1023u) - 512;
    double cf = a.coef[i];
    a.samp[l] = make_double4((double)nx, (double)ny, (double)nz, cf);
    if (a.n_out) {
        a.n_out[3 * l + 0] = nx;
        a.n_out[3 * l + 1] = ny;
        a.n_out[3 * l + 2] = nz;
    }
    if (a.coef_out) a.coef_out[l] = cf;
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_sample, dim3((a.P + 63) / 64), dim3(64), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// structure factors: lanes own samples, particles stream through LDS
// ---------------------------------------------------------------------------

template <bool CELL, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_rho_partial(RhoArgs a)
{
    __shared__ double4 sp[kRhoChunk];
    int chunk = blockIdx.x;
    int j0 = chunk * kRhoChunk;
    int nj = min(kRhoChunk, a.N - j0);
    for (int t = threadIdx.x; t < nj; t += kBlock) {
        int j = j0 + t;
        double4 v;
        if (CELL) v = a.xs[j];
        else v = make_double4(a.x[j], a.x[a.N + j], a.x[2 * a.N + j], a.q[j]);
        sp[t] = make_double4(v.x * a.inv_L, v.y * a.inv_L, v.z * a.inv_L, v.w);
    }
    __syncthreads();
    int l = blockIdx.y * kBlock + threadIdx.x;
    if (l >= a.P) return;
    double4 k = a.samp[l];
    double re = 0.0, im = 0.0;
    for (int t = 0; t < nj; ++t) {
        double4 s = sp[t];
        double u = k.x * s.x + k.y * s.y + k.z * s.z;
        if (MIXED) {
            float sn, cs;
            sincos_rev_f32(u, &sn, &cs);
            re += s.w * (double)cs;
            im += s.w * (double)sn;
        } else {
            double sn, cs;
            sincos_rev(u, &sn, &cs);
            re += s.w * cs;
            im += s.w * sn;
        }
    }
    a.part[(size_t)chunk * a.P + l] = make_double2(re, im);
}

// One workgroup per sample: fixed-order sum of the chunk partials.
__global__ __launch_bounds__(kBlock) void k_rho_reduce(RhoArgs a)
{
    __shared__ double red[kBlock];
    int l = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int c = threadIdx.x; c < a.nchunk; c += kBlock) {
        double2 v = a.part[(size_t)c * a.P + l];
        re += v.x;
        im += v.y;
    }
    re = block_sum_256(re, red);
    __syncthreads();
    im = block_sum_256(im, red);
    if (threadIdx.x == 0) {
        double cf = a.samp[l].w;
        a.rho[l] = make_double2(re, im);
        a.gk[l] = make_double2(cf * re, cf * im);
        a.eF[l] = 0.5 * cf * (re * re + im * im);
        if (a.rho_out) {
            a.rho_out[2 * l] = re;
            a.rho_out[2 * l + 1] = im;
        }
    }
}

hipError_t launch_rho_partial(const RhoArgs &a, hipStream_t st)
{
    dim3 grid(a.nchunk, (a.P + kBlock - 1) / kBlock);
    if (a.xs) {
        if (a.mixed) hipLaunchKernelGGL((k_rho_partial<true, true>), grid, dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_rho_partial<true, false>), grid, dim3(kBlock), 0, st, a);
    } else {
        if (a.mixed) hipLaunchKernelGGL((k_rho_partial<false, true>), grid, dim3(kBlock), 0, st, a);
        else hipLaunchKernelGGL((k_rho_partial<false, false>), grid, dim3(kBlock), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_rho_reduce(const RhoArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_rho_reduce, dim3(a.P), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// near field: one thread per particle (cell order), 27-cell stencil with a
// per-cell image shift (valid because nc >= 3)
// ---------------------------------------------------------------------------

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_near(NearArgs a)
{
    __shared__ double red[kBlock];
    int p = blockIdx.x * kBlock + threadIdx.x;
    double en = 0.0;
    if (p < a.N) {
        const int nc = a.g.nc;
        const double L = a.g.L;
        double4 pi = a.xs[p];
        int c0x = cell_coord(pi.x, a.g.inv_cell, nc);
        int c0y = cell_coord(pi.y, a.g.inv_cell, nc);
        int c0z = cell_coord(pi.z, a.g.inv_cell, nc);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int oz = -1; oz <= 1; ++oz) {
            int cz = c0z + oz;
            double sz = 0.0;
            if (cz < 0) { cz += nc; sz = -L; } else if (cz >= nc) { cz -= nc; sz = L; }
            for (int oy = -1; oy <= 1; ++oy) {
                int cy = c0y + oy;
                double sy = 0.0;
                if (cy < 0) { cy += nc; sy = -L; } else if (cy >= nc) { cy -= nc; sy = L; }
                for (int ox = -1; ox <= 1; ++ox) {
                    int cx = c0x + ox;
                    double sx = 0.0;
                    if (cx < 0) { cx += nc; sx = -L; } else if (cx >= nc) { cx -= nc; sx = L; }
                    int cell = (cz * nc + cy) * nc + cx;
                    int jb = a.cell_start[cell], je = a.cell_start[cell + 1];
                    double bx = pi.x - sx, by = pi.y - sy, bz = pi.z - sz;
                    for (int j = jb; j < je; ++j) {
                        if (j == p) continue;
                        double4 pj = a.xs[j];
                        double dx = bx - pj.x, dy = by - pj.y, dz = bz - pj.z;
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (!(r2 < a.rc2)) continue;
                        double qq = pi.w * pj.w;
                        if (MIXED) {
                            float r2f = (float)r2;
                            float irf = rsqrtf(r2f);
                            float rf = r2f * irf;
                            float ey = __expf(-rf * (float)a.sog.inv_lambda);
                            float f1 = ey * (1.0f + rf * (float)a.sog.inv_lambda) * irf * irf * irf;
                            float gs = 0.0f, fs = 0.0f;
                            for (int g = 0; g < a.sog.n; ++g) {
                                float eg = __expf(-(float)a.sog.s[g] * r2f);
                                gs += (float)a.sog.cs2[g] * eg;
                                fs += (float)a.sog.c[g] * eg;
                            }
                            double fac = qq * (double)(f1 - gs);
                            fx += fac * dx;
                            fy += fac * dy;
                            fz += fac * dz;
                            en += qq * (double)(ey * irf - fs);
                        } else {
                            double r = sqrt(r2);
                            double ir = 1.0 / r;
                            double ey = exp(-r * a.sog.inv_lambda);
                            double f1 = ey * (1.0 + r * a.sog.inv_lambda) * (ir * ir * ir);
                            double gs = 0.0, fs = 0.0;
                            for (int g = 0; g < a.sog.n; ++g) {
                                double eg = exp(-a.sog.s[g] * r2);
                                gs += a.sog.cs2[g] * eg;
                                fs += a.sog.c[g] * eg;
                            }
                            double fac = qq * (f1 - gs);
                            fx += fac * dx;
                            fy += fac * dy;
                            fz += fac * dz;
                            en += qq * (ey * ir - fs);
                        }
                    }
                }
            }
        }
        a.fnear[p] = fx;
        a.fnear[a.N + p] = fy;
        a.fnear[2 * a.N + p] = fz;
    }
    double tot = block_sum_256(0.5 * en, red);
    if (threadIdx.x == 0) a.epart[blockIdx.x] = tot;
}

hipError_t launch_near(const NearArgs &a, hipStream_t st)
{
    dim3 grid((a.N + kBlock - 1) / kBlock);
    if (a.mixed) hipLaunchKernelGGL(k_near<true>, grid, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_near<false>, grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// far field: one thread per particle (cell order), samples broadcast from LDS;
// assembles near + far into the caller's order and applies the second half-kick
// ---------------------------------------------------------------------------

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_far(FarArgs a)
{
    __shared__ double4 sk[kBlock];
    __shared__ double2 sg[kBlock];
    __shared__ double red[kBlock];
    int p = blockIdx.x * kBlock + threadIdx.x;
    bool live = p < a.N;
    double4 pi = live ? a.xs[p] : make_double4(0.0, 0.0, 0.0, 0.0);
    double sx = pi.x * a.inv_L, sy = pi.y * a.inv_L, sz = pi.z * a.inv_L;
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int l0 = 0; l0 < a.P; l0 += kBlock) {
        __syncthreads();
        if (l0 + (int)threadIdx.x < a.P) {
            sk[threadIdx.x] = a.samp[l0 + threadIdx.x];
            sg[threadIdx.x] = a.gk[l0 + threadIdx.x];
        }
        __syncthreads();
        int nl = min(kBlock, a.P - l0);
        for (int t = 0; t < nl; ++t) {
            double4 k = sk[t];
            double2 g = sg[t];
            double u = k.x * sx + k.y * sy + k.z * sz;
            double im;
            if (MIXED) {
                float sn, cs;
                sincos_rev_f32(u, &sn, &cs);
                im = g.y * (double)cs - g.x * (double)sn;
            } else {
                double sn, cs;
                sincos_rev(u, &sn, &cs);
                im = g.y * cs - g.x * sn;
            }
            ax += im * k.x;
            ay += im * k.y;
            az += im * k.z;
        }
    }
    double ke = 0.0;
    if (live) {
        double sc = -pi.w * a.two_pi_over_L;
        double fnx = a.fnear[p], fny = a.fnear[a.N + p], fnz = a.fnear[2 * a.N + p];
        double fx = fnx + sc * ax, fy = fny + sc * ay, fz = fnz + sc * az;
        int i = a.order[p];
        a.f[i] = fx;
        a.f[a.N + i] = fy;
        a.f[2 * a.N + i] = fz;
        if (a.f_near_out) {
            a.f_near_out[i] = fnx;
            a.f_near_out[a.N + i] = fny;
            a.f_near_out[2 * a.N + i] = fnz;
        }
        if (!isfinite(fx + fy + fz)) atomicOr(a.flag, 1);
        if (a.v) {
            double mi = a.m[i];
            double hm = a.half_dt / mi;
            double vx = a.v[i] + hm * fx, vy = a.v[a.N + i] + hm * fy, vz = a.v[2 * a.N + i] + hm * fz;
            a.v[i] = vx;
            a.v[a.N + i] = vy;
            a.v[2 * a.N + i] = vz;
            ke = 0.5 * mi * (vx * vx + vy * vy + vz * vz);
        }
    }
    if (a.kepart) {
        double tot = block_sum_256(ke, red);
        if (threadIdx.x == 0) a.kepart[blockIdx.x] = tot;
    }
}

hipError_t launch_far(const FarArgs &a, hipStream_t st)
{
    dim3 grid((a.N + kBlock - 1) / kBlock);
    if (a.mixed) hipLaunchKernelGGL(k_far<true>, grid, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_far<false>, grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// energies: fixed-order sums of the block partials
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_energy(EnergyArgs a)
{
    __shared__ double red[kBlock];
    double un = 0.0, ke = 0.0, uf = 0.0;
    for (int b = threadIdx.x; b < a.nnear; b += kBlock) un += a.epart[b];
    for (int l = threadIdx.x; l < a.P; l += kBlock) uf += a.eF[l];
    if (a.kepart)
        for (int b = threadIdx.x; b < a.nfar; b += kBlock) ke += a.kepart[b];
    un = block_sum_256(un, red);
    __syncthreads();
    uf = block_sum_256(uf, red);
    __syncthreads();
    ke = block_sum_256(ke, red);
    if (threadIdx.x == 0) {
        a.out[0] = un;
        a.out[1] = uf;
        a.out[2] = a.Uk0;
        a.out[3] = a.Uself;
        a.out[4] = a.Ubg;
        a.out[5] = ke;
    }
}

hipError_t launch_energy(const EnergyArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace rbsog

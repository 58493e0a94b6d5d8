// gfx950 kernels of librbsog: structure factors rho(k).
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace rbsog {

// ---------------------------------------------------------------------------
// structure factors: lanes own samples, particles stream through LDS.
// A workgroup takes a chunk of particles (64..256, chosen so that the grid has
// enough waves to cover the chip) and up to 256 samples, and writes one
// partial sum per (chunk, sample); a second kernel adds the partials of each
// sample in a fixed order.
// ---------------------------------------------------------------------------

template <bool CELL, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_rho_partial(RhoArgs a)
{
    __shared__ double4 sp[kRhoChunkMax];
    int chunk = blockIdx.x;
    int j0 = chunk * a.chunk;
    int nj = min(a.chunk, a.N - j0);
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
            sincos_rev(u, a.sc, &sn, &cs);
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

int rho_chunk(int N, int P)
{
    // enough workgroups for ~8 waves per SIMD (4 waves per workgroup, 1024 SIMDs)
    int groups = (P + kBlock - 1) / kBlock;
    for (int c = kRhoChunkMax; c > 64; c >>= 1)
        if ((int64_t)((N + c - 1) / c) * groups >= 2048) return c;
    return 64;
}

hipError_t launch_rho_partial(const RhoArgs &a, hipStream_t st)
{
    if (a.N < 1 || a.P < 1 || a.chunk < 1 || a.chunk > kRhoChunkMax || !a.samp || !a.part ||
        (!a.xs && (!a.x || !a.q)))
        return hipErrorInvalidValue;
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
    if (!a.part || !a.rho || !a.gk || !a.eF || !a.samp) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rho_reduce, dim3(a.P), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}


}  // namespace rbsog

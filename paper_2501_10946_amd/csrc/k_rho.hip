// gfx950 kernels of librbsog: structure factors rho(k).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "dev_common.h"

namespace rbsog {

// the virial factors of eW: by |n|^2 from vm (a cube), or mode by mode from
// the Fourier coefficients (a cuboid)
static bool vm_ok(const RhoArgs &a) { return a.vm || (a.nG >= 1 && a.nG <= kMaxGauss && a.fa && a.fb); }

// Partial sums per (group, sample): rho_partial_body (shared with the near
// kernel, which can run it in its first workgroups) is in dev_common.h.

template <bool CELL, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_rho_partial(RhoArgs a)
{
    rho_partial_body<CELL, MIXED, false>(a, (int)blockIdx.x);
}

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_rho_partial_batch(const RhoArgs *__restrict__ tab,
                                                              const EnsItem *__restrict__ items)
{
    const EnsItem e = items[blockIdx.x];
    rho_partial_body<true, MIXED, true>(tab[e.r], e.b);   // the finer table, as the single system's step
}

// rho_reduce_body is in dev_common.h.
RBSOG_KERNELS(rho_reduce, RhoArgs, kBlock)

int rho_chunk(int N, int P)
{
    // the staged groups of a workgroup fit in LDS: a workgroup's lanes touch at
    // most 255 / P + 2 groups
    int cap = kRhoStage / (255 / P + 2);
    int c = 1;
    while (2 * c <= cap && 2 * c <= kRhoChunkMax) c *= 2;
    // RBSOG_RHO_CHUNK (a power of two within the cap) overrides the choice: a tuning knob
    if (const char *e = std::getenv("RBSOG_RHO_CHUNK")) {
        int v = std::atoi(e);
        if (v >= 1 && v <= c && (v & (v - 1)) == 0) return v;
    }
    // at least ~4 waves per SIMD (4096 waves of 64 lanes) where N and P allow
    while (c > 8 && (int64_t)((N + c - 1) / c) * P < 4096 * 64) c /= 2;
    return c;
}

bool rho_partial_ok(const RhoArgs &a)
{
    const int64_t lanes = (int64_t)a.nchunk * a.P;
    return !(a.N < 1 || a.P < 1 || a.chunk < 1 || a.chunk > kRhoChunkMax || !a.samp || !a.part ||
             (!a.xs && (!a.x || !a.q)) || (!a.mixed && !a.tab) ||
             (int64_t)(255 / a.P + 2) * a.chunk > kRhoStage || (int64_t)a.nchunk * a.chunk < a.N ||
             (lanes + kBlock - 1) / kBlock > 0x7fffffff);
}

int rho_chunk_shared(int N, int P, bool mixed)
{
    // the near workgroups supply the occupancy: groups as large as a staging
    // area of at most 16 KB allows (every workgroup of the shared launch
    // carries it), never smaller than the group of the launch of their own, so
    // that the partials fit the same buffer
    int c = 1;
    while (2 * c <= kRhoChunkMax && rho_lds_bytes(P, 2 * c, mixed, false) <= 16384 && (255 / P + 2) * 2 * c <= kRhoStage)
        c *= 2;
    return std::max(c, rho_chunk(N, P));
}

hipError_t launch_rho_partial(const RhoArgs &a, hipStream_t st)
{
    if (!rho_partial_ok(a)) return hipErrorInvalidValue;
    const int64_t lanes = (int64_t)a.nchunk * a.P;
    dim3 grid((unsigned)((lanes + kBlock - 1) / kBlock));
    size_t lds = rho_lds_bytes(a.P, a.chunk, a.mixed, false);
    if (a.xs) {
        if (a.mixed) hipLaunchKernelGGL((k_rho_partial<true, true>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_rho_partial<true, false>), grid, dim3(kBlock), lds, st, a);
    } else {
        if (a.mixed) hipLaunchKernelGGL((k_rho_partial<false, true>), grid, dim3(kBlock), lds, st, a);
        else hipLaunchKernelGGL((k_rho_partial<false, false>), grid, dim3(kBlock), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_rho_reduce(const RhoArgs &a, hipStream_t st)
{
    if (!a.part || !a.rho || !a.gk || !a.eF || !a.samp || (a.eW && !vm_ok(a))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rho_reduce, dim3(rho_reduce_blocks(a.P)), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// structure factors over the whole lattice (the deterministic reference):
// one lane per mode, the particles streamed through LDS in tiles of 256, each
// lane summing them in two interleaved chains; writes rho, coef rho and the
// energy term of every mode directly
// ---------------------------------------------------------------------------

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_rho_full(RhoArgs a)
{
    __shared__ double4 sp[kBlock];
    __shared__ double2 tab[kPhaseTab];
    const int t = threadIdx.x;
    if (!MIXED)
        for (int k = t; k < kPhaseTab; k += kBlock) tab[k] = a.tab[k];
    const int l = blockIdx.x * kBlock + t;
    const bool live = l < a.P;
    // phase units of the precision, per axis
    const double phx = MIXED ? a.inv_L[0] : a.inv_L[0] * kPhaseTab;
    const double phy = MIXED ? a.inv_L[1] : a.inv_L[1] * kPhaseTab;
    const double phz = MIXED ? a.inv_L[2] : a.inv_L[2] * kPhaseTab;
    const double4 k = live ? a.samp[l] : make_double4(0.0, 0.0, 0.0, 0.0);
    double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
    for (int j0 = 0; j0 < a.N; j0 += kBlock) {
        __syncthreads();
        if (j0 + t < a.N) {
            double4 v = a.xs[j0 + t];
            sp[t] = make_double4(v.x * phx, v.y * phy, v.z * phz, v.w);
        }
        __syncthreads();
        const int nj = min(kBlock, a.N - j0);
        int i = 0;
        for (; i + 1 < nj; i += 2) {
            rho_term<true, MIXED>(a, tab, k, sp[i], re0, im0);
            rho_term<true, MIXED>(a, tab, k, sp[i + 1], re1, im1);
        }
        if (i < nj) rho_term<true, MIXED>(a, tab, k, sp[i], re0, im0);
    }
    if (live) {
        const double re = re0 + re1, im = im0 + im1, cf = k.w;
        a.rho[l] = make_double2(re, im);
        a.gk[l] = make_double2(cf * re, cf * im);
        a.eF[l] = 0.5 * cf * (re * re + im * im);
        if (a.eW) a.eW[l] = cf * (re * re + im * im) * (1.5 - mode_vm(a, k));
        if (a.rho_out) {
            a.rho_out[2 * l] = re;
            a.rho_out[2 * l + 1] = im;
        }
    }
}

hipError_t launch_rho_full(const RhoArgs &a, hipStream_t st)
{
    if (a.N < 1 || a.P < 1 || !a.xs || !a.samp || !a.rho || !a.gk || !a.eF || (!a.mixed && !a.tab) ||
        (a.eW && !vm_ok(a)))
        return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.P + kBlock - 1) / kBlock));
    if (a.mixed) hipLaunchKernelGGL(k_rho_full<true>, grid, dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_rho_full<false>, grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// Ensemble: one launch over every replica's groups (items: rho_blocks per
// replica) with the largest staging any of them needs, then the reduction
// (items: P per replica).
size_t rho_lds_bytes(int P, int chunk, bool mixed, bool fine)
{
    return sizeof(double4) * ((mixed ? 0 : (fine ? kFarTab : kPhaseTab) / 2) + (size_t)(255 / P + 2) * chunk);
}

hipError_t launch_rho_batch(const RhoArgs *tab, const EnsItem *part_items, int npart, size_t lds, bool mixed,
                            const EnsItem *red_items, int nred, hipStream_t st)
{
    if (!tab || !part_items || !red_items || npart < 1 || nred < 1 || lds > 65536) return hipErrorInvalidValue;
    if (mixed) hipLaunchKernelGGL((k_rho_partial_batch<true>), dim3(npart), dim3(kBlock), lds, st, tab, part_items);
    else hipLaunchKernelGGL((k_rho_partial_batch<false>), dim3(npart), dim3(kBlock), lds, st, tab, part_items);
    hipLaunchKernelGGL(k_rho_reduce_batch, dim3(nred), dim3(kBlock), 0, st, tab, red_items);
    return hipGetLastError();
}

}  // namespace rbsog

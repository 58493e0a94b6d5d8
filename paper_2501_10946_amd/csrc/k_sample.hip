// gfx950 kernel of librbsog: i.i.d. draws of the Fourier modes.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace rbsog {

// ---------------------------------------------------------------------------
// sampling: P i.i.d. modes per step from the shell CDF (bit-exact integer/IEEE
// steps), for a batch of consecutive steps in one launch
// ---------------------------------------------------------------------------

constexpr int kSampleThreads = 64;

// Draw idx of the launch: mode l of step a.step + shift + s, idx = s P + l.
__device__ inline void sample_body(const SampleArgs &a, int b, uint64_t shift)
{
    int64_t idx = (int64_t)b * kSampleThreads + threadIdx.x;
    if (idx >= (int64_t)a.P * a.nstep) return;
    int s = (int)(idx / a.P), l = (int)(idx - (int64_t)s * a.P);
    uint64_t w[4];
    philox4x64_10((uint64_t)l, a.step + shift + (uint64_t)s, 0, 0, a.seed, (uint64_t)a.replica, w);
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
    a.samp[idx] = make_double4((double)nx, (double)ny, (double)nz, cf);
    if (a.n_out) {
        a.n_out[3 * l + 0] = nx;
        a.n_out[3 * l + 1] = ny;
        a.n_out[3 * l + 2] = nz;
    }
    if (a.coef_out) a.coef_out[l] = cf;
}

__global__ __launch_bounds__(kSampleThreads) void k_sample(SampleArgs a) { sample_body(a, (int)blockIdx.x, 0); }

// Ensemble: one step per replica, the replica's step being its table entry's
// step plus the ensemble step counter (read from device memory, so that a
// captured launch sequence can be replayed step after step).
__global__ __launch_bounds__(kSampleThreads) void k_sample_batch(const SampleArgs *__restrict__ tab,
                                                                 const EnsItem *__restrict__ items,
                                                                 const uint64_t *shift)
{
    const EnsItem e = items[blockIdx.x];
    sample_body(tab[e.r], e.b, *shift);
}

hipError_t launch_sample_batch(const SampleArgs *tab, const EnsItem *items, int n, const uint64_t *shift,
                               hipStream_t st)
{
    if (!tab || !items || n < 1 || !shift) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sample_batch, dim3(n), dim3(kSampleThreads), 0, st, tab, items, shift);
    return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t st)
{
    if (a.P < 1 || a.nstep < 1 || a.nshell < 1 || !a.cdf || !a.coef || !a.first || !a.size || !a.lattice ||
        !a.samp || (a.nstep > 1 && (a.n_out || a.coef_out)))
        return hipErrorInvalidValue;
    int64_t n = (int64_t)a.P * a.nstep;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + kSampleThreads - 1) / kSampleThreads)), dim3(kSampleThreads),
                       0, st, a);
    return hipGetLastError();
}


}  // namespace rbsog

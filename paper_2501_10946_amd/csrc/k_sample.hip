// gfx950 kernels of librbsog: the draws of the Fourier modes, i.i.d. or by the
// Metropolis-Hastings chain.
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

// ---------------------------------------------------------------------------
// Metropolis-Hastings draws: one wave walks the chain over the P * nstep draws
// of the launch in order (step-major).  Each lane prepares one proposal of a
// chunk of 64 -- Philox words (l, step, 2, 0), the shell and point from the
// proposal CDF, the acceptance product a coef(i') -- and the chain then
// visits the chunk's lanes in order with the state in scalar registers: move
// to proposal j iff the chain is empty or a_j coef(i'_j) < coef(i_cur).
// ---------------------------------------------------------------------------

__device__ inline int readlane_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ inline double readlane_f64s(double v, int l)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__global__ __launch_bounds__(kSampleThreads) void k_sample_mh(SampleArgs a)
{
    const int lane = (int)threadIdx.x;
    const int64_t total = (int64_t)a.P * a.nstep;
    int cur_p = a.mh[0], cur_i = a.mh[1];
    double cur_c = cur_i >= 0 ? a.coef[cur_i] : 0.0;
    for (int64_t base = 0; base < total; base += kSampleThreads) {
        const int64_t idx = base + lane;
        int pp = 0, ip = 0;
        double x = 0.0, cp = 0.0;
        if (idx < total) {
            const int s = (int)(idx / a.P), l = (int)(idx - (int64_t)s * a.P);
            uint64_t w[4];
            philox4x64_10((uint64_t)l, a.step + (uint64_t)s, 2, 0, a.seed, (uint64_t)a.replica, w);
            const double target = (double)(w[0] >> 11) * 0x1p-53 * a.Sq;
            int lo = 0, hi = a.nshell;
            while (lo < hi) {
                int mid = lo + ((hi - lo) >> 1);
                if (a.cdf_q[mid] > target) hi = mid; else lo = mid + 1;
            }
            ip = lo < a.nshell ? lo : a.nshell - 1;
            pp = a.first[ip] + (int)__umul64hi(w[1], (uint64_t)a.size[ip]);
            cp = a.coef[ip];
            x = (double)(w[2] >> 11) * 0x1p-53 * cp;
        }
        const int n = (int)((total - base) < kSampleThreads ? (total - base) : kSampleThreads);
        int my_p = 0, my_i = 0;
        for (int j = 0; j < n; ++j) {   // uniform: the chain in scalar registers
            const double xj = readlane_f64s(x, j);
            if (cur_i < 0 || xj < cur_c) {
                cur_p = readlane_i32(pp, j);
                cur_i = readlane_i32(ip, j);
                cur_c = readlane_f64s(cp, j);
            }
            if (lane == j) {
                my_p = cur_p;
                my_i = cur_i;
            }
        }
        if (idx < total) {
            const uint32_t pk = (uint32_t)a.lattice[my_p];
            const int nx = (int)(pk & 1023u) - 512, ny = (int)((pk >> 10) & 1023u) - 512;
            const int nz = (int)((pk >> 20) & 1023u) - 512;
            const double cf = a.coef[my_i];
            a.samp[idx] = make_double4((double)nx, (double)ny, (double)nz, cf);
            if (a.n_out) {
                const int l = (int)(idx % a.P);
                a.n_out[3 * l + 0] = nx;
                a.n_out[3 * l + 1] = ny;
                a.n_out[3 * l + 2] = nz;
                if (a.coef_out) a.coef_out[l] = cf;
            } else if (a.coef_out) {
                a.coef_out[idx % a.P] = cf;
            }
        }
    }
    if (lane == 0) {
        a.mh[0] = cur_p;
        a.mh[1] = cur_i;
    }
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t st)
{
    if (a.P < 1 || a.nstep < 1 || a.nshell < 1 || !a.cdf || !a.coef || !a.first || !a.size || !a.lattice ||
        !a.samp || (a.nstep > 1 && (a.n_out || a.coef_out)))
        return hipErrorInvalidValue;
    if (a.mh) {
        if (!a.cdf_q || !(a.Sq > 0.0)) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_sample_mh, dim3(1), dim3(kSampleThreads), 0, st, a);
        return hipGetLastError();
    }
    int64_t n = (int64_t)a.P * a.nstep;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + kSampleThreads - 1) / kSampleThreads)), dim3(kSampleThreads),
                       0, st, a);
    return hipGetLastError();
}


}  // namespace rbsog

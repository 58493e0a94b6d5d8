// gfx950 kernels of librbsog: the global baths of the time loop.
//
// Section 5.1 equilibrates in the NVT ensemble with Nose-Hoover dynamics; the
// other global scheme offered is Berendsen's weak coupling.  Either acts as a
// half-step operator T(dt/2) on the velocities before and after each
// velocity-Verlet step (g = 3N degrees of freedom, tau = 1/rate, K the kinetic
// energy):
//   Nose-Hoover, one thermostat of mass Q = g kT tau^2:
//     xi += (dt/4)(2K - g kT)/Q;  v *= e^{-xi dt/2};  eta += (dt/2) xi;
//     xi += (dt/4)(2K - g kT)/Q  (K taken after the scaling);
//   Berendsen: v *= lambda, lambda^2 = 1 + (dt/(2 tau))(g kT/(2K) - 1).
// Between two steps the closing half-step of one and the opening one of the
// next run back to back in one single-workgroup kernel, which leaves the
// product of their factors for the next first half-kick to apply.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace rbsog {

namespace {

__device__ inline double half_step(const BathArgs &a, double &xi, double &eta, double &K)
{
    if (a.kind == kBathNoseHoover) {
        xi += 0.25 * a.dt * (2.0 * K - a.gkT) / a.Q;
        const double sc = exp(-0.5 * a.dt * xi);
        K = K * (sc * sc);
        eta += 0.5 * a.dt * xi;
        xi += 0.25 * a.dt * (2.0 * K - a.gkT) / a.Q;
        return sc;
    }
    if (!(K > 0.0)) return 1.0;
    double lam2 = 1.0 + 0.5 * a.dt * a.rate * (a.gkT / (2.0 * K) - 1.0);
    if (lam2 < 0.0) lam2 = 0.0;
    K = K * lam2;
    return sqrt(lam2);
}

__global__ __launch_bounds__(kBlock) void k_bath(BathArgs a)
{
    __shared__ double red[kBlock];
    double k = 0.0;
    for (int b = threadIdx.x; b < a.nfar; b += kBlock) k += a.kepart[b];
    k = block_sum_256(k, red);
    if (threadIdx.x == 0) {
        double xi = a.bath[0], eta = a.bath[1], K = k, s = 1.0;
        if (a.mode & 2) {
            s = s * half_step(a, xi, eta, K);
            a.bath[3] = K;
        }
        if (a.mode & 1) s = s * half_step(a, xi, eta, K);
        a.bath[0] = xi;
        a.bath[1] = eta;
        a.bath[2] = s;
    }
}

// one partial per 64 particles, summed in a fixed tree (the far kernel's blocks)
__global__ __launch_bounds__(64) void k_ke_partials(int N, const double *__restrict__ vs,
                                                    const double *__restrict__ ms, double *__restrict__ kepart)
{
    __shared__ double red[64];
    const int t = (int)threadIdx.x, p = (int)blockIdx.x * 64 + t;
    double ke = 0.0;
    if (p < N) {
        const double vx = vs[p], vy = vs[N + p], vz = vs[2 * N + p];
        ke = 0.5 * ms[p] * (vx * vx + vy * vy + vz * vz);
    }
    red[t] = ke;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) kepart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kBlock) void k_scale_v(int N, double *__restrict__ vs, const double *__restrict__ scale)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < 3 * (int64_t)N) vs[k] = vs[k] * *scale;
}

}  // namespace

hipError_t launch_bath(const BathArgs &a, hipStream_t st)
{
    if ((a.kind != kBathNoseHoover && a.kind != kBathBerendsen) || a.mode < 1 || a.mode > 3 || a.nfar < 1 ||
        !a.kepart || !a.bath || !(a.dt > 0.0) || !(a.gkT > 0.0) || !(a.rate > 0.0) ||
        (a.kind == kBathNoseHoover && !(a.Q > 0.0)))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bath, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_ke_partials(int N, const double *vs, const double *ms, double *kepart, hipStream_t st)
{
    if (N < 1 || !vs || !ms || !kepart) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ke_partials, dim3(far_blocks(N)), dim3(64), 0, st, N, vs, ms, kepart);
    return hipGetLastError();
}

hipError_t launch_scale_v(int N, double *vs, const double *scale, hipStream_t st)
{
    if (N < 1 || !vs || !scale) return hipErrorInvalidValue;
    const int64_t n = 3 * (int64_t)N;
    hipLaunchKernelGGL(k_scale_v, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, N, vs, scale);
    return hipGetLastError();
}

}  // namespace rbsog

// Issue cost of FP64 elementary functions on gfx950, measured: the price the
// throughput roofline puts on the exponentials, square roots and sines and
// cosines that the method's pair and mode sums call for.  Each kernel runs
// eight independent dependent chains per lane of one operation (the device
// library's double exp, sincos or sqrt, or a plain FMA as the unit), on a
// grid that fills every compute unit; the ratio of a function's time per call
// to the FMA's is its cost in FMA issue slots.  Not part of the force path:
// the benchmark loads this library (libprice.so) on its own.
#include <hip/hip_runtime.h>

#include <cmath>

namespace {

constexpr int kChains = 8;
constexpr int kThreads = 256;

enum Op { kFma = 0, kExp = 1, kSinCos = 2, kSqrt = 3, kRsqrt = 4 };

template <int OP>
__global__ __launch_bounds__(kThreads) void k_price(double *out, int iters, double seed)
{
    double x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = seed + 1e-7 * (double)(threadIdx.x + kThreads * k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            if (OP == kFma) {
                x[k] = fma(x[k], 0.9999999, 1e-9);        // stays near 1e-2
            } else if (OP == kExp) {
                x[k] = exp(-x[k]);                         // fixed point 0.567
            } else if (OP == kSinCos) {
                double s, c;
                sincos(x[k], &s, &c);
                x[k] = fma(c, 0.5, s);                     // one FMA beside the call
            } else if (OP == kSqrt) {
                x[k] = sqrt(x[k] + 1.0);                   // one add beside the call
            } else {
                x[k] = rsqrt(x[k] + 1.0);
            }
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc += x[k];
    out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

}  // namespace

// Runs operation `op` (0 FMA, 1 exp, 2 sincos, 3 sqrt, 4 rsqrt) for `iters`
// iterations of eight chains per lane on `blocks` workgroups of 256 lanes and
// writes the kernel's milliseconds (HIP events) to *ms.  Allocates and frees
// its own output buffer.  Returns 0, or -1 on a bad argument or HIP error.
extern "C" int rbsog_price_run(int op, int iters, int blocks, double *ms)
{
    if (op < 0 || op > 4 || iters < 1 || blocks < 1 || !ms) return -1;
    double *out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&out, sizeof(double) * (size_t)blocks * kThreads);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto launch = [&](int n) {
        switch (op) {
        case kFma: hipLaunchKernelGGL(k_price<kFma>, dim3(blocks), dim3(kThreads), 0, 0, out, n, 0.01); break;
        case kExp: hipLaunchKernelGGL(k_price<kExp>, dim3(blocks), dim3(kThreads), 0, 0, out, n, 0.5); break;
        case kSinCos: hipLaunchKernelGGL(k_price<kSinCos>, dim3(blocks), dim3(kThreads), 0, 0, out, n, 0.3); break;
        case kSqrt: hipLaunchKernelGGL(k_price<kSqrt>, dim3(blocks), dim3(kThreads), 0, 0, out, n, 1.0); break;
        default: hipLaunchKernelGGL(k_price<kRsqrt>, dim3(blocks), dim3(kThreads), 0, 0, out, n, 1.0); break;
        }
        return hipGetLastError();
    };
    if (e == hipSuccess) e = launch(1);   // warm-up (code object load)
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipEventRecord(e0, 0);
    if (e == hipSuccess) e = launch(iters);
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return -1;
    *ms = (double)t;
    return 0;
}

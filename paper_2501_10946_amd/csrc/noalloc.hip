// rbsog_rho_noalloc: the structure factors of given modes (the computation of
// rbsog_compute_rho, with the caller's modes instead of drawn ones) for
// callers that cannot allocate device memory.  Every buffer beyond the
// caller's inputs and output -- the modes as the kernels read them, the
// rotation table, the per-(group, mode) partial sums and the reduction's
// outputs -- lives in one file-scope device array of kScratchBytes, which each
// GPU the library runs on holds until the process ends.  The kernels are those
// of rbsog_compute_rho, with the same group size, so both entry points give
// the same sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "system.h"

namespace rbsog {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kMaxDevices = 64;

// The scratch array.  In host code its name is a host-side stand-in, never a
// device address: kernels and copies get the address resolved per device at
// set-up (scratch_ptr).
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};

// Resolves this device's copy of `scratch` and fills its rotation table, once
// per device (synchronously; the first call on a device must not be captured).
int scratch_ptr(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RBSOG_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(RBSOG_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(RBSOG_EHIP, "hipGetSymbolAddress: %s", hipGetErrorString(e));
        double tab[2 * kPhaseTable];
        phase_table(tab);
        e = hipMemcpy(p, tab, sizeof(tab), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(RBSOG_EHIP, "rotation table: %s", hipGetErrorString(e));
        g_ptr[dev] = (char *)p;
    }
    *out = g_ptr[dev];
    return RBSOG_OK;
}

// samp[l] = (n_x, n_y, n_z, 0) of the caller's int32 modes
__global__ __launch_bounds__(kBlock) void k_modes_from_n(const int32_t *__restrict__ n, double4 *__restrict__ samp,
                                                          int P)
{
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l < P) samp[l] = make_double4((double)n[3 * l], (double)n[3 * l + 1], (double)n[3 * l + 2], 0.0);
}

}  // namespace
}  // namespace rbsog

using namespace rbsog;

extern "C" int rbsog_rho_noalloc(int64_t N, double L, const double *x_dev, const double *q_dev, int P,
                                 const int32_t *n_dev, int precision, void *hip_stream, double *rho_dev)
{
    if (N < 1 || N > ((int64_t)1 << 27) - 1) return fail(RBSOG_EINVAL, "N must lie in [1, 2^27 - 1]");
    if (P < 1 || P > 4096) return fail(RBSOG_EINVAL, "P must lie in [1, 4096]");
    if (!(L > 0.0) || !std::isfinite(L)) return fail(RBSOG_EINVAL, "L must be positive and finite");
    if (precision != RBSOG_FP64 && precision != RBSOG_MIXED) return fail(RBSOG_EINVAL, "unknown precision");
    if (!x_dev || !q_dev || !n_dev || !rho_dev) return fail(RBSOG_EINVAL, "null x, q, n or rho");
    // layout of the scratch: rotation table, modes, rho, coef rho, energy terms, partials
    const int chunk = rho_chunk((int)N, P);
    const int nchunk = (int)((N + chunk - 1) / chunk);
    const size_t o_tab = 0;
    const size_t o_samp = align_up(o_tab + sizeof(double2) * kPhaseTable);
    const size_t o_rho = align_up(o_samp + sizeof(double4) * (size_t)P);
    const size_t o_gk = align_up(o_rho + sizeof(double2) * (size_t)P);
    const size_t o_eF = align_up(o_gk + sizeof(double2) * (size_t)P);
    const size_t o_part = align_up(o_eF + sizeof(double) * (size_t)P);
    const size_t need = o_part + sizeof(double2) * (size_t)nchunk * (size_t)P;
    if (need > kScratchBytes)
        return fail(RBSOG_EINVAL, "N = %lld and P = %d need %zu scratch bytes, beyond the %zu of rbsog_rho_noalloc",
                    (long long)N, P, need, kScratchBytes);
    char *s = nullptr;
    int rc = scratch_ptr(&s);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    RhoArgs a{};
    a.N = (int)N;
    a.P = P;
    a.chunk = chunk;
    a.nchunk = nchunk;
    a.inv_L[0] = a.inv_L[1] = a.inv_L[2] = 1.0 / L;
    a.xs = nullptr;
    a.x = x_dev;
    a.q = q_dev;
    a.samp = (const double4 *)(s + o_samp);
    a.part = (double2 *)(s + o_part);
    a.rho = (double2 *)(s + o_rho);
    a.gk = (double2 *)(s + o_gk);
    a.eF = (double *)(s + o_eF);
    a.rho_out = rho_dev;
    a.mixed = precision == RBSOG_MIXED;
    a.tab = (const double2 *)(s + o_tab);
    a.ss = make_sincos_short();
    hipLaunchKernelGGL(k_modes_from_n, dim3((P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, n_dev,
                       (double4 *)(s + o_samp), P);
    HIPCHECK(hipGetLastError());
    HIPCHECK(launch_rho_partial(a, st));
    HIPCHECK(launch_rho_reduce(a, st));
    return RBSOG_OK;
}

// Observables of Section 5.1 on the device: the static structure factor by
// lattice shell (computed with the structure-factor kernels of the far field
// over every mode of the shells), the pair-distance histogram behind the
// radial distribution function (over the fine cell grid of a system), and the
// unwrapped displacements behind the mean squared displacement with the
// velocity autocorrelation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dev_common.h"
#include "system.h"

namespace rbsog {
namespace {

// modes in flight per pass of the structure-factor kernels
constexpr int kSsfModes = 1024;

struct SsfPlan {
    int64_t K;   // modes with 1 <= |n|^2 <= m_s
    int P;       // modes per pass (the last pass takes the rest)
    size_t o_tab, o_modes, o_rho, o_gk, o_eF, o_start, o_part, total;
};

// partial sums of a pass of P modes: its particle groups times P
size_t ssf_partials(int64_t N, int P)
{
    const int c = rho_chunk((int)N, P);
    return (size_t)((N + c - 1) / c) * (size_t)P;
}

SsfPlan ssf_plan(int64_t N, int m_s)
{
    SsfPlan p{};
    p.K = lattice_points(m_s);
    p.P = (int)std::max<int64_t>(1, std::min<int64_t>(p.K, kSsfModes));
    const int rest = (int)(p.K % p.P);
    const size_t npart = std::max(ssf_partials(N, p.P), rest ? ssf_partials(N, rest) : (size_t)0);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    p.o_tab = take(sizeof(double2) * kPhaseTable);
    p.o_modes = take(sizeof(double4) * (size_t)std::max<int64_t>(p.K, 1));
    p.o_rho = take(sizeof(double2) * (size_t)std::max<int64_t>(p.K, 1));
    p.o_gk = take(sizeof(double2) * (size_t)p.P);
    p.o_eF = take(sizeof(double) * (size_t)p.P);
    p.o_start = take(sizeof(int64_t) * ((size_t)m_s + 2));
    p.o_part = take(sizeof(double2) * npart);
    p.total = off;
    return p;
}

// s[m] = mean over the modes of shell m of |rho|^2, summed in mode order
__global__ __launch_bounds__(kBlock) void k_ssf_shells(const double2 *__restrict__ rho,
                                                       const int64_t *__restrict__ start, int m_s,
                                                       double *__restrict__ s)
{
    const int m = blockIdx.x * kBlock + threadIdx.x;
    if (m > m_s) return;
    const int64_t a = start[m], b = start[m + 1];
    double acc = 0.0;
    for (int64_t p = a; p < b; ++p) acc += rho[p].x * rho[p].x + rho[p].y * rho[p].y;
    s[m] = b > a ? acc / (double)(b - a) : 0.0;
}

// ---------------------------------------------------------------------------
// pair-distance histogram
// ---------------------------------------------------------------------------

struct RdfArgs {
    int N, nbins;
    CellGeom g;               // the fine grid: cells >= r_max / 2 wide, 5 x 5 x 5 stencil
    const double4 *xs;        // cell order
    const int32_t *cell_start;
    double rmax2, dr;
    unsigned long long *hist;
};

constexpr int kRdfMaxBins = 4096;

// One particle per thread walks the 5 x 5 x 5 cells around its own (images
// through the cell shift, so each neighbour within r_max <= L/3 is met once)
// and bins every other particle with r < r_max; a workgroup's counts go
// through LDS, then one 64-bit atomic add per non-empty bin.  Integer counts:
// the result does not depend on the order of the additions.
__global__ __launch_bounds__(kBlock) void k_rdf(RdfArgs a)
{
    __shared__ unsigned int h[kRdfMaxBins];
    for (int b = threadIdx.x; b < a.nbins; b += kBlock) h[b] = 0u;
    __syncthreads();
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < a.N) {
        const double4 r = a.xs[p];
        const int ncx = a.g.nc[0], ncy = a.g.nc[1], ncz = a.g.nc[2];
        const int cx = cell_coord(r.x, a.g.inv_cell[0], ncx), cy = cell_coord(r.y, a.g.inv_cell[1], ncy),
                  cz = cell_coord(r.z, a.g.inv_cell[2], ncz);
        for (int dz = -2; dz <= 2; ++dz) {
            int z = cz + dz;
            double sz = 0.0;
            if (z < 0) { z += ncz; sz = -a.g.L[2]; } else if (z >= ncz) { z -= ncz; sz = a.g.L[2]; }
            for (int dy = -2; dy <= 2; ++dy) {
                int y = cy + dy;
                double sy = 0.0;
                if (y < 0) { y += ncy; sy = -a.g.L[1]; } else if (y >= ncy) { y -= ncy; sy = a.g.L[1]; }
                for (int dx = -2; dx <= 2; ++dx) {
                    int x = cx + dx;
                    double sx = 0.0;
                    if (x < 0) { x += ncx; sx = -a.g.L[0]; } else if (x >= ncx) { x -= ncx; sx = a.g.L[0]; }
                    const int c = (z * ncy + y) * ncx + x;
                    for (int j = a.cell_start[c]; j < a.cell_start[c + 1]; ++j) {
                        if (j == p) continue;
                        const double4 q = a.xs[j];
                        const double ux = r.x - (q.x + sx), uy = r.y - (q.y + sy), uz = r.z - (q.z + sz);
                        const double r2 = ux * ux + uy * uy + uz * uz;
                        if (r2 < a.rmax2) {
                            int b = (int)floor(sqrt(r2) / a.dr);
                            if (b >= a.nbins) b = a.nbins - 1;
                            atomicAdd(&h[b], 1u);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < a.nbins; b += kBlock)
        if (h[b]) atomicAdd(&a.hist[b], (unsigned long long)h[b]);
}

// ---------------------------------------------------------------------------
// displacement tracking, MSD and VACF
// ---------------------------------------------------------------------------

struct TrackBox {
    double L[3], inv_L[3];
};

__global__ __launch_bounds__(kBlock) void k_track(int64_t N, TrackBox b, const double *__restrict__ x,
                                                  double *__restrict__ x_last, double *__restrict__ disp)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= 3 * N) return;
    const int a = (int)(k / N);   // the axis of component k (SoA [3][N])
    const double xn = x[k];
    double d = xn - x_last[k];
    d = d - b.L[a] * rint(d * b.inv_L[a]);
    disp[k] += d;
    x_last[k] = xn;
}

constexpr int kMsdBlocks = 1024;   // fixed grid: partials summed in one order whatever N is

// per-block partial sums of |disp|^2 and v0 . v over a fixed grid-stride
// assignment of particles, then one block adds the partials in block order
__global__ __launch_bounds__(kBlock) void k_msd_part(int64_t N, const double *__restrict__ disp,
                                                     const double *__restrict__ v0, const double *__restrict__ v,
                                                     double2 *__restrict__ part)
{
    __shared__ double red[kBlock];
    double m = 0.0, c = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (int64_t)kMsdBlocks * kBlock)
        for (int d = 0; d < 3; ++d) {
            const double u = disp[d * N + i];
            m = fma(u, u, m);
            c = fma(v0[d * N + i], v[d * N + i], c);
        }
    m = block_sum_256(m, red);
    __syncthreads();
    c = block_sum_256(c, red);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(m, c);
}

__global__ __launch_bounds__(kBlock) void k_msd_final(int64_t N, const double2 *__restrict__ part,
                                                      double *__restrict__ out)
{
    __shared__ double red[kBlock];
    double m = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < kMsdBlocks; b += kBlock) {
        m += part[b].x;
        c += part[b].y;
    }
    m = block_sum_256(m, red);
    __syncthreads();
    c = block_sum_256(c, red);
    if (threadIdx.x == 0) {
        out[0] = m / (double)N;
        out[1] = c / (double)N;
    }
}

}  // namespace
}  // namespace rbsog

using namespace rbsog;

extern "C" int rbsog_track_box(int64_t N, double Lx, double Ly, double Lz, const double *x_dev, double *x_last_dev,
                               double *disp_dev, void *hip_stream)
{
    if (N < 1 || N > ((int64_t)1 << 27) - 1) return fail(RBSOG_EINVAL, "N must lie in [1, 2^27 - 1]");
    const double Lb[3] = {Lx, Ly, Lz};
    TrackBox b{};
    for (int a = 0; a < 3; ++a) {
        if (!(Lb[a] > 0.0) || !std::isfinite(Lb[a])) return fail(RBSOG_EINVAL, "box edges must be positive and finite");
        b.L[a] = Lb[a];
        b.inv_L[a] = 1.0 / Lb[a];
    }
    if (!x_dev || !x_last_dev || !disp_dev) return fail(RBSOG_EINVAL, "null x, x_last or disp");
    const int64_t n3 = 3 * N;
    hipLaunchKernelGGL(k_track, dim3((unsigned)((n3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, (hipStream_t)hip_stream,
                       N, b, x_dev, x_last_dev, disp_dev);
    HIPCHECK(hipGetLastError());
    return RBSOG_OK;
}

extern "C" int rbsog_track(int64_t N, double L, const double *x_dev, double *x_last_dev, double *disp_dev,
                           void *hip_stream)
{
    if (!(L > 0.0) || !std::isfinite(L)) return fail(RBSOG_EINVAL, "L must be positive and finite");
    return rbsog_track_box(N, L, L, L, x_dev, x_last_dev, disp_dev, hip_stream);
}

extern "C" int rbsog_msd_scratch_size(size_t *bytes)
{
    if (!bytes) return fail(RBSOG_EINVAL, "null bytes");
    *bytes = sizeof(double2) * kMsdBlocks;
    return RBSOG_OK;
}

extern "C" int rbsog_msd_vacf(int64_t N, const double *disp_dev, const double *v0_dev, const double *v_dev,
                              void *scratch_dev, size_t scratch_bytes, void *hip_stream, double *out_dev)
{
    if (N < 1 || N > ((int64_t)1 << 27) - 1) return fail(RBSOG_EINVAL, "N must lie in [1, 2^27 - 1]");
    if (!disp_dev || !v0_dev || !v_dev || !scratch_dev || !out_dev)
        return fail(RBSOG_EINVAL, "null disp, v0, v, scratch or out");
    if (scratch_bytes < sizeof(double2) * kMsdBlocks)
        return fail(RBSOG_EWORKSPACE, "scratch of %zu bytes is below the %zu needed", scratch_bytes,
                    sizeof(double2) * kMsdBlocks);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_msd_part, dim3(kMsdBlocks), dim3(kBlock), 0, st, N, disp_dev, v0_dev, v_dev,
                       (double2 *)scratch_dev);
    HIPCHECK(hipGetLastError());
    hipLaunchKernelGGL(k_msd_final, dim3(1), dim3(kBlock), 0, st, N, (const double2 *)scratch_dev, out_dev);
    HIPCHECK(hipGetLastError());
    return RBSOG_OK;
}

extern "C" int rbsog_ssf_scratch_size(int64_t N, int m_s, size_t *bytes)
{
    if (!bytes) return fail(RBSOG_EINVAL, "null bytes");
    if (N < 1 || N > ((int64_t)1 << 27) - 1) return fail(RBSOG_EINVAL, "N must lie in [1, 2^27 - 1]");
    if (m_s < 1 || m_s > kMaxLatticeM) return fail(RBSOG_EINVAL, "m_s must lie in [1, %d]", kMaxLatticeM);
    *bytes = ssf_plan(N, m_s).total;
    return RBSOG_OK;
}

extern "C" int rbsog_ssf(int64_t N, double L, const double *x_dev, const double *w_dev, int m_s, void *scratch_dev,
                         size_t scratch_bytes, void *hip_stream, double *s_dev)
{
    size_t need = 0;
    int rc = rbsog_ssf_scratch_size(N, m_s, &need);
    if (rc) return rc;
    if (!(L > 0.0) || !std::isfinite(L)) return fail(RBSOG_EINVAL, "L must be positive and finite");
    if (!x_dev || !w_dev || !s_dev || !scratch_dev) return fail(RBSOG_EINVAL, "null x, w, s or scratch");
    if (((uintptr_t)scratch_dev % kAlign) != 0) return fail(RBSOG_EINVAL, "scratch must be 256-byte aligned");
    if (scratch_bytes < need) return fail(RBSOG_EWORKSPACE, "scratch of %zu bytes is below the %zu needed", scratch_bytes, need);
    const SsfPlan pl = ssf_plan(N, m_s);
    hipStream_t st = (hipStream_t)hip_stream;
    char *s = (char *)scratch_dev;
    // modes of the shells in (|n|^2, nx, ny, nz) order, unit weight, and the
    // first mode of each shell
    std::vector<int32_t> packed((size_t)pl.K);
    lattice_copy(m_s, packed.data());
    std::vector<double> modes(4 * (size_t)pl.K);
    std::vector<int64_t> start((size_t)m_s + 2, 0);
    for (int64_t i = 0; i < pl.K; ++i) {
        const uint32_t pk = (uint32_t)packed[(size_t)i];
        const int nx = (int)(pk & 1023u) - kLatticeBias, ny = (int)((pk >> 10) & 1023u) - kLatticeBias;
        const int nz = (int)((pk >> 20) & 1023u) - kLatticeBias;
        modes[4 * i] = nx;
        modes[4 * i + 1] = ny;
        modes[4 * i + 2] = nz;
        modes[4 * i + 3] = 1.0;
        start[(size_t)(nx * nx + ny * ny + nz * nz) + 1] += 1;
    }
    for (int m = 1; m <= m_s + 1; ++m) start[(size_t)m] += start[(size_t)m - 1];
    double tab[2 * kPhaseTable];
    phase_table(tab);
    HIPCHECK(hipMemcpyAsync(s + pl.o_tab, tab, sizeof(tab), hipMemcpyHostToDevice, st));
    if (pl.K > 0)
        HIPCHECK(hipMemcpyAsync(s + pl.o_modes, modes.data(), sizeof(double) * modes.size(), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(s + pl.o_start, start.data(), sizeof(int64_t) * start.size(), hipMemcpyHostToDevice, st));
    const double4 *dm = (const double4 *)(s + pl.o_modes);
    double2 *drho = (double2 *)(s + pl.o_rho);
    for (int64_t c0 = 0; c0 < pl.K; c0 += pl.P) {
        RhoArgs a{};
        a.N = (int)N;
        a.P = (int)std::min<int64_t>(pl.P, pl.K - c0);
        a.chunk = rho_chunk((int)N, a.P);
        a.nchunk = (int)((N + a.chunk - 1) / a.chunk);
        a.inv_L[0] = a.inv_L[1] = a.inv_L[2] = 1.0 / L;
        a.x = x_dev;
        a.q = w_dev;
        a.samp = dm + c0;
        a.part = (double2 *)(s + pl.o_part);
        a.rho = drho + c0;
        a.gk = (double2 *)(s + pl.o_gk);
        a.eF = (double *)(s + pl.o_eF);
        a.mixed = 0;
        a.tab = (const double2 *)(s + pl.o_tab);
        a.ss = make_sincos_short();
        HIPCHECK(launch_rho_partial(a, st));
        HIPCHECK(launch_rho_reduce(a, st));
    }
    hipLaunchKernelGGL(k_ssf_shells, dim3((m_s + 1 + kBlock - 1) / kBlock), dim3(kBlock), 0, st, drho,
                       (const int64_t *)(s + pl.o_start), m_s, s_dev);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));   // the host-side mode tables are released on return
    return RBSOG_OK;
}

extern "C" int rbsog_rdf(rbsog_handle *h, const double *x_dev, double r_max, int nbins, unsigned long long *hist_dev)
{
    if (!h || !x_dev || !hist_dev) return fail(RBSOG_EINVAL, "null handle, x or hist");
    if (!(r_max > 0.0) || !(r_max <= h->sog.r_c)) return fail(RBSOG_EINVAL, "r_max must lie in (0, r_c]");
    if (nbins < 1 || nbins > kRdfMaxBins) return fail(RBSOG_EINVAL, "nbins must lie in [1, %d]", kRdfMaxBins);
    // the positions into cell order on the fine grid (cells >= r_c / 2 >= r_max / 2)
    PermArgs in = perm_args(h, (double *)x_dev, nullptr, nullptr);
    HIPCHECK(launch_state_in(in, h->st));
    CellArgs ca = cell_args(h, h->gf, nullptr, false);
    HIPCHECK(launch_cell_build(ca, h->st));
    h->lists_valid = false;   // the rows moved: the next evaluation builds its lists again
    RdfArgs a{};
    a.N = (int)h->p.N;
    a.nbins = nbins;
    a.g = h->gf;
    a.xs = h->xs;
    a.cell_start = h->cell_start;
    a.rmax2 = r_max * r_max;
    a.dr = r_max / nbins;
    a.hist = hist_dev;
    for (int d = 0; d < 3; ++d)
        if (a.g.nc[d] < 5) return fail(RBSOG_EINVAL, "fine grid of %d cells is below the 5-cell stencil", a.g.nc[d]);
    hipLaunchKernelGGL(k_rdf, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, h->st, a);
    HIPCHECK(hipGetLastError());
    return RBSOG_OK;
}

// Host-only audit of the workspace plan (no GPU needed): for a sweep of
// system parameters, every buffer the kernels index holds the largest index
// their launch shapes can reach, on every cell grid a system can use (the
// coarse grid of rbsog_build_cells, the fine grid of the force evaluation, and
// the finer grid a hot system's default skin drops to), and the fine grids'
// 5 x 5 x 5 stencil covers the list radius.  Prints one line per failure and
// exits non-zero if any.  A second part checks that every launcher refuses
// arguments that would send a kernel outside its buffers (a missing buffer, a
// grid too coarse for the 5 x 5 x 5 stencil, a structure-factor group beyond
// the staging area) on the host, before anything is launched; it runs only
// where no GPU is visible, so that a missing check cannot launch a kernel on
// the placeholder pointers it passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "system.h"

using namespace rbsog;


static int failures = 0;

#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            ++failures;                                    \
            std::printf("FAIL %s: ", #cond);               \
            std::printf(__VA_ARGS__);                      \
            std::printf("\n");                             \
        }                                                  \
    } while (0)

static size_t span(size_t a, size_t b) { return b - a; }   // bytes between two consecutive offsets

static void audit(int64_t N, const double Lb[3], double lambda, double rc, int P, double skin)
{
    const double L = Lb[0];
    rbsog_sog s{};
    if (rbsog_sog_init(lambda, rc, 1e-4, 1, RBSOG_AUTO, RBSOG_AUTO, &s) != RBSOG_OK) {
        std::printf("skip: no SOG for lambda %g r_c %g\n", lambda, rc);
        return;
    }
    rbsog_params p{};
    p.N = N;
    p.L = L;
    p.kT = 1.0;
    p.P = P;
    p.mmax = 0;
    p.seed = 1;
    p.precision = RBSOG_FP64;
    p.density = RBSOG_ADAPTIVE;
    p.skin = skin;
    p.full_k = 0;
    p.Ly = Lb[1];
    p.Lz = Lb[2];
    if (check_params(&p, &s) != RBSOG_OK) return;   // refused before any launch
    const Derived d = derive(&p, &s);
    const Layout w = make_layout(N, d, P, false);
    char tag[160];
    std::snprintf(tag, sizeof tag, "N %lld L %.4g x %.4g x %.4g lambda %g r_c %g P %d skin %g", (long long)N, Lb[0],
                  Lb[1], Lb[2], lambda, rc, P, skin);
    // cell grids the kernels can index: coarse, fine, fine of a dropped skin
    const int *grids[3] = {d.nc, d.nf, d.nf_tight};
    for (const int *g : grids) {
        const size_t ncell = (size_t)g[0] * g[1] * g[2];
        CHECK(span(w.count, w.cell_start) >= 4 * ncell, "%s grid %d: counts", tag, g[0]);
        CHECK(span(w.cell_start, w.fill) >= 4 * (ncell + 1), "%s grid %d: cell starts", tag, g[0]);
        CHECK(span(w.fill, w.tmp) >= 4 * ncell, "%s grid %d: fill", tag, g[0]);
        CHECK(span(w.tile_sum, w.xb) >= 4 * (size_t)scan_tiles((int)ncell), "%s grid %d: scan tiles", tag, g[0]);
    }
    for (int a = 0; a < 3; ++a) {
        // the 5-cell stencil of each fine grid reaches the list radius; at least 6 cells
        CHECK(d.nf[a] >= 6 && d.nf_tight[a] >= 6, "%s: fine grid below 6 cells (axis %d)", tag, a);
        CHECK(d.rl <= 2.0 * Lb[a] / d.nf[a] * (1 + 1e-15), "%s: list radius %g beyond the stencil of %d cells", tag,
              d.rl, d.nf[a]);
        CHECK(rc <= 2.0 * Lb[a] / d.nf_tight[a] * (1 + 1e-15), "%s: r_c beyond the stencil of the tight grid", tag);
        CHECK(d.nf_tight[a] >= d.nf[a], "%s: the tight grid is coarser", tag);
    }
    // the sampling tables hold one entry per shell (cube) or per point (cuboid)
    CHECK(span(w.cdf, w.coef) >= 8 * (size_t)d.nshells && span(w.cdf_q, w.mh) >= 8 * (size_t)d.nshells,
          "%s: sampling tables", tag);
    CHECK(d.cuboid ? d.nshells == d.nlat : d.nshells == d.mmax, "%s: table capacity", tag);
    // neighbour lists: list_rows(kp) entries per particle of the padded tiles, for
    // both list radii (the capacity only shrinks when the skin drops)
    const int kp_tight = near_capacity(N, Lb[0] * Lb[1] * Lb[2], rc);
    const int kp = d.kp > kp_tight ? d.kp : kp_tight;
    const int rows = list_rows(kp);
    CHECK(rows % kListBlock == 0 && rows >= 5 * kp, "%s: list rows of whole blocks", tag);
    CHECK(span(w.nbr, w.nbr_cnt) >= 4 * (size_t)rows * (size_t)list_padded(N), "%s: list rows", tag);
    CHECK(list_at((int)list_padded(N) - 1, rows - 1, rows) < (size_t)rows * (size_t)list_padded(N),
          "%s: last list entry", tag);
    // the evaluation reads a particle's block b as two int4 at list_at(p, 8 b, rows): 16-byte aligned
    CHECK(list_at(63, kListBlock, rows) - list_at(63, 0, rows) == (size_t)kListBlock &&
          list_at(1, 0, rows) % 4 == 0, "%s: block stride", tag);
    // structure-factor partials: groups of the standalone launch and of the
    // shared launch (both precisions) within the buffer
    const size_t part_cap = span(w.part, w.rho) / 16;
    for (int mixed = 0; mixed < 2; ++mixed) {
        const int c = rho_chunk_shared((int)N, P, mixed != 0);
        const size_t nch = (size_t)((N + c - 1) / c);
        CHECK(nch * (size_t)P <= part_cap, "%s: shared-launch partials (mixed %d)", tag, mixed);
        CHECK((255 / P + 2) * c <= kRhoStage, "%s: staged groups exceed the stage (mixed %d)", tag, mixed);
    }
    {
        const int c = rho_chunk((int)N, P);
        CHECK((size_t)((N + c - 1) / c) * (size_t)P <= part_cap, "%s: standalone partials", tag);
    }
    CHECK(span(w.samp, w.part) >= 32 * (size_t)P * (size_t)d.sbatch, "%s: sampled modes", tag);
    CHECK(span(w.fnear, w.epart) >= 8 * 3 * (size_t)kNearLanes * (size_t)N, "%s: near partial forces", tag);
    CHECK(span(w.epart, w.kepart) >= 16 * (size_t)near_blocks((int)N), "%s: near energy and virial partials", tag);
    CHECK(span(w.eW, w.vm) >= 8 * (size_t)d.nmodes, "%s: virial terms of the modes", tag);
    // the reduction indexes vm by |n|^2 of a sampled mode, at most m_max
    CHECK(span(w.vm, w.fnear) >= 8 * ((size_t)d.mmax + 1), "%s: virial factors by |n|^2", tag);
    CHECK(span(w.kepart, w.flag) >= 8 * (size_t)far_blocks((int)N), "%s: kinetic partials", tag);
    CHECK(span(w.xs, w.xs_old) >= 32 * (size_t)N && span(w.ms, w.ms_old) >= 8 * (size_t)N, "%s: rows", tag);
    CHECK(span(w.tab, w.tab_far) >= 16 * (size_t)kPhaseTable, "%s: rotation table", tag);
    CHECK(span(w.tab_far, w.cdf_q) >= 16 * (size_t)kFarTable, "%s: far rotation table", tag);
    CHECK(span(w.cdf_q, w.mh) >= 8 * (size_t)d.nshells, "%s: proposal CDF of the chain", tag);
    CHECK(span(w.mh, w.bath) >= 8, "%s: chain state", tag);
    CHECK(span(w.bath, w.fab) >= 8 * (size_t)kBathWords, "%s: bath state", tag);
    CHECK(w.total >= w.fab + 16 * (size_t)kMaxGauss, "%s: total", tag);
}

// every call below carries one argument a kernel cannot run on, and must be
// refused with hipErrorInvalidValue
static void guards()
{
    static double4 d4[4];
    static double d[16];
    static double2 d2[4];
    static int32_t i32[16];
    static int32_t *const ip = i32;
    auto refused = [](hipError_t e, const char *what) {
        CHECK(e == hipErrorInvalidValue, "launch not refused: %s (returned %d)", what, (int)e);
    };
    // cells: every buffer present but one
    CellArgs c{};
    c.N = 10;
    c.g.nc[0] = c.g.nc[1] = c.g.nc[2] = 3;
    c.g.ncell = 27;
    c.xs = d4;
    c.order = ip;
    c.xs_old = d4;
    c.order_old = ip;
    c.ms = d;
    c.ms_old = d;
    c.xb = d;
    c.cell_id = ip;
    c.count = ip;
    c.cell_start = ip;
    c.fill = ip;
    c.tmp = ip;
    c.tile_sum = ip;
    c.ticket = nullptr;
    refused(launch_cell_build(c, nullptr), "cell build without the scan ticket");
    c.ticket = ip;
    c.N = 0;
    refused(launch_cell_build(c, nullptr), "cell build of no particles");
    c.N = 10;
    c.vs = d;   // velocities to move but no snapshot of them
    refused(launch_cell_build(c, nullptr), "cell build moving velocities without their snapshot");
    // global baths
    BathArgs ba{};
    ba.kind = kBathNoseHoover;
    ba.mode = 3;
    ba.dt = 0.01;
    ba.gkT = 30.0;
    ba.Q = 1.0;
    ba.rate = 1.0;
    ba.nfar = 1;
    ba.kepart = d;
    ba.bath = d;
    BathArgs bb = ba;
    bb.mode = 0;
    refused(launch_bath(bb, nullptr), "bath step of no half-step");
    bb = ba;
    bb.kind = 1;
    refused(launch_bath(bb, nullptr), "bath kernel for a local (Langevin) bath");
    bb = ba;
    bb.Q = 0.0;
    refused(launch_bath(bb, nullptr), "Nose-Hoover of no mass");
    bb = ba;
    bb.kepart = nullptr;
    refused(launch_bath(bb, nullptr), "bath without kinetic partials");
    refused(launch_ke_partials(0, d, d, d, nullptr), "kinetic partials of no particles");
    refused(launch_scale_v(4, d, nullptr, nullptr), "velocity scaling without its factor");
    // near field
    NearArgs n{};
    n.N = 10;
    n.g.nc[0] = n.g.nc[1] = n.g.nc[2] = 6;
    n.g.ncell = 216;
    n.rc2 = 1.0;
    n.rl2 = 1.2;
    n.w[0] = n.w[1] = n.w[2] = 1.0;
    n.kp = 4;
    n.xs = d4;
    n.cell_start = ip;
    n.nbr = ip;
    n.nbr_cnt = ip;
    n.fnear = d;
    n.sog.n = 2;
    NearArgs b = n;
    b.g.nc[2] = 5;
    refused(launch_nlist(b, nullptr), "list build on a grid of 5 cells (the stencil would wrap onto itself)");
    refused(launch_near(b, nullptr), "evaluation on a grid of 5 cells");
    b = n;
    b.rl2 = 0.9;
    refused(launch_nlist(b, nullptr), "list radius below r_c");
    b = n;
    b.kp = 0;
    refused(launch_nlist(b, nullptr), "list of no capacity");
    b = n;
    b.nbr = nullptr;
    refused(launch_near(b, nullptr), "evaluation without lists");
    b = n;
    b.energy = 1;
    refused(launch_near(b, nullptr), "energies without their partials");
    b = n;
    b.sog.n = 0;
    refused(launch_near(b, nullptr), "no Gaussians");
    b.sog.n = kMaxGauss + 1;
    refused(launch_near(b, nullptr), "more Gaussians than the argument block holds");
    b = n;
    b.nrho = 4;
    refused(launch_near(b, nullptr), "structure-factor workgroups not a multiple of 8");
    // structure factors
    RhoArgs r{};
    r.N = 1000;
    r.P = 200;
    r.chunk = 64;
    r.nchunk = 16;
    r.xs = d4;
    r.samp = d4;
    r.part = d2;
    r.rho = d2;
    r.gk = d2;
    r.eF = d;
    r.tab = d2;
    b = n;
    b.nrho = 8;
    b.red = r;
    b.red.mixed = 1;
    refused(launch_near(b, nullptr), "structure-factor partials of another precision than the near field");
    b.red = r;
    refused(launch_near(b, nullptr), "fewer structure-factor workgroups than the partials need");
    RhoArgs q = r;
    q.chunk = 512;
    q.nchunk = 2;
    refused(launch_rho_partial(q, nullptr), "groups larger than the largest group");
    q = r;
    q.P = 1;
    q.chunk = 256;
    q.nchunk = 4;
    refused(launch_rho_partial(q, nullptr), "staged groups beyond the staging area");
    q = r;
    q.nchunk = 15;
    refused(launch_rho_partial(q, nullptr), "groups that do not cover every particle");
    q = r;
    q.tab = nullptr;
    refused(launch_rho_partial(q, nullptr), "FP64 phases without the rotation table");
    q = r;
    q.samp = nullptr;
    refused(launch_rho_reduce(q, nullptr), "reduction without modes");
    // far field, drift, sampling, state copies, energies
    FarArgs f{};
    f.N = 10;
    f.P = 8;
    f.xs = d4;
    f.order = ip;
    f.samp = d4;
    f.gk = d2;
    f.fnear = d;
    f.f = d;
    f.flag = ip;
    f.tab = d2;
    f.drift = 1;
    refused(launch_far(f, nullptr), "fused drift without its buffers");
    f.drift = 0;
    f.vs = d;
    refused(launch_far(f, nullptr), "second half-kick without masses");
    KickDriftArgs k{};
    k.N = 10;
    k.xs = d4;
    k.vs = d;
    k.fs = d;
    k.ms = d;
    k.xb = d;
    k.flag = ip;
    refused(launch_kick_drift(k, nullptr), "drift without the rebuild gate");
    SampleArgs sa{};
    sa.P = 8;
    sa.nstep = 2;
    sa.nshell = 3;
    sa.cdf = d;
    sa.coef = d;
    sa.first = ip;
    sa.size = ip;
    sa.lattice = ip;
    sa.samp = d4;
    sa.n_out = ip;
    refused(launch_sample(sa, nullptr), "mode output of more than one step");
    PermArgs pa{};
    pa.N = 10;
    pa.x = d;
    pa.q = d;
    pa.m = d;
    pa.xs = d4;
    pa.ms = d;
    refused(launch_state_in(pa, nullptr), "state copy without the cell order");
    pa.order = ip;
    pa.v = d;
    refused(launch_state_in(pa, nullptr), "velocities to copy without their cell-order rows");
    EnergyArgs ea{};
    ea.epart = d;
    ea.eF = d;
    refused(launch_energy(ea, nullptr), "energies without an output row");
    refused(launch_iota(nullptr, 10, nullptr), "cell order without its array");
}

int main()
{
    const double n = 3.0 / (4.0 * 3.141592653589793);   // number density of the workloads
    struct Sys {
        int64_t N;
        double lambda, rc;
    } sys[] = {{1, 1.0, 0.5},      {150, 0.5, 2.5},   {600, 1.0, 3.0},     {1000, 1.0, 3.0},
               {2600, 2.0, 4.0},   {5000, 2.0, 4.0},  {100000, 2.0, 4.0},  {200000, 2.0, 4.0},
               {1000000, 10.0, 5.0}, {500, 10.0, 4.0}, {50000, 0.5, 4.0}};
    const int Ps[] = {1, 7, 64, 200, 300, 500, 1500, 4096};
    const double skins[] = {-1.0, 0.0, 0.3, 1.5, 100.0};
    int cases = 0;
    for (const Sys &y : sys) {
        const double L0 = std::cbrt((double)y.N / n);
        // the workload's box, and the smallest box the checks admit (three cells)
        // and cuboids: elongated along one axis, and with one edge at three cells
        const double Ls[][3] = {{L0, L0, L0},
                                {3.0 * y.rc, 3.0 * y.rc, 3.0 * y.rc},
                                {3.0 * y.rc * (1.0 + 1e-12), 3.0 * y.rc * (1.0 + 1e-12), 3.0 * y.rc * (1.0 + 1e-12)},
                                {L0, 1.3 * L0, 0.8 * L0},
                                {3.0 * y.rc, 2.0 * L0, L0}};
        for (int k = 0; k < 5; ++k)
            for (int P : Ps)
                for (double sk : skins) {
                    // a cuboid's lattice is enumerated point by point: fewer combinations
                    if (k >= 3 && ((P != 7 && P != 500) || (sk != -1.0 && sk != 0.0))) continue;
                    audit(y.N, Ls[k], y.lambda, y.rc, P, sk);
                    ++cases;
                }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (ndev == 0) {
        guards();
        std::printf("launch guards checked\n");
    } else {
        std::printf("launch guards not checked: a GPU is visible\n");
    }
    std::printf("audited %d parameter sets, %d failures\n", cases, failures);
    return failures ? 1 : 0;
}

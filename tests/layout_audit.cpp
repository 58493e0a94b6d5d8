// Host-only audit of the workspace plan (no GPU needed): for a sweep of
// system parameters, every buffer the kernels index holds the largest index
// their launch shapes can reach, on every cell grid a system can use (the
// coarse grid of rbsog_build_cells, the fine grid of the force evaluation, and
// the finer grid a hot system's default skin drops to), and the fine grids'
// 5 x 5 x 5 stencil covers the list radius.  Prints one line per failure and
// exits non-zero if any.
#include <cmath>
#include <cstdio>
#include <vector>

#include "system.h"

using namespace rbsog;

namespace rbsog {
int near_capacity(int64_t N, double L, double rl, int nf);
}

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

static void audit(int64_t N, double L, double lambda, double rc, int P, double skin)
{
    rbsog_sog s{};
    if (rbsog_sog_init(lambda, rc, 1e-4, RBSOG_AUTO, RBSOG_AUTO, &s) != RBSOG_OK) {
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
    if (check_params(&p, &s) != RBSOG_OK) return;   // refused before any launch
    const Derived d = derive(&p, &s);
    const Layout w = make_layout(N, d, P, false);
    char tag[160];
    std::snprintf(tag, sizeof tag, "N %lld L %.4g lambda %g r_c %g P %d skin %g", (long long)N, L, lambda, rc, P,
                  skin);
    // cell grids the kernels can index: coarse, fine, fine of a dropped skin
    const int grids[3] = {d.nc, d.nf, d.nf_tight};
    for (int g : grids) {
        const size_t ncell = (size_t)g * g * g;
        CHECK(span(w.count, w.cell_start) >= 4 * ncell, "%s grid %d: counts", tag, g);
        CHECK(span(w.cell_start, w.fill) >= 4 * (ncell + 1), "%s grid %d: cell starts", tag, g);
        CHECK(span(w.fill, w.tmp) >= 4 * ncell, "%s grid %d: fill", tag, g);
        CHECK(span(w.tile_sum, w.xb) >= 4 * (size_t)scan_tiles((int)ncell), "%s grid %d: scan tiles", tag, g);
    }
    // the 5-cell stencil of each fine grid reaches the list radius; at least 6 cells
    CHECK(d.nf >= 6 && d.nf_tight >= 6, "%s: fine grid below 6 cells", tag);
    CHECK(d.rl <= 2.0 * L / d.nf * (1 + 1e-15), "%s: list radius %g beyond the stencil of %d cells", tag, d.rl, d.nf);
    CHECK(rc <= 2.0 * L / d.nf_tight * (1 + 1e-15), "%s: r_c beyond the stencil of the tight grid", tag);
    CHECK(d.nf_tight >= d.nf, "%s: the tight grid is coarser", tag);
    // neighbour lists: list_rows(kp) entries per particle of the padded tiles, for
    // both list radii (the capacity only shrinks when the skin drops)
    const int kp_tight = near_capacity(N, L, rc, d.nf_tight);
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
    CHECK(span(w.epart, w.kepart) >= 8 * (size_t)near_blocks((int)N), "%s: near energy partials", tag);
    CHECK(span(w.kepart, w.flag) >= 8 * (size_t)far_blocks((int)N), "%s: kinetic partials", tag);
    CHECK(span(w.xs, w.xs_old) >= 32 * (size_t)N && span(w.ms, w.ms_old) >= 8 * (size_t)N, "%s: rows", tag);
    CHECK(w.total >= w.tab + 16 * kPhaseTable, "%s: total", tag);
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
        const double Ls[] = {L0, 3.0 * y.rc, 3.0 * y.rc * (1.0 + 1e-12)};
        for (double L : Ls)
            for (int P : Ps)
                for (double sk : skins) {
                    audit(y.N, L, y.lambda, y.rc, P, sk);
                    ++cases;
                }
    }
    std::printf("audited %d parameter sets, %d failures\n", cases, failures);
    return failures ? 1 : 0;
}

// C-ABI of librbsog (declared in include/rbsog.h): parameter checks, workspace
// layout, table upload and the per-evaluation launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "system.h"

namespace rbsog {

static_assert(kPhaseTable == kPhaseTab, "host and device rotation tables differ in size");
static_assert(kFarTable == kFarTab, "host and device far-field tables differ in size");

namespace {
thread_local std::string g_error;
}  // namespace

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }


// groups of the structure-factor partial buffer: an upper bound on those of any launch (rho_chunk <= rho_chunk_shared)
int nchunks(int64_t N, int P) { return (int)((N + rho_chunk((int)N, P) - 1) / rho_chunk((int)N, P)); }

CellGeom make_geom(const double Lb[3], const int nc[3])
{
    CellGeom g{};
    for (int d = 0; d < 3; ++d) {
        g.nc[d] = nc[d];
        g.L[d] = Lb[d];
        g.inv_cell[d] = (double)nc[d] / Lb[d];
    }
    g.ncell = nc[0] * nc[1] * nc[2];
    return g;
}

void box_edges(const rbsog_params *p, double Lb[3])
{
    Lb[0] = p->L;
    Lb[1] = p->Ly > 0.0 ? p->Ly : p->L;
    Lb[2] = p->Lz > 0.0 ? p->Lz : p->L;
}


// kp, a fifth of a particle's list capacity (the list holds list_rows(kp), 5 kp
// rounded up to whole blocks):
// 1.5x the expected number of neighbours within the list radius divided by
// five, plus 16; a particle with more neighbours walks its cells directly
// instead, so this only sizes the fast path.  RBSOG_NEAR_CAPACITY overrides it
// (a tuning knob).
int near_capacity(int64_t N, double V, double rl)
{
    if (const char *e = std::getenv("RBSOG_NEAR_CAPACITY")) {
        int v = std::atoi(e);
        if (v >= 1 && v <= 4096) return v;
    }
    double n = (double)N / V;
    double expected = n * (4.0 / 3.0) * kPi * rl * rl * rl / 5.0;
    return std::min(4096, std::max(8, (int)std::ceil(1.5 * expected + 16.0)));
}

// Cells per axis of the fine grid for lists of radius rl: width >= rl / 2, at least 6.
static int fine_cells(double L, double rl) { return std::max(6, (int)std::floor(2.0 * L / rl)); }

Derived derive(const rbsog_params *p, const rbsog_sog *s)
{
    Derived d{};
    // default skin 0.125 r_c (the fastest of 0.05..0.33 r_c on the N = 1e5 plasma);
    // never so large that the fine grid drops below 6 cells
    box_edges(p, d.Lb);
    d.cuboid = !(d.Lb[0] == d.Lb[1] && d.Lb[1] == d.Lb[2]);
    const double Lmin = std::min(d.Lb[0], std::min(d.Lb[1], d.Lb[2]));
    double skin = p->skin < 0.0 ? 0.125 * s->r_c : p->skin;
    skin = std::max(0.0, std::min(skin, Lmin / 3.0 - s->r_c));
    d.rl = s->r_c + skin;
    for (int a = 0; a < 3; ++a) {
        d.nc[a] = (int)std::floor(d.Lb[a] / s->r_c);
        d.nf[a] = fine_cells(d.Lb[a], s->r_c + skin);
        d.nf_tight[a] = fine_cells(d.Lb[a], s->r_c);
        // the 5-cell stencil reaches 2 w = 2 L / nf: keep the list radius within it
        d.rl = std::min(d.rl, 2.0 * d.Lb[a] / (double)d.nf[a]);
    }
    d.skin = std::max(0.0, d.rl - s->r_c);
    if (d.cuboid) {
        d.mmax = 0;
        d.nlat = box_lattice_points(*s, d.Lb);
        d.nshells = d.nlat;
    } else {
        d.mmax = p->mmax > 0 ? p->mmax : default_mmax(*s, p->L);
        d.nlat = lattice_points(d.mmax);
        d.nshells = d.mmax;
    }
    d.kp = near_capacity(p->N, d.Lb[0] * d.Lb[1] * d.Lb[2], d.rl);
    d.sbatch = std::max(1, std::min(64, 16384 / std::max(1, p->P)));
    d.full_k = p->full_k ? 1 : 0;
    d.nmodes = d.full_k ? d.nlat : (int64_t)p->P;
    if (d.full_k) d.sbatch = 1;
    return d;
}

Layout make_layout(int64_t N, const Derived &d, int P, bool shared_lattice)
{
    // any grid: the coarse one, the fine one, and the fine one of a dropped skin
    int ncell = std::max(std::max(d.nf[0] * d.nf[1] * d.nf[2], d.nf_tight[0] * d.nf_tight[1] * d.nf_tight[2]),
                         d.nc[0] * d.nc[1] * d.nc[2]);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.lattice = take(shared_lattice ? 0 : sizeof(int32_t) * (size_t)d.nlat);
    L.cdf = take(sizeof(double) * (size_t)d.nshells);
    L.coef = take(sizeof(double) * (size_t)d.nshells);
    L.first = take(sizeof(int32_t) * (size_t)d.nshells);
    L.size = take(sizeof(int32_t) * (size_t)d.nshells);
    L.cell_id = take(sizeof(int32_t) * (size_t)N);
    L.count = take(sizeof(int32_t) * (size_t)ncell);
    L.cell_start = take(sizeof(int32_t) * ((size_t)ncell + 1));
    L.fill = take(sizeof(int32_t) * (size_t)ncell);
    L.tmp = take(sizeof(int32_t) * (size_t)N);
    L.order = take(sizeof(int32_t) * (size_t)N);
    L.order_old = take(sizeof(int32_t) * (size_t)N);
    L.xs = take(sizeof(double) * 4 * (size_t)N);
    L.xs_old = take(sizeof(double) * 4 * (size_t)N);
    L.tile_sum = take(sizeof(int32_t) * (size_t)scan_tiles(ncell));
    L.xb = take(sizeof(double) * 3 * (size_t)N);
    L.vs = take(sizeof(double) * 3 * (size_t)N);
    L.vs_old = take(sizeof(double) * 3 * (size_t)N);
    L.fs = take(sizeof(double) * 3 * (size_t)N);
    L.ms = take(sizeof(double) * (size_t)N);
    L.ms_old = take(sizeof(double) * (size_t)N);
    const size_t nm = (size_t)d.nmodes;
    L.samp = take(sizeof(double) * 4 * (d.full_k ? nm : (size_t)P * (size_t)d.sbatch));
    L.part = take(d.full_k ? 0 : sizeof(double) * 2 * (size_t)nchunks(N, P) * (size_t)P);
    L.rho = take(sizeof(double) * 2 * nm);
    L.gk = take(sizeof(double) * 2 * nm);
    L.eF = take(sizeof(double) * nm);
    L.eW = take(sizeof(double) * nm);
    L.vm = take(sizeof(double) * ((size_t)d.mmax + 1));
    L.fnear = take(sizeof(double) * 3 * kNearLanes * (size_t)N);
    L.epart = take(sizeof(double) * 2 * (size_t)near_blocks((int)N));
    L.kepart = take(sizeof(double) * (size_t)far_blocks((int)N));
    L.flag = take(sizeof(int32_t) * 8);
    L.energy = take(sizeof(double) * 8);
    L.nbr = take(sizeof(int32_t) * (size_t)list_rows(d.kp) * (size_t)list_padded(N));
    L.nbr_cnt = take(sizeof(int32_t) * (size_t)N);
    L.tab = take(sizeof(double) * 2 * kPhaseTable);
    L.tab_far = take(sizeof(double) * 2 * kFarTable);
    L.cdf_q = take(sizeof(double) * (size_t)d.nshells);
    L.mh = take(sizeof(int32_t) * 2);
    L.bath = take(sizeof(double) * kBathWords);
    L.fab = take(sizeof(double) * 2 * kMaxGauss);
    L.total = off;
    return L;
}

int check_params(const rbsog_params *p, const rbsog_sog *s)
{
    if (!p || !s) return fail(RBSOG_EINVAL, "null params or sog");
    if (p->N < 1 || p->N > ((int64_t)1 << 27) - 1) return fail(RBSOG_EINVAL, "N must lie in [1, 2^27 - 1]");
    if (!(p->L > 0.0) || !std::isfinite(p->L)) return fail(RBSOG_EINVAL, "L must be positive and finite");
    if (!(p->kT > 0.0) || !std::isfinite(p->kT)) return fail(RBSOG_EINVAL, "kT must be positive and finite");
    if (p->P < 1 || p->P > 4096) return fail(RBSOG_EINVAL, "P must lie in [1, 4096]");
    if (p->full_k != 0 && p->full_k != 1) return fail(RBSOG_EINVAL, "full_k must be 0 or 1");
    if (p->sampler != RBSOG_SAMPLER_IID && p->sampler != RBSOG_SAMPLER_MH)
        return fail(RBSOG_EINVAL, "sampler must be RBSOG_SAMPLER_IID or RBSOG_SAMPLER_MH");
    if (p->precision != RBSOG_FP64 && p->precision != RBSOG_MIXED) return fail(RBSOG_EINVAL, "unknown precision");
    if (p->density < RBSOG_ADAPTIVE || p->density > RBSOG_DH4PI) return fail(RBSOG_EINVAL, "unknown density");
    if (p->mmax < 0 || p->mmax > kMaxLatticeM) return fail(RBSOG_EINVAL, "mmax must lie in [0, %d]", kMaxLatticeM);
    if (!std::isfinite(p->skin)) return fail(RBSOG_EINVAL, "skin must be finite");
    if (s->nyuk < 0 || s->nyuk > 2) return fail(RBSOG_EINVAL, "sog: nyuk must be 0, 1 or 2");
    if (s->n < 1 || s->n > RBSOG_MAX_GAUSS || (s->nyuk != 2 && s->n != s->M1 + s->M2 + 1))
        return fail(RBSOG_EINVAL, "sog: inconsistent number of Gaussians");
    if (!(s->r_c > 0.0) || !(s->lambda > 0.0)) return fail(RBSOG_EINVAL, "sog: lambda and r_c must be positive");
    if (s->nyuk == 2)
        for (int t = 0; t < 2; ++t)
            if (!(s->yl[t] > 0.0) || !std::isfinite(s->yl[t]) || !std::isfinite(s->ya[t]))
                return fail(RBSOG_EINVAL, "sog: the kernel's terms need positive, finite lengths and finite weights");
    if (!(p->Ly >= 0.0) || !std::isfinite(p->Ly) || !(p->Lz >= 0.0) || !std::isfinite(p->Lz))
        return fail(RBSOG_EINVAL, "Ly and Lz must be finite and >= 0 (0: equal to L)");
    double Lb[3];
    box_edges(p, Lb);
    double nfp = 1.0;
    for (int a = 0; a < 3; ++a) {
        double nc = std::floor(Lb[a] / s->r_c);
        if (nc < 3.0) return fail(RBSOG_EINVAL, "box too small: floor(L_%c / r_c) = %g < 3", "xyz"[a], nc);
        nfp *= std::floor(2.0 * Lb[a] / s->r_c);
    }
    if (nfp > (double)(1 << 26)) return fail(RBSOG_EINVAL, "too many cells (L / r_c too large)");
    const bool cuboid = !(Lb[0] == Lb[1] && Lb[1] == Lb[2]);
    if (cuboid) {
        if (p->mmax != 0) return fail(RBSOG_EINVAL, "a cuboid box takes the default lattice (mmax = 0)");
        if (p->sampler != RBSOG_SAMPLER_IID) return fail(RBSOG_EINVAL, "a cuboid box draws i.i.d. modes only");
        if (box_lattice_points(*s, Lb) < 1)
            return fail(RBSOG_EINVAL, "the cuboid's lattice is empty or exceeds |n_d| = 511");
    }
    return RBSOG_OK;
}



int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

}  // namespace rbsog

using namespace rbsog;

namespace rbsog {

enum KernelClass { kCells = 0, kKickDrift, kSample, kRhoPartial, kRhoReduce, kNear, kFar, kEnergy, kNlist };
constexpr int kTimingEvents = 4096;

// Turns recorded event pairs into accumulated milliseconds (synchronises).
hipError_t harvest(rbsog_handle *h)
{
    if (h->records.empty()) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) return e;
    for (auto &r : h->records) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, h->events[r.second], h->events[r.second + 1]);
        if (e != hipSuccess) return e;
        h->timing_ms[r.first] += ms;
        h->launches[r.first] += 1;
    }
    h->records.clear();
    h->used = 0;
    return hipSuccess;
}


CellArgs cell_args(rbsog_handle *h, const CellGeom &g, const int32_t *gate, bool carry_v)
{
    CellArgs a{};
    a.N = (int)h->p.N;
    a.g = g;
    a.xs = h->xs;
    a.order = h->order;
    a.vs = carry_v ? h->vs : nullptr;
    a.xs_old = h->xs_old;
    a.order_old = h->order_old;
    a.vs_old = h->vs_old;
    a.ms = h->ms;
    a.ms_old = h->ms_old;
    a.xb = h->xb;
    a.cell_id = h->cell_id;
    a.count = h->count;
    a.cell_start = h->cell_start;
    a.fill = h->fill;
    a.tmp = h->tmp;
    a.tile_sum = h->tile_sum;
    a.ticket = h->ticket;
    a.gate = gate;
    return a;
}

PermArgs perm_args(rbsog_handle *h, double *x, double *v, double *f)
{
    PermArgs a{};
    a.N = (int)h->p.N;
    a.order = h->order;
    a.x = x;
    a.v = v;
    a.f = f;
    a.q = h->q;
    a.m = h->m;
    a.xs = h->xs;
    a.vs = h->vs;
    a.fs = h->fs;
    a.ms = h->ms;
    return a;
}

NearArgs near_args(rbsog_handle *h, const int32_t *gate, bool energy)
{
    NearArgs na{};
    na.N = (int)h->p.N;
    na.g = h->gf;
    for (int d = 0; d < 3; ++d) {
        na.w[d] = h->d.Lb[d] / (double)h->gf.nc[d];
        na.inv_L[d] = 1.0 / h->d.Lb[d];
    }
    na.margin = 1e-9 * std::max(h->d.Lb[0], std::max(h->d.Lb[1], h->d.Lb[2]));
    na.e2 = make_exp2_poly();
    na.nbr = h->nbr;
    na.nbr_cnt = h->nbr_cnt;
    na.kp = h->d.kp;
    na.rc2 = h->sog.r_c * h->sog.r_c;
    na.rl2 = h->d.rl * h->d.rl;
    na.gate = gate;
    na.sog = h->sd;
    na.xs = h->xs;
    na.cell_start = h->cell_start;
    na.fnear = h->fnear;
    na.epart = h->epart;
    na.mixed = h->p.precision == RBSOG_MIXED;
    na.energy = energy;
    return na;
}

SampleArgs sample_args(rbsog_handle *h, uint64_t step, int nstep)
{
    SampleArgs a{};
    a.P = h->p.P;
    a.nstep = nstep;
    a.step = step;
    a.seed = h->p.seed;
    a.replica = h->p.replica;
    a.nshell = h->nshell;
    a.S = h->S;
    a.cdf = h->cdf;
    a.coef = h->coef;
    a.first = h->first;
    a.size = h->size;
    a.lattice = h->lattice;
    a.samp = h->samp;
    if (h->p.sampler == RBSOG_SAMPLER_MH) {
        a.cdf_q = h->cdf_q;
        a.Sq = h->Sq;
        a.mh = h->mh;
    }
    return a;
}

RhoArgs rho_args(rbsog_handle *h, const double4 *samp)
{
    RhoArgs a{};
    a.N = (int)h->p.N;
    a.P = (int)h->d.nmodes;
    // the group size of the single-system step (partials in the near launch);
    // the ensemble's partial launch uses the same, so that a replica sums in
    // the same order as the system alone.  nchunks() (the buffer) bounds it.
    a.chunk = rho_chunk_shared((int)h->p.N, h->p.P, h->p.precision == RBSOG_MIXED);
    a.nchunk = (int)((h->p.N + a.chunk - 1) / a.chunk);
    for (int d = 0; d < 3; ++d) a.inv_L[d] = 1.0 / h->d.Lb[d];
    a.xs = h->xs;
    a.samp = samp;
    a.part = h->part;
    a.rho = h->rho;
    a.gk = h->gk;
    a.eF = h->eF;
    a.eW = h->eW;
    if (h->d.cuboid) {   // virial factors from the Fourier coefficients, mode by mode
        a.vm = nullptr;
        a.nG = h->sog.n;
        a.fa = h->fab;
        a.fb = h->fab + kMaxGauss;
    } else {
        a.vm = h->vm;
    }
    a.mixed = h->p.precision == RBSOG_MIXED;
    a.tab = h->tab;
    a.ss = make_sincos_short();
    a.tab_fine = h->tab_far;
    a.sf = make_sincos_far();
    return a;
}

// Cell order + neighbour lists of the fine grid for the rows in xs: always
// (gate == null, a single evaluation) or only when the device gate is raised
// (the step path, where the drift has already moved the rows).
int prepare(rbsog_handle *h, const int32_t *gate, bool carry_v)
{
    CellArgs ca = cell_args(h, h->gf, gate, carry_v);
    HIPCHECK(timed(h, kCells, [&] { return launch_cell_build(ca, h->st); }));
    NearArgs na = near_args(h, gate, false);
    HIPCHECK(timed(h, kNlist, [&] { return launch_nlist(na, h->st); }));
    h->lists_valid = true;
    return RBSOG_OK;
}

// The modes of `step` in samp: drawn for `ahead` steps from it unless an
// earlier draw already holds them.
int modes(rbsog_handle *h, uint64_t step, int ahead, const double4 **samp)
{
    if (h->d.full_k) {   // every lattice mode, uploaded at creation
        *samp = h->samp;
        return RBSOG_OK;
    }
    if (!(h->samp_n > 0 && step >= h->samp_step && step - h->samp_step < (uint64_t)h->samp_n)) {
        int n = std::max(1, std::min(ahead, h->d.sbatch));
        SampleArgs sa = sample_args(h, step, n);
        HIPCHECK(timed(h, kSample, [&] { return launch_sample(sa, h->st); }));
        h->samp_step = step;
        h->samp_n = n;
    }
    *samp = h->samp + (size_t)(step - h->samp_step) * (size_t)h->p.P;
    return RBSOG_OK;
}

FarArgs far_args(rbsog_handle *h, const double4 *samp, double *f, double *f_near, bool kick, double dt)
{
    FarArgs fa{};
    fa.N = (int)h->p.N;
    fa.P = (int)h->d.nmodes;
    for (int d = 0; d < 3; ++d) {
        fa.two_pi_over_L[d] = (2.0 * kPi) / h->d.Lb[d];
        fa.inv_L[d] = 1.0 / h->d.Lb[d];
    }
    fa.xs = h->xs;
    fa.order = h->order;
    fa.samp = samp;
    fa.gk = h->gk;
    fa.fnear = h->fnear;
    fa.f = f;
    fa.f_near_out = f_near;
    fa.fs = kick ? h->fs : nullptr;
    fa.vs = kick ? h->vs : nullptr;
    fa.ms = h->ms;
    fa.half_dt = 0.5 * dt;
    fa.kepart = kick ? h->kepart : nullptr;
    fa.flag = h->flag;
    fa.mixed = h->p.precision == RBSOG_MIXED;
    fa.tab = h->tab_far;
    fa.ss = make_sincos_far();
    return fa;
}

EnergyArgs energy_args(rbsog_handle *h, double *out, bool kick)
{
    EnergyArgs ea{};
    ea.nnear = near_blocks((int)h->p.N);
    ea.nfar = far_blocks((int)h->p.N);
    ea.P = (int)h->d.nmodes;
    ea.epart = h->epart;
    ea.kepart = kick ? h->kepart : nullptr;
    ea.eF = h->eF;
    ea.eW = h->eW;
    ea.Uk0 = h->Uk0;
    ea.Uself = h->Uself;
    ea.Ubg = h->Ubg;
    ea.out = out;
    return ea;
}

// Structure factors, near field, far field (+ optional kick) and the energy
// sums of one evaluation whose cell order, lists and modes are prepared.
Thermo thermo(const rbsog_handle *h, double dt, uint64_t step)
{
    Thermo t{};
    if (h->friction > 0.0) {
        t.on = 1;
        t.c1 = std::exp(-h->friction * dt);
        t.c2kT = (1.0 - t.c1 * t.c1) * h->bath_kT;
        t.seed = h->p.seed;
        t.replica = h->p.replica;
        t.step = step;
    }
    return t;
}

BathArgs bath_args(const rbsog_handle *h, double dt, int mode)
{
    BathArgs b{};
    b.kind = h->bath_kind;
    b.mode = mode;
    b.dt = dt;
    b.gkT = 3.0 * (double)h->p.N * h->bath_kT;
    b.rate = h->bath_rate;
    b.Q = b.gkT / (h->bath_rate * h->bath_rate);
    b.nfar = far_blocks((int)h->p.N);
    b.kepart = h->kepart;
    b.bath = h->bath;
    return b;
}

int evaluate(rbsog_handle *h, const double4 *samp, double *f, double *f_near, bool kick, double dt, double *energy,
             int32_t *gate_raise, int32_t *gate_clear, uint64_t next_step, int bath_mode)
{
    RhoArgs ra = rho_args(h, samp);
    NearArgs na = near_args(h, nullptr, energy != nullptr);
    if (h->d.full_k) {
        HIPCHECK(timed(h, kRhoPartial, [&] { return launch_rho_full(ra, h->st); }));
    } else {
        // the partial sums run in the near kernel's first workgroups
        na.red = ra;
        na.nrho = (int)((rho_blocks(ra.nchunk, ra.P) + 7) / 8 * 8);
        // Spread through a launch of several rounds of workgroups, the partial
        // sums fill the issue slots the near field's gathers leave (near launches
        // of the plasmas: N = 2e5, 4 178 workgroups, 115 -> 108 us; N = 6e5,
        // 536 -> 450 us; N = 1e6, 19 350 workgroups, 0.91 -> 0.74 ms).  A launch
        // the chip holds at once gains nothing from that and runs best with the
        // longer partial-sum workgroups dispatched first (N = 1e5: 1 789
        // workgroups, 49.5 us first, 53.6 us spread).
        na.interleave = (int64_t)na.nrho + near_blocks((int)h->p.N) >= kInterleaveBlocks;
        if (const char *e = std::getenv("RBSOG_NEAR_INTERLEAVE"))   // 0 / 1: a tuning knob
            na.interleave = std::atoi(e) != 0;
    }
    HIPCHECK(timed(h, kNear, [&] { return launch_near(na, h->st); }));
    if (!h->d.full_k) HIPCHECK(timed(h, kRhoReduce, [&] { return launch_rho_reduce(ra, h->st); }));
    FarArgs fa = far_args(h, samp, f, f_near, kick, dt);
    fa.gate_clear = gate_clear;
    fa.rebuilds = gate_clear ? h->rebuilds : nullptr;
    if (kick && gate_raise) {
        fa.drift = 1;
        fa.dt = dt;
        for (int d = 0; d < 3; ++d) fa.L[d] = h->d.Lb[d];
        fa.half_skin2 = 0.25 * h->d.skin * h->d.skin;
        fa.xb = h->xb;
        fa.xs_next = h->xs;
        fa.gate_raise = gate_raise;
        fa.th = thermo(h, dt, next_step);
    }
    HIPCHECK(timed(h, kFar, [&] { return launch_far(fa, h->st); }));
    // a global bath: the step's closing half-step (and the next one's opening)
    // on the kinetic energy the far kernel's half-kick left
    if (kick && bath_mode) HIPCHECK(timed(h, kKickDrift, [&] { return launch_bath(bath_args(h, dt, bath_mode), h->st); }));
    if (energy) {
        EnergyArgs ea = energy_args(h, energy, kick);
        if (kick && bath_mode) ea.ke_set = h->bath + 3;
        HIPCHECK(timed(h, kEnergy, [&] { return launch_energy(ea, h->st); }));
    }
    return RBSOG_OK;
}

}  // namespace rbsog

extern "C" const char *rbsog_last_error(void) { return g_error.c_str(); }

extern "C" int rbsog_workspace_size(const rbsog_params *p, const rbsog_sog *s, size_t *bytes)
{
    int rc = check_params(p, s);
    if (rc) return rc;
    if (!bytes) return fail(RBSOG_EINVAL, "bytes is null");
    *bytes = make_layout(p->N, derive(p, s), p->P, false).total;
    return RBSOG_OK;
}

extern "C" int rbsog_create(const rbsog_params *p, const rbsog_sog *s, const double *q_dev, const double *m_dev,
                            void *ws_dev, size_t ws_bytes, void *hip_stream, rbsog_handle **out)
{
    int rc = create_system(p, s, q_dev, m_dev, ws_dev, ws_bytes, (hipStream_t)hip_stream, nullptr, out);
    if (rc) return rc;
    // a system stepped by rbsog_step reads its rebuild count back (pinned host
    // word, an event) to decide whether a default skin pays
    rbsog_handle *h = *out;
    if (h->skin_default) {
        hipError_t e = hipHostMalloc((void **)&h->rb_host, sizeof(int32_t), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->rb_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            rbsog_destroy(h);
            *out = nullptr;
            return fail(RBSOG_EHIP, "rebuild counter: %s", hipGetErrorString(e));
        }
    }
    return RBSOG_OK;
}

namespace rbsog {

int create_system(const rbsog_params *p, const rbsog_sog *s, const double *q_dev, const double *m_dev, void *ws_dev,
                  size_t ws_bytes, hipStream_t stream, const int32_t *lattice_dev, rbsog_handle **out,
                  const double *q_host, const double *m_host, bool sync)
{
    int rc = check_params(p, s);
    if (rc) return rc;
    if (!q_dev || !m_dev || !out) return fail(RBSOG_EINVAL, "null q, m or out");
    if (!ws_dev || ((uintptr_t)ws_dev % kAlign)) return fail(RBSOG_EWORKSPACE, "workspace must be 256-byte aligned");
    rbsog_handle *h = new (std::nothrow) rbsog_handle{};
    if (!h) return fail(RBSOG_ENOMEM, "handle allocation");
    h->p = *p;
    h->sog = *s;
    h->q = q_dev;
    h->m = m_dev;
    h->st = stream;
    h->d = derive(p, s);
    h->g = make_geom(h->d.Lb, h->d.nc);
    h->gf = make_geom(h->d.Lb, h->d.nf);
    h->V = h->d.Lb[0] * h->d.Lb[1] * h->d.Lb[2];
    if (h->d.full_k && (lattice_dev || h->d.nlat > 0x7fffffff)) {
        delete h;
        return fail(RBSOG_EINVAL, "full_k needs a lattice of fewer than 2^31 points in the system's own workspace");
    }
    h->lay = make_layout(p->N, h->d, p->P, lattice_dev != nullptr);
    if (ws_bytes < h->lay.total) {
        size_t need = h->lay.total;
        delete h;
        return fail(RBSOG_EWORKSPACE, "workspace of %zu bytes is below the %zu needed", ws_bytes, need);
    }
    // sum q and sum q^2 in particle order (they enter the measure, eq. 3.22),
    // from the caller's host copies when given, else read back from the device
    std::vector<double> qh;
    hipError_t e = hipSuccess;
    if (!q_host || !m_host) {
        qh.resize((size_t)p->N);
        e = hipMemcpyAsync(qh.data(), q_dev, sizeof(double) * (size_t)p->N, hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) {
            delete h;
            return fail(RBSOG_EHIP, "reading q: %s", hipGetErrorString(e));
        }
    }
    double q1 = 0.0, q2 = 0.0;
    charge_sums(q_host ? q_host : qh.data(), p->N, &q1, &q2);
    if (!q_host || !m_host) {
        e = hipMemcpyAsync(qh.data(), m_dev, sizeof(double) * (size_t)p->N, hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) {
            delete h;
            return fail(RBSOG_EHIP, "reading m: %s", hipGetErrorString(e));
        }
    }
    h->m_min = (q_host && m_host) ? *std::min_element(m_host, m_host + p->N) : *std::min_element(qh.begin(), qh.end());
    h->skin_default = p->skin < 0.0;   // only the default skin adapts
    h->dt_checked = 0.0;
    h->rb_host = nullptr;
    h->rb_ev = nullptr;
    h->rb_pending = false;
    h->rb_steps = h->steps_done = 0;
    h->Q1 = q1;
    h->Q2 = q2;
    if (!(q2 > 0.0)) {
        delete h;
        return fail(RBSOG_EINVAL, "all charges are zero");
    }
    Tables t;
    build_tables(*s, *p, q2, h->d.mmax, &t, lattice_dev == nullptr);
    h->nshell = t.nshell;
    h->S = t.S;
    h->ws = (char *)ws_dev;
    char *w = h->ws;
    const Layout &L = h->lay;
    h->lattice = lattice_dev ? (int32_t *)lattice_dev : (int32_t *)(w + L.lattice);
    h->cdf = (double *)(w + L.cdf);
    h->coef = (double *)(w + L.coef);
    h->first = (int32_t *)(w + L.first);
    h->size = (int32_t *)(w + L.size);
    h->cell_id = (int32_t *)(w + L.cell_id);
    h->count = (int32_t *)(w + L.count);
    h->cell_start = (int32_t *)(w + L.cell_start);
    h->fill = (int32_t *)(w + L.fill);
    h->tmp = (int32_t *)(w + L.tmp);
    h->order = (int32_t *)(w + L.order);
    h->order_old = (int32_t *)(w + L.order_old);
    h->xs = (double4 *)(w + L.xs);
    h->xs_old = (double4 *)(w + L.xs_old);
    h->tile_sum = (int32_t *)(w + L.tile_sum);
    h->xb = (double *)(w + L.xb);
    h->vs = (double *)(w + L.vs);
    h->vs_old = (double *)(w + L.vs_old);
    h->fs = (double *)(w + L.fs);
    h->ms = (double *)(w + L.ms);
    h->ms_old = (double *)(w + L.ms_old);
    h->samp = (double4 *)(w + L.samp);
    h->part = (double2 *)(w + L.part);
    h->rho = (double2 *)(w + L.rho);
    h->gk = (double2 *)(w + L.gk);
    h->eF = (double *)(w + L.eF);
    h->eW = (double *)(w + L.eW);
    h->vm = (double *)(w + L.vm);
    h->fnear = (double *)(w + L.fnear);
    h->epart = (double *)(w + L.epart);
    h->kepart = (double *)(w + L.kepart);
    h->flag = (int32_t *)(w + L.flag);
    h->gate = h->flag + 1;
    h->ticket = h->flag + 3;
    h->rebuilds = h->flag + 4;
    h->phase = 0;
    h->samp_n = 0;
    h->energy = (double *)(w + L.energy);
    h->nbr = (int32_t *)(w + L.nbr);
    h->nbr_cnt = (int32_t *)(w + L.nbr_cnt);
    h->tab = (double2 *)(w + L.tab);
    h->tab_far = (double2 *)(w + L.tab_far);
    h->fab = (double *)(w + L.fab);
    h->cdf_q = (double *)(w + L.cdf_q);
    h->mh = (int32_t *)(w + L.mh);
    h->bath = (double *)(w + L.bath);
    double tabh[2 * kPhaseTable];
    phase_table(tabh);
    h->lists_valid = false;
    e = hipSuccess;
    if (!lattice_dev)
        e = hipMemcpyAsync(h->lattice, t.packed.data(), sizeof(int32_t) * t.packed.size(), hipMemcpyHostToDevice,
                           h->st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->cdf, t.cdf.data(), sizeof(double) * t.nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->coef, t.coef.data(), sizeof(double) * t.nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->first, t.shell_first.data(), sizeof(int32_t) * t.nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->size, t.shell_size.data(), sizeof(int32_t) * t.nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->tab, tabh, sizeof(tabh), hipMemcpyHostToDevice, h->st);
    std::vector<double> tabf(2 * (size_t)kFarTable);
    far_table(tabf.data());
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->tab_far, tabf.data(), sizeof(double) * tabf.size(), hipMemcpyHostToDevice, h->st);
    // Metropolis-Hastings draws: the proposal measure's CDF (F = 1) over the
    // same shells, and an empty chain
    std::vector<double> cdfq;
    const int32_t mh0[2] = {0, -1};
    if (e == hipSuccess && p->sampler == RBSOG_SAMPLER_MH && !h->d.full_k) {
        rbsog_params pq = *p;
        pq.density = RBSOG_FLAT;
        Tables tq;
        build_tables(*s, pq, q2, h->d.mmax, &tq, false);
        if (tq.nshell != t.nshell) e = hipErrorInvalidValue;   // both list the shells with r3(m) > 0
        cdfq = tq.cdf;
        h->Sq = tq.S;
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->cdf_q, cdfq.data(), sizeof(double) * cdfq.size(), hipMemcpyHostToDevice, h->st);
        if (e == hipSuccess) e = hipMemcpyAsync(h->mh, mh0, sizeof(mh0), hipMemcpyHostToDevice, h->st);
    }
    static const double bath0[kBathWords] = {};
    if (e == hipSuccess) e = hipMemcpyAsync(h->bath, bath0, sizeof(bath0), hipMemcpyHostToDevice, h->st);
    double fabh[2 * kMaxGauss] = {};
    for (int g = 0; g < s->n; ++g) {
        fabh[g] = s->A[g];
        fabh[kMaxGauss + g] = s->B[g];
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h->fab, fabh, sizeof(fabh), hipMemcpyHostToDevice, h->st);
    std::vector<double> vmh((size_t)h->d.mmax + 1);
    virial_table(*s, p->L, h->d.mmax, vmh.data());
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->vm, vmh.data(), sizeof(double) * vmh.size(), hipMemcpyHostToDevice, h->st);
    // full lattice: every n with its coefficient Fhat(k^2)/V, k = 2 pi n / L
    std::vector<double> full;
    if (e == hipSuccess && h->d.full_k) {
        const double V = h->V;
        full.resize(4 * (size_t)t.nlat);
        for (int64_t i = 0; i < t.nlat; ++i) {
            uint32_t pk = (uint32_t)t.packed[(size_t)i];
            int nx = (int)(pk & 1023u) - kLatticeBias, ny = (int)((pk >> 10) & 1023u) - kLatticeBias;
            int nz = (int)((pk >> 20) & 1023u) - kLatticeBias;
            full[4 * i] = nx;
            full[4 * i + 1] = ny;
            full[4 * i + 2] = nz;
            full[4 * i + 3] = fhat(*s, box_k2(h->d.Lb, nx, ny, nz)) / V;
        }
        e = hipMemcpyAsync(h->samp, full.data(), sizeof(double) * full.size(), hipMemcpyHostToDevice, h->st);
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->flag, 0, sizeof(int32_t) * 8, h->st);
    if (e == hipSuccess) e = hipMemsetAsync(h->count, 0, L.cell_start - L.count, h->st);
    if (e == hipSuccess) e = launch_iota(h->order, (int)p->N, h->st);   // a cell order before the first build
    // the uploads above are from host memory this function releases: pageable
    // copies are staged by the runtime before the calls return, so only the
    // single-system path's documented synchronisation remains
    if (e == hipSuccess && sync) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
        delete h;
        return fail(RBSOG_EHIP, "uploading tables: %s", hipGetErrorString(e));
    }
    // kernel-side SOG and the constant energies (Section 4.1)
    const double log2e = 1.4426950408889634;
    const KernelTerms kt = kernel_terms(*s);
    h->sd.n = s->n;
    h->sd.inv_lambda = 1.0 / kt.l[0];
    h->sd.inv_lambda_log2e = log2e / kt.l[0];
    h->sd.two = kt.n == 2 ? 1 : 0;
    h->sd.ya1 = kt.a[0];
    h->sd.ya2 = kt.a[1];
    h->sd.inv_lambda2 = 1.0 / kt.l[1];
    h->sd.inv_lambda2_log2e = log2e / kt.l[1];
    for (int j = 0; j < s->n; ++j) {
        h->sd.c[j] = s->c[j];
        h->sd.s_log2e[j] = s->s[j] * log2e;
        h->sd.cs2[j] = 2.0 * s->c[j] * s->s[j];
    }
    static_assert(kNearPolyDeg + 1 == sizeof(h->sd.hpoly) / sizeof(double), "near polynomial size");
    // the polynomial pair function serves the FP64 kernels only (mixed precision
    // evaluates the exponentials in FP32), so a mixed system skips the fit
    h->sd.poly = p->precision == RBSOG_FP64 ? near_poly(*s, s->r_c, h->sd.hpoly, h->sd.kpoly) : 0;
    h->sd.y_scale = 2.0 / s->r_c;
    if (const char *e = std::getenv("RBSOG_NEAR_POLY"))   // 0: evaluate the Gaussians one by one
        if (std::atoi(e) == 0) h->sd.poly = 0;
    h->Uk0 = s->Fhat0 * q1 * q1 / (2.0 * h->V);
    h->Uself = -0.5 * q2 * s->F0;
    // the kernel's integral over space, 4 pi sum_t a_t l_t^2 (4 pi lambda^2 for
    // both kernels; summed so that either is taken as given)
    double l2 = 0.0;
    for (int t = 0; t < kt.n; ++t) l2 += kt.a[t] * kt.l[t] * kt.l[t];
    h->Ubg = -(q1 * q1) * (4.0 * kPi * l2) / (2.0 * h->V);
    *out = h;
    return RBSOG_OK;
}

}  // namespace rbsog

extern "C" int rbsog_get_info(const rbsog_handle *h, rbsog_info *out)
{
    if (!h || !out) return fail(RBSOG_EINVAL, "null handle or out");
    out->N = h->p.N;
    out->nc = h->g.nc[0];
    out->mmax = h->d.mmax;
    out->nshell = h->nshell;
    out->nlat = h->d.nlat;
    out->S = h->S;
    out->Q1 = h->Q1;
    out->Q2 = h->Q2;
    out->ws_bytes = h->lay.total;
    out->skin = h->d.skin;
    out->nf = h->gf.nc[0];
    out->near_capacity = h->d.kp;
    out->near_poly = h->sd.poly;
    out->nc_y = h->g.nc[1];
    out->nc_z = h->g.nc[2];
    return RBSOG_OK;
}

extern "C" int rbsog_build_cells(rbsog_handle *h, const double *x_dev, int32_t *cell_start_dev, int32_t *order_dev)
{
    if (!h || !x_dev) return fail(RBSOG_EINVAL, "null handle or x");
    PermArgs in = perm_args(h, (double *)x_dev, nullptr, nullptr);   // state_in reads x only
    HIPCHECK(timed(h, kKickDrift, [&] { return launch_state_in(in, h->st); }));
    CellArgs a = cell_args(h, h->g, nullptr, false);
    HIPCHECK(timed(h, kCells, [&] { return launch_cell_build(a, h->st); }));
    h->lists_valid = false;  // the workspace now holds the coarse list
    if (cell_start_dev)
        HIPCHECK(hipMemcpyAsync(cell_start_dev, h->cell_start, sizeof(int32_t) * ((size_t)h->g.ncell + 1),
                                hipMemcpyDeviceToDevice, h->st));
    if (order_dev)
        HIPCHECK(hipMemcpyAsync(order_dev, h->order, sizeof(int32_t) * (size_t)h->p.N, hipMemcpyDeviceToDevice, h->st));
    return RBSOG_OK;
}

extern "C" int rbsog_sample_k(rbsog_handle *h, uint64_t step, int32_t *n_dev, double *coef_dev)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    if (h->d.full_k) return fail(RBSOG_EINVAL, "a full_k system samples no modes");
    SampleArgs a = sample_args(h, step, 1);
    a.n_out = n_dev;
    a.coef_out = coef_dev;
    HIPCHECK(timed(h, kSample, [&] { return launch_sample(a, h->st); }));
    h->samp_step = step;
    h->samp_n = 1;
    return RBSOG_OK;
}

extern "C" int rbsog_compute_rho(rbsog_handle *h, uint64_t step, const double *x_dev, double *rho_dev)
{
    if (!h || !x_dev || !rho_dev) return fail(RBSOG_EINVAL, "null handle, x or rho");
    if (h->d.full_k) return fail(RBSOG_EINVAL, "rbsog_compute_rho samples modes; not for a full_k system");
    const double4 *samp = nullptr;
    int rc = modes(h, step, 1, &samp);
    if (rc) return rc;
    RhoArgs a = rho_args(h, samp);
    // a launch of its own: the group size that fills the GPU by itself
    a.chunk = rho_chunk((int)h->p.N, h->p.P);
    a.nchunk = nchunks(h->p.N, h->p.P);
    a.xs = nullptr;
    a.x = x_dev;
    a.q = h->q;
    a.rho_out = rho_dev;
    HIPCHECK(timed(h, kRhoPartial, [&] { return launch_rho_partial(a, h->st); }));
    HIPCHECK(timed(h, kRhoReduce, [&] { return launch_rho_reduce(a, h->st); }));
    return RBSOG_OK;
}

extern "C" int rbsog_compute_forces(rbsog_handle *h, uint64_t step, const double *x_dev, double *f_dev,
                                    double *f_near_dev, double *energy_dev)
{
    if (!h || !x_dev || !f_dev) return fail(RBSOG_EINVAL, "null handle, x or f");
    PermArgs in = perm_args(h, (double *)x_dev, nullptr, nullptr);   // state_in reads x only
    HIPCHECK(timed(h, kKickDrift, [&] { return launch_state_in(in, h->st); }));
    int rc = prepare(h, nullptr, false);
    if (rc) return rc;
    const double4 *samp = nullptr;
    rc = modes(h, step, 1, &samp);
    if (rc) return rc;
    return evaluate(h, samp, f_dev, f_near_dev, false, 0.0, energy_dev);
}

namespace rbsog {

// The default skin pays off only when lists outlive several steps.  Once dt is
// known the fastest of the 3N Maxwell velocity components, ~sqrt(2 ln 3N kT /
// m_min), is compared with the skin: when it would cross skin/2 within two
// steps, lists of r_c alone rebuilt every step are cheaper.  The fine grid is
// then re-derived for the list radius r_c (more, smaller cells: the workspace
// is sized for that grid from the start) with a list capacity for r_c, and the
// next step rebuilds.  Results do not depend on the skin beyond the rounding
// of sums taken in another order.
static void drop_skin(rbsog_handle *h)
{
    h->d.skin = 0.0;
    h->d.rl = h->sog.r_c;
    for (int d = 0; d < 3; ++d) h->d.nf[d] = h->d.nf_tight[d];
    h->d.kp = std::min(h->d.kp, near_capacity(h->p.N, h->V, h->d.rl));
    h->gf = make_geom(h->d.Lb, h->d.nf);
    h->lists_valid = false;
}

bool adapt_skin(rbsog_handle *h, double dt)
{
    if (!h->skin_default || h->d.skin == 0.0 || !(dt > h->dt_checked) || !(h->m_min > 0.0)) return false;
    h->dt_checked = dt;
    const double kT = std::max(h->p.kT, h->bath_kT);   // a thermostat may hold the system hotter
    const double vmax = std::sqrt(2.0 * std::log(3.0 * (double)h->p.N + 1.0) * kT / h->m_min);
    if (!(0.5 * h->d.skin < 2.0 * vmax * dt)) return false;
    drop_skin(h);
    return true;
}

// The thermal estimate misses systems that run hotter than their kT (a
// random start relaxing into a strongly coupled state heats far above it):
// there the count of rebuilt steps decides.  After each rbsog_step the device
// count is copied to a pinned host word behind an event; the next call reads
// it if the copy has completed (never waiting) and drops the skin when more
// than half of at least ten steps rebuilt their lists.
bool adapt_skin_rebuilds(rbsog_handle *h)
{
    if (!h->rb_pending || !h->skin_default || h->d.skin == 0.0) return false;
    if (hipEventQuery(h->rb_ev) != hipSuccess) return false;   // not arrived yet (or an error: keep the skin)
    h->rb_pending = false;
    if (h->rb_steps < 10 || 2 * (int64_t)*h->rb_host <= h->rb_steps) return false;
    drop_skin(h);
    return true;
}

}  // namespace rbsog

extern "C" int rbsog_step(rbsog_handle *h, double *x_dev, double *v_dev, double *f_dev, uint64_t step0, int nsteps,
                          double dt, double *energy_hist_dev)
{
    if (!h || !x_dev || !v_dev || !f_dev) return fail(RBSOG_EINVAL, "null handle, x, v or f");
    if (nsteps < 0) return fail(RBSOG_EINVAL, "nsteps must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBSOG_EINVAL, "dt must be positive and finite");
    if (nsteps == 0) return RBSOG_OK;
    adapt_skin_rebuilds(h);
    adapt_skin(h, dt);
    // the state moves into cell order (the order of the last build) for the
    // steps and back into the caller's order at the end
    PermArgs io = perm_args(h, x_dev, v_dev, f_dev);
    HIPCHECK(timed(h, kKickDrift, [&] { return launch_state_in(io, h->st); }));
    const bool global = h->bath_kind == kBathNoseHoover || h->bath_kind == kBathBerendsen;
    // The first step's half-kick and drift run as their own kernel; those of
    // the later steps are fused into the far kernel of the step before.  Steps
    // alternate between two rebuild gates: the drift into step n raises gate n,
    // step n's builds read it, and step n's far kernel clears it.
    {
        int32_t *gate = h->gate + h->phase, *gate_next = h->gate + (1 - h->phase);
        // force a rebuild when the workspace holds no lists of the fine grid
        if (!h->lists_valid) HIPCHECK(launch_set_int(gate, 1, h->st));
        KickDriftArgs k{};
        k.N = (int)h->p.N;
        for (int d = 0; d < 3; ++d) {
            k.L[d] = h->d.Lb[d];
            k.inv_L[d] = 1.0 / h->d.Lb[d];
        }
        k.dt = dt;
        k.xs = h->xs;
        k.vs = h->vs;
        k.fs = h->fs;
        k.ms = h->ms;
        k.xb = h->xb;
        k.half_skin2 = 0.25 * h->d.skin * h->d.skin;
        k.gate = gate;
        k.gate_next = gate_next;
        k.flag = h->flag;
        k.th = thermo(h, dt, step0 + 1);
        k.order = h->order;
        if (global) {   // the first step's opening half-step of the bath
            HIPCHECK(timed(h, kKickDrift, [&] { return launch_ke_partials(k.N, h->vs, h->ms, h->kepart, h->st); }));
            HIPCHECK(timed(h, kKickDrift, [&] { return launch_bath(bath_args(h, dt, 1), h->st); }));
            k.vscale = h->bath + 2;
        }
        HIPCHECK(timed(h, kKickDrift, [&] { return launch_kick_drift(k, h->st); }));
    }
    for (int n = 0; n < nsteps; ++n) {
        int32_t *gate = h->gate + h->phase, *gate_next = h->gate + (1 - h->phase);
        int rc = prepare(h, gate, true);
        if (rc) return rc;
        const double4 *samp = nullptr;
        uint64_t step = step0 + (uint64_t)n + 1;
        rc = modes(h, step, nsteps - n, &samp);
        if (rc) return rc;
        double *e = energy_hist_dev ? energy_hist_dev + kEnergyCols * (size_t)n : nullptr;
        const bool last = n + 1 == nsteps;
        // a global bath keeps the next step's half-kick and drift out of the far
        // kernel: its velocity factor needs the whole system's kinetic energy
        rc = evaluate(h, samp, nullptr, nullptr, true, dt, e, (last || global) ? nullptr : gate_next, gate, step + 1,
                      global ? (last ? 2 : 3) : 0);
        if (rc) return rc;
        if (global && !last) {
            KickDriftArgs k{};
            k.N = (int)h->p.N;
            for (int d = 0; d < 3; ++d) {
                k.L[d] = h->d.Lb[d];
                k.inv_L[d] = 1.0 / h->d.Lb[d];
            }
            k.dt = dt;
            k.xs = h->xs;
            k.vs = h->vs;
            k.fs = h->fs;
            k.ms = h->ms;
            k.xb = h->xb;
            k.half_skin2 = 0.25 * h->d.skin * h->d.skin;
            k.gate = gate_next;
            k.flag = h->flag;
            k.vscale = h->bath + 2;
            HIPCHECK(timed(h, kKickDrift, [&] { return launch_kick_drift(k, h->st); }));
        }
        h->phase = 1 - h->phase;
    }
    if (global)   // the last step's closing half-step
        HIPCHECK(timed(h, kKickDrift, [&] { return launch_scale_v((int)h->p.N, h->vs, h->bath + 2, h->st); }));
    HIPCHECK(timed(h, kKickDrift, [&] { return launch_state_out(io, h->st); }));
    h->steps_done += nsteps;
    if (h->rb_host && h->skin_default && h->d.skin > 0.0) {
        HIPCHECK(hipMemcpyAsync(h->rb_host, h->rebuilds, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
        HIPCHECK(hipEventRecord(h->rb_ev, h->st));
        h->rb_pending = true;
        h->rb_steps = h->steps_done;
    }
    return RBSOG_OK;
}

extern "C" int rbsog_check(rbsog_handle *h)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    int32_t flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, h->flag, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
    HIPCHECK(hipStreamSynchronize(h->st));
    if (flag) {
        HIPCHECK(launch_set_int(h->flag, 0, h->st));
        HIPCHECK(hipStreamSynchronize(h->st));
        return fail(RBSOG_ENONFINITE, "non-finite force or over-long step detected");
    }
    return RBSOG_OK;
}

extern "C" int rbsog_timing_enable(rbsog_handle *h, int enable)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    HIPCHECK(harvest(h));
    if (enable && h->events.empty()) {
        h->events.resize(kTimingEvents);
        for (auto &e : h->events) HIPCHECK(hipEventCreate(&e));
    }
    h->timing = enable != 0;
    for (int k = 0; k < RBSOG_NUM_KERNEL_CLASSES; ++k) {
        h->timing_ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return RBSOG_OK;
}

extern "C" int rbsog_timing_read(rbsog_handle *h, rbsog_timing *out)
{
    if (!h || !out) return fail(RBSOG_EINVAL, "null handle or out");
    HIPCHECK(harvest(h));
    for (int k = 0; k < RBSOG_NUM_KERNEL_CLASSES; ++k) {
        out->ms[k] = h->timing_ms[k];
        out->launches[k] = h->launches[k];
        h->timing_ms[k] = 0.0;
        h->launches[k] = 0;
    }
    return RBSOG_OK;
}

extern "C" int rbsog_set_kT(rbsog_handle *h, double kT)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    if (!(kT > 0.0) || !std::isfinite(kT)) return fail(RBSOG_EINVAL, "kT must be positive and finite");
    if (h->d.full_k) {   // no sampling: the full lattice does not depend on kT
        h->p.kT = kT;
        return RBSOG_OK;
    }
    rbsog_params p = h->p;
    p.kT = kT;
    Tables t;
    build_tables(h->sog, p, h->Q2, h->d.mmax, &t, false);
    if (t.nshell != h->nshell) return fail(RBSOG_EINVAL, "shell count changed with kT");
    hipError_t e = hipSuccess;
    if (!h->kt_host) {
        e = hipHostMalloc((void **)&h->kt_host, sizeof(double) * 2 * (size_t)h->nshell, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->kt_ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail(RBSOG_EHIP, "rbsog_set_kT staging: %s", hipGetErrorString(e));
    } else {
        e = hipEventSynchronize(h->kt_ev);   // the previous upload has left the staging buffer
        if (e != hipSuccess) return fail(RBSOG_EHIP, "rbsog_set_kT: %s", hipGetErrorString(e));
    }
    std::copy(t.cdf.begin(), t.cdf.end(), h->kt_host);
    std::copy(t.coef.begin(), t.coef.end(), h->kt_host + h->nshell);
    // stream order puts the new tables after every draw enqueued before this call
    e = hipMemcpyAsync(h->cdf, h->kt_host, sizeof(double) * h->nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->coef, h->kt_host + h->nshell, sizeof(double) * h->nshell, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = hipEventRecord(h->kt_ev, h->st);
    if (e != hipSuccess) return fail(RBSOG_EHIP, "rbsog_set_kT upload: %s", hipGetErrorString(e));
    if (kT > h->p.kT) h->dt_checked = 0.0;   // a hotter system: the default skin's thermal check runs again
    h->p.kT = kT;
    h->S = t.S;
    h->samp_n = 0;   // modes drawn ahead with the old measure are drawn again
    return RBSOG_OK;
}

extern "C" int rbsog_set_bath(rbsog_handle *h, int kind, double rate, double kT)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    if (kind < RBSOG_BATH_NONE || kind > RBSOG_BATH_BERENDSEN) return fail(RBSOG_EINVAL, "unknown bath kind");
    if (kind != RBSOG_BATH_NONE) {
        if (!(rate > 0.0) || !std::isfinite(rate)) return fail(RBSOG_EINVAL, "the bath rate must be positive and finite");
        if (!(kT > 0.0) || !std::isfinite(kT))
            return fail(RBSOG_EINVAL, "the bath temperature must be positive and finite");
    }
    if (kind != RBSOG_BATH_NONE && kT > h->bath_kT) h->dt_checked = 0.0;   // the default skin's thermal check runs again
    h->bath_kind = kind;
    h->friction = kind == RBSOG_BATH_LANGEVIN ? rate : 0.0;
    h->bath_rate = kind == RBSOG_BATH_NONE ? 0.0 : rate;
    h->bath_kT = kind == RBSOG_BATH_NONE ? 0.0 : kT;
    if (kind == RBSOG_BATH_NOSE_HOOVER || kind == RBSOG_BATH_BERENDSEN) {   // xi and eta restart at 0
        static const double zero[kBathWords] = {};
        HIPCHECK(hipMemcpyAsync(h->bath, zero, sizeof(zero), hipMemcpyHostToDevice, h->st));
    }
    return RBSOG_OK;
}

extern "C" int rbsog_set_thermostat(rbsog_handle *h, double friction, double kT)
{
    if (!h) return fail(RBSOG_EINVAL, "null handle");
    if (!(friction >= 0.0) || !std::isfinite(friction)) return fail(RBSOG_EINVAL, "friction must be >= 0 and finite");
    return rbsog_set_bath(h, friction > 0.0 ? RBSOG_BATH_LANGEVIN : RBSOG_BATH_NONE, friction, kT);
}

extern "C" int rbsog_bath_state(rbsog_handle *h, double *out)
{
    if (!h || !out) return fail(RBSOG_EINVAL, "null handle or out");
    double b[kBathWords];
    HIPCHECK(hipMemcpyAsync(b, h->bath, sizeof(b), hipMemcpyDeviceToHost, h->st));
    HIPCHECK(hipStreamSynchronize(h->st));
    out[0] = b[0];
    out[1] = b[1];
    return RBSOG_OK;
}

extern "C" void rbsog_destroy(rbsog_handle *h)
{
    if (!h) return;
    if (!h->records.empty()) (void)hipStreamSynchronize(h->st);
    if (h->kt_ev) {
        (void)hipEventSynchronize(h->kt_ev);
        (void)hipEventDestroy(h->kt_ev);
    }
    if (h->kt_host) (void)hipHostFree(h->kt_host);
    for (auto &e : h->events) (void)hipEventDestroy(e);
    if (h->rb_ev) {
        (void)hipEventSynchronize(h->rb_ev);
        (void)hipEventDestroy(h->rb_ev);
    }
    if (h->rb_host) (void)hipHostFree(h->rb_host);
    delete h;
}

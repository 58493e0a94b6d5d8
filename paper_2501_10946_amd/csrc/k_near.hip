// gfx950 kernel of librbsog: the near field of eq. (3.8),
//   f_i = sum_{j : |d| < r_c} q_i q_j [F_N1(r) + F_N2(r)] d,   d = r_i - r_j (minimum image),
//   F_N1 = exp(-r/lambda)(1 + r/lambda)/r^3,  F_N2 = -2 sum_g c_g s_g exp(-s_g r^2),
//   (F_N1 summed over the terms a_t exp(-r/l_t)(1 + r/l_t)/r^3 of a two-term kernel),
// and the near energy U_N = 1/2 sum q_i q_j (Y(r) - F(r)).
//
// The cell grid is the fine one, cells of width w = L / floor(2L / (r_c + skin))
// >= (r_c + skin) / 2, so the neighbour stencil is 5 x 5 x 5 cells; cell order
// makes each x-row of 5 cells one contiguous index range (two where it wraps
// around the box).  Work is split into (particle, plane) lanes, plane dz =
// -2..2 of the stencil; rows and x-cells whose distance from the particle
// already exceeds the list radius are skipped per particle.
//
//   k_nlist  a wave lists the particles of two x-adjacent cells: lanes take
//            the candidates of the pair's 5 x 5 x 6-cell window 64 at a time
//            (loads coalesced along the rows) and test each against every
//            home particle in turn; the accepted ones are appended in lane
//            order straight into the particles' lists (tile-major: 64
//            particles side by side per row, a tile's rows contiguous), in
//            window order, with a count per particle;
//   k_near   a workgroup owns 256 consecutive particles and one of the
//            kNearLanes lanes per particle (4 waves); lane s evaluates entries
//            s, s + kNearLanes, ... of the particle's list, so the lanes get
//            equal shares (a split by plane would not: the outer planes hold 0
//            to ~17 entries depending on where the particle sits in its cell).
//            Each lane runs down its entries with the next index and the next
//            neighbour position already in flight, and stores its partial
//            force; the far-field kernel adds the partials in lane order.  In FP64
//            the pair function is, when its fit is accurate, one polynomial
//            in r (r^3 times the force factor, 24 to 28 FMAs, no exponential),
//            otherwise the number of Gaussians is a template parameter for
//            the common counts; coefficients stay in scalar registers.  When a
//            particle's list overflowed at the build, its lanes walk the
//            candidates of the current positions, plane by plane.  A
//            single system's launch also computes the structure-factor
//            partial sums in its first workgroups: the gathers above leave
//            the arithmetic units idle much of the time, the partial sums
//            keep them busy (the reduction follows as a launch of its own).
//
// Lists hold every j within r_c + skin at the build.  The step path rebuilds
// them (and the cell order) only when some particle has moved more than
// skin / 2 since the last build, so every pair within r_c is listed; pairs
// listed but now beyond r_c are skipped in the evaluation.
//
// Each lane sums its share of a particle's force in list order and the
// shares are added in a fixed order: the result is deterministic.
#include <hip/hip_runtime.h>

#include "dev_common.h"

namespace rbsog {

constexpr int kNearPlanes = 5;                 // stencil planes dz = -2..2
constexpr int kListThreads = 64 * kListWaves;  // list build: one cell pair per wave
constexpr int kEvalThreads = 256;              // evaluation: 256 particles x 1 plane
constexpr int kShiftBits = 5;                  // image-shift code 0..26 in the top bits of a range start
constexpr uint32_t kIndexMask = (1u << (32 - kShiftBits)) - 1u;

__device__ inline double shift_of(int code, double L) { return (double)(code - 1) * L; }

// Distance from coordinate y to the slab [c w - m, (c + 1) w + m] (0 inside).
__device__ inline double slab_gap(double y, int c, double w, double m)
{
    double lo = (double)c * w - m, hi = (double)(c + 1) * w + m;
    return fmax(0.0, fmax(lo - y, y - hi));
}

// One candidate range: particles [start, end) of the cell-ordered copy, all
// under one image shift (code = xc + 3 yc + 9 zc, each 0/1/2 for -L/0/+L).
struct Range {
    int32_t start_code;     // start | code << 27
    int32_t end;
};

// The (particle, plane) a lane works on, with its home cell.
struct Lane {
    int p, plane;
    double4 pi;
    int cx, cy, cz, zc;     // home x, y; wrapped z cell of the plane and its shift code
    double gz;              // z-gap from the particle to the plane
};

__device__ inline Lane make_lane(const NearArgs &a, int p, int plane)
{
    Lane l;
    l.p = p;
    l.plane = plane;
    l.pi = make_double4(0.0, 0.0, 0.0, 0.0);
    l.cx = l.cy = l.cz = 0;
    l.zc = 1;
    l.gz = 1e300;
    if (p < a.N) {
        const int nfz = a.g.nc[2];
        l.pi = a.xs[p];
        l.cx = cell_coord(l.pi.x, a.g.inv_cell[0], a.g.nc[0]);
        l.cy = cell_coord(l.pi.y, a.g.inv_cell[1], a.g.nc[1]);
        int czu = cell_coord(l.pi.z, a.g.inv_cell[2], nfz) + plane - 2;
        l.gz = slab_gap(l.pi.z, czu, a.w[2], a.margin);
        l.cz = czu;
        if (czu < 0) { l.cz += nfz; l.zc = 0; } else if (czu >= nfz) { l.cz -= nfz; l.zc = 2; }
    }
    return l;
}

// The candidate ranges of row `row` (dy = row - 2) for a lane within radius
// sqrt(R2) (R2 <= the list radius squared, which the fine grid is built for):
// 0, 1 or 2 ranges.
__device__ inline int row_ranges(const NearArgs &a, const Lane &l, int row, double R2, Range out[2])
{
    const int nf = a.g.nc[0], nfy = a.g.nc[1];
    const double m = a.margin;
    int cyu = l.cy + row - 2;
    double gy = slab_gap(l.pi.y, cyu, a.w[1], m);
    double rem = R2 - gy * gy - l.gz * l.gz;
    if (!(rem > 0.0)) return 0;
    int dxlo = -2, dxhi = 2;
    for (int k = 0; k < 2; ++k) {   // at most two x-cells per side can be culled
        double gl = slab_gap(l.pi.x, l.cx + dxlo, a.w[0], m);
        if (dxlo < 0 && !(gl * gl < rem)) ++dxlo;
        double gh = slab_gap(l.pi.x, l.cx + dxhi, a.w[0], m);
        if (dxhi > 0 && !(gh * gh < rem)) --dxhi;
    }
    int xa = l.cx + dxlo, xb = l.cx + dxhi;   // unwrapped; xb - xa <= 4 < nf
    int cyw = cyu, yc = 1;
    if (cyw < 0) { cyw += nfy; yc = 0; } else if (cyw >= nfy) { cyw -= nfy; yc = 2; }
    int base = (l.cz * nfy + cyw) * nf;
    int code = 3 * yc + 9 * l.zc;
    int n = 0;
    // piece left of the wrap (or the whole row), then the piece past it
    int lo0 = xa < 0 ? xa + nf : xa, hi0 = xa < 0 ? nf - 1 : min(xb, nf - 1);
    int xc0 = xa < 0 ? 0 : 1;
    int s0 = a.cell_start[base + lo0], e0 = a.cell_start[base + hi0 + 1];
    // (out[] written at fixed indices only, so that it stays in registers)
    if (s0 < e0) {
        out[0] = Range{(int32_t)((uint32_t)s0 | ((uint32_t)(code + xc0) << 27)), e0};
        n = 1;
    }
    if (xa < 0 || xb > nf - 1) {
        int hi1 = xa < 0 ? xb : xb - nf;
        int xc1 = xa < 0 ? 1 : 2;
        int s1 = a.cell_start[base], e1 = a.cell_start[base + hi1 + 1];
        if (s1 < e1) {
            const Range r{(int32_t)((uint32_t)s1 | ((uint32_t)(code + xc1) << 27)), e1};
            if (n == 0) out[0] = r;
            else out[1] = r;
            ++n;
        }
    }
    return n;
}

// FP64 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps.
__device__ inline double rsqrt_f64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double hx = 0.5 * x;
    double e = fma(-hx * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-hx * y, y, 0.5);
    return fma(y, e, y);
}

// Gaussians of the pair function: NG > 0 is a compile-time count, 0 the
// run-time count of the argument block; NG < 0: the whole pair function from
// the polynomials of the argument block, of degree -NG (FP64).  kPolyNG, the
// full degree, also serves polynomials of a lower degree (their higher powers
// are zero, and Horner's first steps then leave the leading coefficient
// unchanged, so the result is the same bit for bit).
constexpr int kPolyNG = -28;
template <int NG>
__device__ inline int gauss_count(const NearArgs &a) { return NG > 0 ? NG : a.sog.n; }

// Horner in y of the degree-D polynomial c (ascending powers).
template <int D>
__device__ inline double near_poly_eval(const double *c, double y)
{
    static_assert(D >= 1 && D <= 28, "the argument block holds 29 powers");
    double p = c[D];
#pragma unroll
    for (int k = D - 1; k >= 0; --k) p = fma(p, y, c[k]);
    return p;
}

// IMG: the axes (bit d for axis d) on which the minimum-image step is taken;
// the callers leave an axis out only where the step provably changes nothing
// (near_image_axes).
template <bool MIXED, bool ENERGY, int NG, int IMG = 7>
__device__ inline void pair_force(const NearArgs &a, const double4 &pi, const double4 &pj, double &fx, double &fy,
                                  double &fz, double &en, double &vir)
{
    // d by the minimum image (|d| < r_c <= L_d/3)
    double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
    if (IMG & 1) dx = fma(-a.g.L[0], rint(dx * a.inv_L[0]), dx);
    if (IMG & 2) dy = fma(-a.g.L[1], rint(dy * a.inv_L[1]), dy);
    if (IMG & 4) dz = fma(-a.g.L[2], rint(dz * a.inv_L[2]), dz);
    // written out as FMAs: the compiler's own contraction of a sum of squares
    // may pick another product to fuse depending on how d was formed, and the
    // IMG variants must give the same bits
    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (!(r2 < a.rc2)) return;   // listed within r_c + skin, beyond r_c now
    double qq = pi.w * pj.w;
    if (MIXED) {
        float r2f = (float)r2;
        float irf = __builtin_amdgcn_rsqf(r2f);
        float rf = r2f * irf;
        float ey = __builtin_amdgcn_exp2f(-rf * (float)a.sog.inv_lambda_log2e);
        float f1 = ey * (1.0f + rf * (float)a.sog.inv_lambda);
        if (a.sog.two) {   // the second Yukawa term of a two-term kernel
            const float ez = __builtin_amdgcn_exp2f(-rf * (float)a.sog.inv_lambda2_log2e);
            f1 = fmaf((float)a.sog.ya2, ez * (1.0f + rf * (float)a.sog.inv_lambda2), (float)a.sog.ya1 * f1);
            ey = fmaf((float)a.sog.ya2, ez, (float)a.sog.ya1 * ey);
        }
        f1 = f1 * (irf * irf * irf);
        float gs = 0.0f, fs = 0.0f;
#pragma unroll
        for (int g = 0; g < (NG < 0 ? 0 : gauss_count<NG>(a)); ++g) {
            float eg = __builtin_amdgcn_exp2f(-(float)a.sog.s_log2e[g] * r2f);
            gs = fmaf((float)a.sog.cs2[g], eg, gs);
            if (ENERGY) fs = fmaf((float)a.sog.c[g], eg, fs);
        }
        double fac = qq * (double)(f1 - gs);
        fx = fma(fac, dx, fx);
        fy = fma(fac, dy, fy);
        fz = fma(fac, dz, fz);
        if (ENERGY) {
            en = fma(qq, (double)(ey * irf - fs), en);
            vir = fma(fac, r2, vir);   // d . F of the pair
        }
    } else if constexpr (NG < 0) {
        // H(r) / r^3 and K(r) / r with H, K the polynomials in y = 2 r / r_c - 1
        double ir = rsqrt_f64(r2);
        double r = r2 * ir;
        const double y = fma(r, a.sog.y_scale, -1.0);
        double fac = qq * (near_poly_eval<-NG>(a.sog.hpoly, y) * (ir * ir * ir));
        fx = fma(fac, dx, fx);
        fy = fma(fac, dy, fy);
        fz = fma(fac, dz, fz);
        if (ENERGY) {
            en = fma(qq, near_poly_eval<-NG>(a.sog.kpoly, y) * ir, en);
            vir = fma(fac, r2, vir);   // d . F of the pair
        }
    } else {
        double ir = rsqrt_f64(r2);
        double r = r2 * ir;
        double ey = exp2_nonpos(-r * a.sog.inv_lambda_log2e, a.e2);
        double f1 = ey * fma(r, a.sog.inv_lambda, 1.0);
        if (a.sog.two) {   // the second Yukawa term of a two-term kernel
            const double ez = exp2_nonpos(-r * a.sog.inv_lambda2_log2e, a.e2);
            f1 = fma(a.sog.ya2, ez * fma(r, a.sog.inv_lambda2, 1.0), a.sog.ya1 * f1);
            ey = fma(a.sog.ya2, ez, a.sog.ya1 * ey);
        }
        f1 = f1 * (ir * ir * ir);
        double gs = 0.0, fs = 0.0;
        {
#pragma unroll
            for (int g = 0; g < gauss_count<NG>(a); ++g) {
                double eg = exp2_nonpos(-a.sog.s_log2e[g] * r2, a.e2);
                gs = fma(a.sog.cs2[g], eg, gs);
                if (ENERGY) fs = fma(a.sog.c[g], eg, fs);
            }
        }
        double fac = qq * (f1 - gs);
        fx = fma(fac, dx, fx);
        fy = fma(fac, dy, fy);
        fz = fma(fac, dz, fz);
        if (ENERGY) {
            en = fma(qq, ey * ir - fs, en);
            vir = fma(fac, r2, vir);   // d . F of the pair
        }
    }
}

// ---------------------------------------------------------------------------
// neighbour lists
// ---------------------------------------------------------------------------

// The value of v in lane l (l uniform), as a scalar.
__device__ inline double readlane_f64(double v, int l)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The window of cell pair q: two x-adjacent cells of the fine grid (the last
// cell of a row of odd length alone) hold the home particles [h_beg, h_end);
// their candidates are the particles of 25 rows (dz, dy = -2..2) of the cells
// x0 - 2 .. x1 + 2, each row one contiguous range of the cell order or two
// where it wraps, 50 pieces at most.  Lane l < 50 describes piece l; the
// pieces' starts, exclusive prefix sums of their lengths and image-shift codes
// (0/1/2 for -L/0/+L per axis) go to the wave's rows of pstart/ppref/pcode.
// Returns false, uniformly over the wave, when q is past the last pair or the
// pair has no home particle.  A window holds each particle at most once: it is
// at most 6 cells wide in x and 5 in y and z, and the grid has at least 6.
struct PairWindow {
    int h_beg, h_end, total;
};

__device__ inline bool pair_window(const NearArgs &a, int q, int32_t *pstart, int32_t *ppref, int32_t *pcode,
                                   PairWindow &win)
{
    const int lane = threadIdx.x & 63;
    const int nf = a.g.nc[0], nfy = a.g.nc[1], nfz = a.g.nc[2], half = (nf + 1) >> 1;
    if (q >= nfz * nfy * half) return false;
    const int row = q / half, ix = q - row * half;
    const int cz = row / nfy, cy = row - cz * nfy;
    const int x0 = 2 * ix, x1 = min(x0 + 1, nf - 1);
    const int cbase = (cz * nfy + cy) * nf;
    win.h_beg = a.cell_start[cbase + x0];
    win.h_end = a.cell_start[cbase + x1 + 1];
    if (win.h_beg >= win.h_end) return false;
    int ps = 0, plen = 0, pc = 0;
    if (lane < 2 * 25) {
        const int r = lane >> 1, k = lane & 1;
        int czw = cz + r / 5 - 2, zc = 1;
        if (czw < 0) { czw += nfz; zc = 0; } else if (czw >= nfz) { czw -= nfz; zc = 2; }
        int cyw = cy + r % 5 - 2, yc = 1;
        if (cyw < 0) { cyw += nfy; yc = 0; } else if (cyw >= nfy) { cyw -= nfy; yc = 2; }
        const int rb = (czw * nfy + cyw) * nf;
        const int xa = x0 - 2, xb = x1 + 2;   // at most 6 cells <= nf: one side wraps at most
        int lo = xa, hi = xb, xc = 1;
        bool has = k == 0;
        if (xa < 0) {
            has = true;
            if (k == 0) { lo = xa + nf; hi = nf - 1; xc = 0; } else { lo = 0; hi = xb; }
        } else if (xb > nf - 1) {
            has = true;
            if (k == 0) { hi = nf - 1; } else { lo = 0; hi = xb - nf; xc = 2; }
        }
        if (has) {
            ps = a.cell_start[rb + lo];
            plen = a.cell_start[rb + hi + 1] - ps;
            pc = xc | (yc << 2) | (zc << 4);
        }
    }
    int incl = plen;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int u = __shfl_up(incl, off);
        if (lane >= off) incl += u;
    }
    win.total = __shfl(incl, 63);
    pstart[lane] = ps;
    ppref[lane] = incl - plen;
    pcode[lane] = pc;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return true;
}

// The piece of cell pair q's window that holds its home particles (see
// pair_window): the central row's first piece, or its second when the row
// wraps at the low x side.
__device__ inline int pair_window_home_piece(const NearArgs &a, int q)
{
    const int half = (a.g.nc[0] + 1) >> 1;
    const int ix = q - (q / half) * half;
    return 2 * ix - 2 < 0 ? 25 : 24;
}

// The piece of candidate c (< the window's total): the last piece whose prefix
// is <= c (an empty piece shares the prefix of the next, so it is never the
// one found), by binary search over the 64 prefixes.
__device__ inline int window_piece(const int32_t *ppref, int c)
{
    int lo = 0, n = 64;
    while (n > 0) {
        int h2 = n >> 1;
        if (ppref[lo + h2] <= c) { lo += h2 + 1; n -= h2 + 1; }
        else n = h2;
    }
    return lo - 1;
}

// Candidate c of piece l of a window: its particle index j and the image shift
// (sx, sy, sz) the piece is seen under.
__device__ inline int window_candidate(const int32_t *pstart, const int32_t *ppref, const int32_t *pcode, int c,
                                       int l, const double Lb[3], double &sx, double &sy, double &sz)
{
    const int code = pcode[l];
    sx = shift_of(code & 3, Lb[0]);
    sy = shift_of((code >> 2) & 3, Lb[1]);
    sz = shift_of(code >> 4, Lb[2]);
    return pstart[l] + (c - ppref[l]);
}

// One wave lists the neighbours of the home particles of cell pair q,
// kListHomes of them per pass over the window.  Lanes take 64 consecutive
// candidates of the window at a time (loads coalesced along the rows); each
// home particle of the pass, its position read from LDS by every lane (a
// broadcast), is tested against all 64, and the accepted ones are appended
// in lane order (ballot / mbcnt) to that particle's list, the pass's running
// counts staying wave-uniform (scalar registers).  So a particle's list holds
// the candidates within the list radius in window order — planes, rows, wrap
// pieces, cell order — the same list, entry for entry, as a walk of the
// particle's own 5 x 5 x 5 cells: the pair window's extra cells lie at least
// 2 w >= r_c + skin away from the other cell's particles.  A particle with
// more than list_rows(kp) neighbours gets the count list_rows(kp) + 1 (its
// lanes then walk the cells in the evaluation).
constexpr int kListHomes = 16;
// windows of up to this many candidates get a table of each candidate's piece
// (one byte each, in LDS), written once per window: a lookup per candidate in
// place of a binary search per chunk of candidates, which the few home
// particles of a cell pair (~8 at the N = 1e6 plasma) would otherwise share
constexpr int kPieceTab = 2048;
static_assert(kListBlock == 8, "a list block is read as two int4");

__device__ inline void nlist_pair(const NearArgs &a, int q, int wv)
{
    __shared__ int32_t pstart[kListWaves][64], ppref[kListWaves][64], pcode[kListWaves][64];
    __shared__ double hpos[kListWaves][3][kListHomes];
    __shared__ uint8_t pidx[kListWaves][kPieceTab];
    const int lane = threadIdx.x & 63;
    PairWindow win;
    if (!pair_window(a, q, pstart[wv], ppref[wv], pcode[wv], win)) return;   // uniform per wave
    const int total = win.total;
    const bool tabled = total <= kPieceTab;   // uniform
    if (tabled) {   // lane l writes its piece's index over the piece's candidates
        const int b0 = ppref[wv][lane], b1 = lane < 63 ? ppref[wv][lane + 1] : total;
        for (int t = b0; t < b1; ++t) pidx[wv][t] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    const int rows = list_rows(a.kp);
    // The home particles are consecutive candidates of the window's central
    // row (dy = dz = 0, no image shift): piece 24 of that row, or piece 25
    // when the row wraps at the low x side (its first piece is then the
    // wrapped cells).  home_c is the candidate index of h_beg, so the lane
    // that holds a home itself follows from the lane's candidate index.
    const int lhome = pair_window_home_piece(a, q);
    const int home_c = __builtin_amdgcn_readfirstlane(ppref[wv][lhome] + (win.h_beg - pstart[wv][lhome]));
    // the list radius with a relative margin of 1e-12: a candidate is tested
    // as home - (its position + image shift), the evaluation forms the same
    // difference in another order, and a pair on the radius must not be lost
    // to the rounding (extra pairs beyond r_c are skipped by the evaluation)
    const double R2 = a.rl2 * (1.0 + 1e-12);
    for (int hb = win.h_beg; hb < win.h_end; hb += kListHomes) {
        const int nh = min(kListHomes, win.h_end - hb);
        if (lane < nh) {
            const double4 r = a.xs[hb + lane];
            hpos[wv][0][lane] = r.x;
            hpos[wv][1][lane] = r.y;
            hpos[wv][2][lane] = r.z;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the pass's homes' lists are consecutive rows from pass_row on; slot[hh]
        // is the next entry of home hh counted from pass_row (hh rows + count)
        int32_t *pass_row = a.nbr + list_at(hb, 0, rows);
        uint32_t slot[kListHomes];
#pragma unroll
        for (int hh = 0; hh < kListHomes; ++hh) slot[hh] = (uint32_t)(hh * rows);
        const int hc = home_c + (hb - win.h_beg);   // candidate index of the pass's first home
        for (int c0 = 0; c0 < total; c0 += 64) {
            const int c = c0 + lane;
            const bool live = c < total;
            const uint64_t live_m = __builtin_amdgcn_ballot_w64(live);
            const int own = c - hc;   // the pass's home whose own lane this is (any other value: none)
            int j = -1;
            double px = 0.0, py = 0.0, pz = 0.0;   // the candidate, image-shifted
            if (live) {
                double sx, sy, sz;
                const int l = tabled ? (int)pidx[wv][c] : window_piece(ppref[wv], c);
                j = window_candidate(pstart[wv], ppref[wv], pcode[wv], c, l, a.g.L, sx, sy, sz);
                const double4 qj = a.xs[j];
                px = qj.x + sx;
                py = qj.y + sy;
                pz = qj.z + sz;
            }
#pragma unroll
            for (int hh = 0; hh < kListHomes; ++hh) {
                if (hh < nh) {   // uniform
                    // the home's position is read from LDS at each test (a
                    // broadcast), not held in registers for every home
                    __asm__ volatile("" ::: "memory");
                    const double dx = hpos[wv][0][hh] - px, dy = hpos[wv][1][hh] - py, dz = hpos[wv][2][hh] - pz;
                    // the accepted lanes as one wave mask (the distance test,
                    // the live lanes, not the home's own lane); the appends
                    // run under it, at positions by mbcnt.  Appends past the
                    // capacity all land on the row's last entry: the list is
                    // then marked overflowed and never read.
                    const uint64_t m = __builtin_amdgcn_ballot_w64(dx * dx + dy * dy + dz * dz < R2) & live_m &
                                       __builtin_amdgcn_ballot_w64(own != hh);
                    if (__builtin_amdgcn_inverse_ballot_w64(m)) {
                        const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, slot[hh]));
                        const uint32_t kk = min(k, (uint32_t)(hh * rows + rows - 1));
                        *(int32_t *)((char *)pass_row + (kk << 2)) = j;
                    }
                    slot[hh] += (uint32_t)__popcll(m);
                }
            }
        }
        int mine = 0;
#pragma unroll
        for (int hh = 0; hh < kListHomes; ++hh)
            if (lane == hh) mine = (int)(slot[hh] - (uint32_t)(hh * rows));
        if (lane < nh) a.nbr_cnt[hb + lane] = mine > rows ? rows + 1 : mine;
        // the positions of the next pass overwrite these
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__device__ inline void nlist_body(const NearArgs &a, int lb)
{
    if (a.gate && *a.gate == 0) return;
    const int wv = threadIdx.x >> 6;
    nlist_pair(a, lb * kListWaves + wv, wv);
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------

// The axes on which a pair of this wave may need the minimum image (bit d:
// axis d), uniform over the wave: those along which some home particle lies
// within r_c of a face (with a relative margin of 1e-6).  A home particle
// farther from both faces of an axis sees every particle within r_c of it at
// its own unwrapped coordinate on that axis, so the raw difference is the
// displacement itself and the minimum-image step would return it unchanged
// (rint of a ratio below 1/2 is 0); a farther particle shows a raw difference
// at least as large as its true one and stays beyond r_c either way.  Lanes
// past N count as interior.  1 for the x axis alone (a wave of cell-ordered
// particles crosses the box along x), 7 whenever y or z is needed.
__device__ inline int near_image_axes(const NearArgs &a, const double4 &pi, int p)
{
    const double m = sqrt(a.rc2) * (1.0 + 1e-6);
    const bool live = p < a.N;
    const bool ex = live && !(pi.x >= m && pi.x <= a.g.L[0] - m);
    const bool eyz = live && !(pi.y >= m && pi.y <= a.g.L[1] - m && pi.z >= m && pi.z <= a.g.L[2] - m);
    if (__builtin_amdgcn_ballot_w64(eyz)) return 7;
    return __builtin_amdgcn_ballot_w64(ex) ? 1 : 0;
}

// Row j of the cell-ordered positions by a 32-bit byte offset from the
// wave-uniform base (j < 2^27: the offset fits), one address operation
// fewer per neighbour than a 64-bit index.
__device__ inline double4 xs_row(const NearArgs &a, int j)
{
    return *(const double4 *)((const char *)a.xs + ((uint32_t)j << 5));
}

// A lane's share of particle p's list (total <= rows entries): lane s takes
// blocks s, s + kNearLanes, ... (kListBlock consecutive entries each).  A
// block's indices arrive as two 16-byte loads while the block before is
// evaluated, and within a block the positions of two entries are loading
// while the two before are evaluated.  Entries past the count are not used:
// the particle itself (or the last one, for lanes past N) stands in for them
// and is never evaluated.
template <bool MIXED, bool ENERGY, int NG, int IMG>
__device__ inline void near_list(const NearArgs &a, const double4 &pi, int p, int s, int total, int rows, double &fx,
                                 double &fy, double &fz, double &en, double &vir)
{
    const int nblk = (total + kListBlock - 1) / kListBlock;
    const int self = p < a.N ? p : a.N - 1;
    const int32_t *blk = a.nbr + list_at(p, 0, rows);   // block b at blk + b * bstride
    const size_t bstride = (size_t)kListBlock;
    int4 n0 = make_int4(self, self, self, self), n1 = n0;
    if (s < nblk) {
        n0 = *(const int4 *)(blk + (size_t)s * bstride);
        n1 = *(const int4 *)(blk + (size_t)s * bstride + 4);
    }
    for (int b = s; b < nblk; b += kNearLanes) {
        const int ne = min(kListBlock, total - b * kListBlock);
        int jj[kListBlock] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
        const int bn = b + kNearLanes;
        if (bn < nblk) {
            n0 = *(const int4 *)(blk + (size_t)bn * bstride);
            n1 = *(const int4 *)(blk + (size_t)bn * bstride + 4);
        }
#pragma unroll
        for (int e = 0; e < kListBlock; ++e)
            if (e >= ne) jj[e] = self;
        double4 qa = xs_row(a, jj[0]), qb = xs_row(a, jj[1]);
#pragma unroll
        for (int e = 0; e < kListBlock; e += 2) {
            const double4 ca = qa, cb = qb;
            if (e + 2 < kListBlock) {
                qa = xs_row(a, jj[e + 2]);
                qb = xs_row(a, jj[e + 3]);
            }
            if (e < ne) pair_force<MIXED, ENERGY, NG, IMG>(a, pi, ca, fx, fy, fz, en, vir);
            if (e + 1 < ne) pair_force<MIXED, ENERGY, NG, IMG>(a, pi, cb, fx, fy, fz, en, vir);
        }
    }
}

// lb: the logical workgroup (256 particles, one of kNearLanes lanes each).
// SPLIT: choose the minimum-image axes per wave (near_image_axes); the served
// ensemble's small replicas have nearly every wave at a face, so their batch
// launch takes every axis and saves the code.
template <bool MIXED, bool ENERGY, int NG, bool SPLIT = true>
__device__ inline void near_body(const NearArgs &a, int lb)
{
    __shared__ double2 red[kEvalThreads];
    const int t = threadIdx.x;
    const int grp = lb / kNearLanes;
    const int s = lb - grp * kNearLanes;   // this lane of the particle
    const int p = grp * kEvalThreads + t;
    double4 pi = make_double4(0.0, 0.0, 0.0, 0.0);
    int total = 0;
    if (p < a.N) {
        pi = a.xs[p];
        total = a.nbr_cnt[p];
    }
    double fx = 0.0, fy = 0.0, fz = 0.0, en = 0.0, vir = 0.0;
    const int rows = list_rows(a.kp);
    if (total <= rows) {
        // the minimum-image axes: uniform over the lanes that take this branch
        const int img = SPLIT ? near_image_axes(a, pi, p) : 7;
        if (img == 0) near_list<MIXED, ENERGY, NG, 0>(a, pi, p, s, total, rows, fx, fy, fz, en, vir);
        else if (img == 1) near_list<MIXED, ENERGY, NG, 1>(a, pi, p, s, total, rows, fx, fy, fz, en, vir);
        else near_list<MIXED, ENERGY, NG, 7>(a, pi, p, s, total, rows, fx, fy, fz, en, vir);
    } else {
        // the particle's list overflowed at the build: its lanes walk the
        // cells of the stencil planes dz = plane - 2 (lane s the planes s,
        // s + kNearLanes, ...) around the current position.  Particles may
        // have moved up to skin/2 out of the cells they were sorted into (and
        // wrapped around the box), so the cells are culled with the list
        // radius and the pair function itself (minimum image, r < r_c)
        // decides.
        for (int plane = s; plane < kNearPlanes; plane += kNearLanes) {
            const Lane l = make_lane(a, p, plane);
            if (l.gz * l.gz < a.rl2) {
                for (int row = 0; row < 5; ++row) {
                    Range g[2];
                    const int n = row_ranges(a, l, row, a.rl2, g);
#pragma unroll
                    for (int k = 0; k < 2; ++k) {   // fixed indices: g stays in registers
                        if (k >= n) break;
                        const int j0 = g[k].start_code & (int32_t)kIndexMask;
                        for (int j = j0; j < g[k].end; ++j)
                            if (j != p) pair_force<MIXED, ENERGY, NG>(a, pi, a.xs[j], fx, fy, fz, en, vir);
                    }
                }
            }
        }
    }
    if (p < a.N) {
        double *o = a.fnear + (size_t)s * 3 * a.N + p;
        o[0] = fx;
        o[a.N] = fy;
        o[2 * (size_t)a.N] = fz;
    }
    if (ENERGY) {   // each pair is seen from both ends: half of its energy and virial from each
        red[t] = make_double2(0.5 * en, 0.5 * vir);
        __syncthreads();
        for (int off = kEvalThreads / 2; off > 0; off >>= 1) {
            if (t < off) red[t] = make_double2(red[t].x + red[t + off].x, red[t].y + red[t + off].y);
            __syncthreads();
        }
        if (t == 0) {
            a.epart[lb] = red[0].x;
            a.epart[near_blocks(a.N) + lb] = red[0].y;
        }
    }
}

// Single system: workgroups remapped so that neighbouring groups share an XCD.
__global__ __launch_bounds__(kListThreads) void k_nlist(NearArgs a)
{
    nlist_body(a, xcd_block((int)blockIdx.x, (int)gridDim.x));
}

// Mixed precision without energies: held to the registers of 5 waves per SIMD
// (it needs a few more than 96 otherwise, and its gathers want the waves).
template <bool MIXED, bool ENERGY, int NG>
__global__ __launch_bounds__(kEvalThreads) __attribute__((amdgpu_waves_per_eu(MIXED && !ENERGY ? 5 : 1))) void k_near(
    NearArgs a)
{
    static_assert(kEvalThreads == kBlock, "the structure-factor workgroups have kBlock threads");
    const int b = (int)blockIdx.x;
    if (a.nrho == 0 || !a.interleave) {
        if (b < a.nrho) {   // uniform per workgroup
            if (b < rho_blocks(a.red.nchunk, a.red.P)) rho_partial_body<true, MIXED, true>(a.red, b);
            return;
        }
        near_body<MIXED, ENERGY, NG>(a, xcd_block(b - a.nrho, (int)gridDim.x - a.nrho));
        return;
    }
    // The structure-factor workgroups are spread evenly through the launch in
    // whole groups of 8 (one per XCD), so that every compute unit holds
    // arithmetic-bound partial sums beside the near field's gather-bound
    // waves; the near groups keep their dispatch order, and with it the XCD
    // mapping, and the partial last group is a near group.
    const int64_t gr = a.nrho / 8, gn = (gridDim.x - a.nrho + 7) / 8, G = gr + gn;
    const int64_t g = b / 8;
    const int64_t before = (g * gr + G - 1) / G;          // structure-factor groups before group g
    const int64_t upto = ((g + 1) * gr + G - 1) / G;
    if (upto > before) {   // uniform per workgroup
        const int rb = (int)(before * 8 + (b & 7));
        if (rb < rho_blocks(a.red.nchunk, a.red.P)) rho_partial_body<true, MIXED, true>(a.red, rb);
        return;
    }
    near_body<MIXED, ENERGY, NG>(a, xcd_block((int)((g - before) * 8 + (b & 7)), (int)gridDim.x - a.nrho));
}

__global__ __launch_bounds__(kListThreads) void k_nlist_batch(const NearArgs *__restrict__ tab,
                                                              const EnsItem *__restrict__ items)
{
    const EnsItem e = items[blockIdx.x];
    nlist_body(tab[e.r], e.b);
}

template <bool MIXED, bool ENERGY, int NG>
__global__ __launch_bounds__(kEvalThreads) void k_near_batch(const NearArgs *__restrict__ tab,
                                                             const EnsItem *__restrict__ items)
{
    const EnsItem e = items[blockIdx.x];
    if constexpr (NG == 0) {
        near_body<MIXED, ENERGY, NG, false>(tab[e.r], e.b);
    } else {
        // read before any store, the copy's fields become scalar loads
        const NearArgs a = tab[e.r];
        near_body<MIXED, ENERGY, NG, false>(a, e.b);
    }
}

// A launch with a missing buffer is refused on the host.
static bool near_args_ok(const NearArgs &a)
{
    return a.N >= 1 && a.xs && a.cell_start && a.nbr && a.nbr_cnt && a.fnear && a.kp >= 1 &&
           a.g.nc[0] >= 6 && a.g.nc[1] >= 6 && a.g.nc[2] >= 6 &&
           a.rc2 > 0.0 && a.rl2 >= a.rc2 && a.w[0] > 0.0 && a.w[1] > 0.0 && a.w[2] > 0.0 && (!a.energy || a.epart) && a.nrho >= 0 && a.nrho % 8 == 0 &&
           (a.nrho == 0 || (a.red.xs && rho_partial_ok(a.red) && a.red.mixed == a.mixed && (a.mixed || a.red.tab_fine) &&
                            a.nrho >= rho_blocks(a.red.nchunk, a.red.P)));
}

hipError_t launch_nlist(const NearArgs &a, hipStream_t st)
{
    if (!near_args_ok(a)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nlist, dim3(nlist_blocks(a.g.nc)), dim3(kListThreads), 0, st, a);
    return hipGetLastError();
}

template <bool MIXED, bool ENERGY>
static void launch_near_ng(const NearArgs &a, dim3 grid, hipStream_t st)
{
    dim3 block(kEvalThreads);
    const size_t lds = a.nrho > 0 ? rho_lds_bytes(a.red.P, a.red.chunk, MIXED, true) : 0;
    if (!MIXED && a.sog.poly) {   // the polynomials' degree: 24, 26 or 28
        if (a.sog.poly <= 24) hipLaunchKernelGGL((k_near<false, ENERGY, -24>), grid, block, lds, st, a);
        else if (a.sog.poly <= 26) hipLaunchKernelGGL((k_near<false, ENERGY, -26>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((k_near<false, ENERGY, kPolyNG>), grid, block, lds, st, a);
        return;
    }
    switch (a.sog.n) {
#define RBSOG_NEAR_NG(n) \
    case n: hipLaunchKernelGGL((k_near<MIXED, ENERGY, n>), grid, block, lds, st, a); return;
        RBSOG_NEAR_NG(1)
        RBSOG_NEAR_NG(2)
        RBSOG_NEAR_NG(3)
        RBSOG_NEAR_NG(4)
        RBSOG_NEAR_NG(5)
        RBSOG_NEAR_NG(6)
        RBSOG_NEAR_NG(7)
        RBSOG_NEAR_NG(8)
#undef RBSOG_NEAR_NG
    default: hipLaunchKernelGGL((k_near<MIXED, ENERGY, 0>), grid, block, lds, st, a); return;
    }
}

hipError_t launch_nlist_batch(const NearArgs *tab, const EnsItem *items, int n, hipStream_t st)
{
    if (!tab || !items || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_nlist_batch, dim3(n), dim3(kListThreads), 0, st, tab, items);
    return hipGetLastError();
}

hipError_t launch_near_batch(const NearArgs *tab, const EnsItem *items, int n, int ng, bool mixed, bool energy,
                             hipStream_t st)
{
    if (!tab || !items || n < 1 || ng < 0 || ng > 9 || (ng == 9 && mixed)) return hipErrorInvalidValue;
    if (ng == 9) {   // FP64 replicas whose Gaussian sums are polynomials
        if (energy) hipLaunchKernelGGL((k_near_batch<false, true, kPolyNG>), dim3(n), dim3(kEvalThreads), 0, st, tab,
                                       items);
        else hipLaunchKernelGGL((k_near_batch<false, false, kPolyNG>), dim3(n), dim3(kEvalThreads), 0, st, tab,
                                items);
        return hipGetLastError();
    }
    dim3 grid(n), block(kEvalThreads);
#define RBSOG_NEAR_B(M, E, G) \
    if (mixed == M && energy == E && ng == G) { \
        hipLaunchKernelGGL((k_near_batch<M, E, G>), grid, block, 0, st, tab, items); \
        return hipGetLastError(); \
    }
#define RBSOG_NEAR_BG(G) RBSOG_NEAR_B(true, true, G) RBSOG_NEAR_B(true, false, G) \
    RBSOG_NEAR_B(false, true, G) RBSOG_NEAR_B(false, false, G)
    RBSOG_NEAR_BG(0) RBSOG_NEAR_BG(1) RBSOG_NEAR_BG(2) RBSOG_NEAR_BG(3) RBSOG_NEAR_BG(4)
    RBSOG_NEAR_BG(5) RBSOG_NEAR_BG(6) RBSOG_NEAR_BG(7) RBSOG_NEAR_BG(8)
#undef RBSOG_NEAR_BG
#undef RBSOG_NEAR_B
    return hipErrorInvalidValue;
}

hipError_t launch_near(const NearArgs &a, hipStream_t st)
{
    if (!near_args_ok(a) || a.sog.n < 1 || a.sog.n > kMaxGauss) return hipErrorInvalidValue;
    dim3 grid(near_blocks(a.N) + a.nrho);
    if (a.mixed) {
        if (a.energy) launch_near_ng<true, true>(a, grid, st);
        else launch_near_ng<true, false>(a, grid, st);
    } else {
        if (a.energy) launch_near_ng<false, true>(a, grid, st);
        else launch_near_ng<false, false>(a, grid, st);
    }
    return hipGetLastError();
}

}  // namespace rbsog

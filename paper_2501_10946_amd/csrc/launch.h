// Kernel argument blocks and launcher declarations of librbsog.  Every device
// pointer here points into the caller's workspace or the caller's particle
// arrays; launchers enqueue on the given stream and return the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dev_math.h"

namespace rbsog {

constexpr int kBlock = 256;        // threads per workgroup of the streaming and pair kernels
constexpr int kScanPer = 8;        // cell counts per thread of the scan
constexpr int kScanTile = kBlock * kScanPer;
constexpr int kRhoChunkMax = 256;  // particles per structure-factor group (at most)
constexpr int kRhoStage = 1024;    // particles one structure-factor workgroup stages at most
constexpr int kMaxGauss = 32;

// One workgroup of a batched (ensemble) launch: replica slot r, workgroup b of
// that replica's own grid.
struct EnsItem {
    int32_t r, b;
};

// A kernel body `name##_body(const Args &, int b)` gives two kernels: k_name
// for one system (b = blockIdx.x) and k_name_batch over the items of a work
// list, each reading its replica's argument block from a device table.
#define RBSOG_KERNELS(name, Args, threads)                                                               \
    __global__ __launch_bounds__(threads) void k_##name(Args a) { name##_body(a, (int)blockIdx.x); }     \
    __global__ __launch_bounds__(threads) void k_##name##_batch(const Args *__restrict__ tab,             \
                                                               const EnsItem *__restrict__ items)      \
    {                                                                                                    \
        const EnsItem e = items[blockIdx.x];                                                             \
        name##_body(tab[e.r], e.b);                                                                      \
    }

// SOG coefficients as the kernels need them.
struct SogDev {
    int n;                      // Gaussians
    double inv_lambda;          // 1/lambda
    double inv_lambda_log2e;    // log2(e)/lambda: exp(-r/lambda) = 2^(-r log2(e)/lambda)
    // a second Yukawa term (the EGS kernel): Y = ya1 e^{-r/l1}/r + ya2 e^{-r/l2}/r
    // with l1 in inv_lambda above; two == 0 for the Yukawa kernel (ya1 = 1)
    int two;
    double ya1, ya2;
    double inv_lambda2, inv_lambda2_log2e;
    double c[kMaxGauss];        // F(r) = sum c exp(-s r^2)
    double s_log2e[kMaxGauss];  // s log2(e): exp(-s r^2) = 2^(-s log2(e) r^2)
    double cs2[kMaxGauss];      // 2 c s (force factor of the Gaussians)
    // the pair function as polynomials of y = r y_scale - 1 of degree poly
    // (0: none; the powers above it are zero)
    int poly;
    double y_scale;             // 2 / r_c
    double hpoly[29];           // r^3 (F_N1 + F_N2), ascending powers of y
    double kpoly[29];           // r (Y - F)
};

// Geometry of the cell list (a cube has equal entries on the three axes).
struct CellGeom {
    int nc[3];             // cells along x, y, z
    int ncell;             // nc[0] nc[1] nc[2]
    double L[3];           // box edges
    double inv_cell[3];    // nc[d] / L[d]
};

// --- cells -----------------------------------------------------------------
// The particle state lives in cell order: xs[p] = (x, y, z, q) of the particle
// in cell position p, order[p] its index in the caller's arrays.  A build sorts
// the current rows by (cell, caller index) and moves each row (and, when
// given, its velocity) to its new position; the id pass snapshots the rows so
// that the rank pass can write the new order in place.
struct CellArgs {
    int N;
    CellGeom g;
    double4 *xs;           // [N] (x, y, z, q) in cell order, rewritten in the new order
    int32_t *order;        // [N] cell order -> caller index, rewritten
    double *vs;            // null, or SoA [3][N] cell-order velocities carried into the new order
    double4 *xs_old;       // [N] snapshot of xs (id pass -> rank pass)
    int32_t *order_old;    // [N] snapshot of order
    double *vs_old;        // SoA [3][N] snapshot of vs (when vs)
    double *ms;            // [N] masses in cell order (valid in the old order on entry), rewritten
    double *ms_old;        // [N] snapshot of ms
    double *xb;            // SoA [3][N] positions at the build, new cell order
    int32_t *cell_id;      // [N] by current cell position
    int32_t *count;        // [ncell]
    int32_t *cell_start;   // [ncell + 1]
    int32_t *fill;         // [ncell]
    int32_t *tmp;          // [N] caller indices of each cell's members, unordered
    int32_t *tile_sum;     // [scan_tiles(ncell)] scan workspace
    int32_t *ticket;       // scan's finished-tile counter: zero between builds
    const int32_t *gate;   // null: always build; else build only when *gate != 0
};
__host__ __device__ inline int scan_tiles(int ncell) { return (ncell + kScanTile - 1) / kScanTile; }
// ids + counts + snapshot, scan (which leaves the counts zero again), scatter,
// stable rank + move; `count` must be zero on entry
hipError_t launch_cell_build(const CellArgs &a, hipStream_t st);
// the same for every replica of a work list: per256 has ceil(N/256) items per
// replica, pertile scan_tiles(ncell)
hipError_t launch_cell_build_batch(const CellArgs *tab, const EnsItem *per256, int n256, const EnsItem *pertile,
                                   int ntile, hipStream_t st);
hipError_t launch_set_int(int32_t *p, int32_t v, hipStream_t st);
// order[p] = p (a valid cell order before the first build)
hipError_t launch_iota(int32_t *order, int N, hipStream_t st);

// Caller arrays <-> cell order through order[]: state_in writes xs (x and q),
// ms, and vs / fs when given; state_out writes x, and v / f when given.
struct PermArgs {
    int N;
    const int32_t *order;
    double *x, *v, *f;     // SoA [3][N], caller order (v, f may be null; state_in only reads them)
    const double *q, *m;   // [N], caller order (state_in)
    double4 *xs;           // [N] cell order
    double *vs, *fs;       // SoA [3][N], cell order
    double *ms;            // [N], cell order
};
hipError_t launch_state_in(const PermArgs &a, hipStream_t st);
hipError_t launch_state_out(const PermArgs &a, hipStream_t st);

// --- integration ------------------------------------------------------------
// Langevin thermostat in the drift (on != 0): the drift becomes the A-O-A of
// the BAOAB splitting, x += (dt/2) v;  v = c1 v + sqrt(c2kT / m) z;  x += (dt/2) v,
// z the particle's normals for force index `step` (langevin_normals).
struct Thermo {
    int on;
    double c1;                 // exp(-friction dt)
    double c2kT;               // (1 - c1^2) k_B T of the bath
    uint64_t seed;
    uint32_t replica;
    uint64_t step;             // force index the drift leads to
};

// First half-kick and drift in cell order.
struct KickDriftArgs {
    int N;
    double L[3], inv_L[3], dt;
    double4 *xs;           // [N] (x, y, z, q), positions updated in place
    double *vs;            // SoA [3][N], updated in place
    const double *fs;      // SoA [3][N]
    const double *ms;      // [N]
    const double *xb;      // SoA [3][N] positions at the last list build
    double half_skin2;     // (skin / 2)^2
    int32_t *gate;         // raised when a particle moved more than skin / 2 since the build
    int32_t *gate_next;    // null, or the next step's gate, cleared
    int *flag;             // set to 1 on a step of a box length or more
    Thermo th;
    const int32_t *order;  // caller index of each row (the thermostat's noise counter; when th.on)
    const double *vscale;  // null, or a device factor the velocities take before the half-kick
};
hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t st);
hipError_t launch_kick_drift_batch(const KickDriftArgs *tab, const EnsItem *per256, int n, hipStream_t st);

// --- sampling ----------------------------------------------------------------
struct SampleArgs {
    int P;
    int nstep;                 // steps drawn: step .. step + nstep - 1
    uint64_t step, seed;
    uint32_t replica;
    int nshell;
    double S;
    const double *cdf;         // [nshell]
    const double *coef;        // [nshell]
    const int32_t *first;      // [nshell]
    const int32_t *size;       // [nshell]
    const int32_t *lattice;    // packed lattice vectors
    double4 *samp;             // [nstep][P] (nx, ny, nz, coef)
    int32_t *n_out;            // [P][3] or null (nstep == 1)
    double *coef_out;          // [P] or null (nstep == 1)
    // Metropolis-Hastings draws when mh is set: proposals from cdf_q (total
    // Sq), chain state mh[2] = (lattice index, shell index; -1 empty)
    const double *cdf_q;       // [nshell]
    double Sq;
    int32_t *mh;
};
// i.i.d. draws, or (a.mh set) the Metropolis-Hastings chain in one workgroup
hipError_t launch_sample(const SampleArgs &a, hipStream_t st);
// ensemble: items of 64 draws, ceil(P/64) per replica, nstep = 1
// (shift: device word holding the ensemble step counter)
hipError_t launch_sample_batch(const SampleArgs *tab, const EnsItem *items, int n, const uint64_t *shift,
                               hipStream_t st);

// --- structure factors -----------------------------------------------------------
struct RhoArgs {
    int N, P, nchunk, chunk;   // chunk = particles per group (a power of two, rho_chunk)
    double inv_L[3];           // 1 / L_d: k . r = 2 pi sum_d n_d x_d / L_d
    const double4 *xs;         // cell-ordered (x, y, z, q), or null to read x/q
    const double *x, *q;       // original-order SoA positions and charges
    const double4 *samp;       // [P]
    double2 *part;             // [nchunk][P] partial sums per (group, sample)
    double2 *rho;              // [P]
    double2 *gk;               // [P] coef * rho
    double *eF;                // [P] coef |rho|^2 / 2
    double *eW;                // null, or [P] coef |rho|^2 (3/2 - vm): the modes' far-field virial terms
    const double *vm;          // [m_max + 1] vm = k^2 G / Fhat by |n|^2 (a cube, when eW)
    // a cuboid (vm null, eW set): vm from k^2 = sum_d (2 pi n_d / L_d)^2 and the
    // decomposition's Fourier coefficients, Fhat = sum_g fa[g] exp(-fb[g] k^2)
    int nG;
    const double *fa, *fb;     // [nG] each
    double *rho_out;           // [P][2] or null
    int mixed;
    const double2 *tab;        // [kPhaseTab] (sin, cos)(2 pi j / kPhaseTab) (FP64 path)
    SinCosShort ss;
    // the far field's finer table ([kFarTab] entries), used by the partial
    // sums of a step (near launch, served ensemble): two FMA fewer per
    // (particle, mode) than the kPhaseTab form, at 14 KB more LDS
    const double2 *tab_fine;
    SinCosFar sf;
};
hipError_t launch_rho_partial(const RhoArgs &a, hipStream_t st);
bool rho_partial_ok(const RhoArgs &a);   // the partial launch's argument checks
hipError_t launch_rho_reduce(const RhoArgs &a, hipStream_t st);
// every mode of samp[P] over all particles of xs, rho/gk/eF written directly
hipError_t launch_rho_full(const RhoArgs &a, hipStream_t st);
// workgroups of the partial kernel and its dynamic LDS bytes
__host__ __device__ inline int64_t rho_blocks(int nchunk, int P) { return ((int64_t)nchunk * P + kBlock - 1) / kBlock; }
// (fine: the kFarTab table of a step's partial sums)
size_t rho_lds_bytes(int P, int chunk, bool mixed, bool fine);
// the reduction: one workgroup per kRedModes adjacent samples
constexpr int kRedModes = 4;
__host__ __device__ inline int rho_reduce_blocks(int P) { return (P + kRedModes - 1) / kRedModes; }
// ensemble: partials (rho_blocks items per replica, lds = the largest
// rho_lds_bytes), then the reduction (rho_reduce_blocks items per replica)
hipError_t launch_rho_batch(const RhoArgs *tab, const EnsItem *part_items, int npart, size_t lds, bool mixed,
                            const EnsItem *red_items, int nred, hipStream_t st);

// --- near field ------------------------------------------------------------
struct NearArgs {
    int N;
    CellGeom g;
    double rc2;
    SogDev sog;
    const double4 *xs;         // cell order
    const int32_t *cell_start;
    double *fnear;             // [kNearLanes][3][N] partial forces of the lanes of each particle, cell order
    double *epart;             // [2][near_blocks(N)] energy, then virial partials (when energy)
    int mixed;
    int energy;
    double w[3];               // cell widths L_d / nc_d (g is the fine grid, nc_d = floor(2 L_d / (r_c + skin)))
    double margin;             // slack of the per-particle cell culling
    double inv_L[3];
    Exp2Poly e2;
    int32_t *nbr;              // list_rows(kp) entries per particle (blocks, list_at): listed j in candidate order
    int32_t *nbr_cnt;          // [N] listed count per particle; list_rows(kp) + 1 when the list overflowed
    int kp;                    // list capacity: list_rows(kp) (about 5 kp) entries per particle
    double rl2;                // squared list radius (r_c + skin)^2; the fine grid has cells >= (r_c + skin)/2
    const int32_t *gate;       // list build: null = always, else only when *gate != 0
    // evaluation of one system: with nrho > 0, nrho workgroups (a multiple of
    // 8) compute the structure-factor partial sums of `red` instead (the launch
    // carries their dynamic LDS), so that they run alongside the near field,
    // whose gathers leave the arithmetic units idle much of the time: the
    // first nrho, or, with interleave, groups of 8 spread evenly through the
    // launch (either way the near workgroups keep their XCD mapping)
    int nrho;
    int interleave;
    RhoArgs red;
};
// near launches of at least this many workgroups (several rounds of the chip's
// resident workgroups) spread their structure-factor workgroups (interleave)
constexpr int64_t kInterleaveBlocks = 3072;
hipError_t launch_nlist(const NearArgs &a, hipStream_t st);
// workgroups per system: list build (cell pairs of the fine grid of nf cells per axis), evaluation
// (256 particles x one of 5 lanes), far field (64 particles)
// list build: one pair of x-adjacent cells per wave, kListWaves waves per workgroup
constexpr int kListWaves = 4;
__host__ __device__ inline int nlist_blocks(const int nf[3])
{
    return (nf[2] * nf[1] * ((nf[0] + 1) / 2) + kListWaves - 1) / kListWaves;
}
// Neighbour lists are particle-major: the `rows` entries of particle p are
// contiguous at list_at(p, 0, rows) (rows a multiple of kListBlock,
// list_rows), so a list build's append of a run of accepted candidates of one
// particle fills consecutive words and the lines of a list are written by the
// one wave that builds it; the evaluation reads a particle's entries in blocks
// of kListBlock (32 bytes, two 16-byte loads).  Measured at the N = 1e6 plasma
// against a layout with the 64 particles of a tile side by side per entry (or
// per block): the build's scattered one-word stores into 64-particle rows cost
// more than the evaluation gains from reading rows of 64 lanes.  Arrays hold
// list_padded(N) particles.
constexpr int kListBlock = 8;
__host__ __device__ inline int list_rows(int kp) { return (5 * kp + kListBlock - 1) / kListBlock * kListBlock; }
__host__ __device__ inline size_t list_at(int p, int k, int rows) { return (size_t)p * (size_t)rows + (size_t)k; }
__host__ __device__ inline int64_t list_padded(int64_t N) { return (N + 63) / 64 * 64; }
// evaluation: a particle's list is dealt round-robin to kNearLanes lanes (3
// measured fastest of 1..5 on the N = 1e5 plasma: longer runs per lane than 5,
// enough waves to hide the gathers unlike 1 or 2)
constexpr int kNearLanes = 3;
__host__ __device__ inline int near_blocks(int N) { return kNearLanes * ((N + 255) / 256); }
__host__ __device__ inline int far_blocks(int N) { return (N + 63) / 64; }
// ensemble: list builds (nlist_blocks items per replica); evaluations of the
// replicas with `ng` Gaussians (0: any count, read at run time; 9: FP64 with
// the polynomial Gaussian sums)
hipError_t launch_nlist_batch(const NearArgs *tab, const EnsItem *items, int n, hipStream_t st);
hipError_t launch_near_batch(const NearArgs *tab, const EnsItem *items, int n, int ng, bool mixed, bool energy,
                             hipStream_t st);
// Particles per structure-factor partial for a system of N particles and P samples.
int rho_chunk(int N, int P);
// The same when the partials run in the near launch's first workgroups (>= rho_chunk).
int rho_chunk_shared(int N, int P, bool mixed);
hipError_t launch_near(const NearArgs &a, hipStream_t st);

// --- far field + assembly + second half-kick ---------------------------------------
struct FarArgs {
    int N, P;
    double two_pi_over_L[3], inv_L[3];
    const double4 *xs;         // cell order
    const int32_t *order;
    const double4 *samp;       // [P] (nx, ny, nz, coef)
    const double2 *gk;         // [P] coef * rho
    const double *fnear;       // [kNearLanes][3][N] partial near forces of the lanes, cell order
    double *f;                 // null, or SoA [3][N] forces in caller order (through order)
    double *f_near_out;        // null, or SoA [3][N] near forces in caller order
    double *fs;                // null, or SoA [3][N] forces in cell order
    double *vs;                // null, or SoA [3][N] cell-order velocities to kick
    const double *ms;          // [N] cell-order masses (when vs)
    double half_dt;
    double *kepart;            // [far_blocks(N)] kinetic-energy partials (when vs)
    int *flag;                 // set to 1 on a non-finite force
    int mixed;
    const double2 *tab;        // [kFarTab] (sin, cos)(2 pi j / kFarTab) (FP64 path)
    SinCosFar ss;
    int32_t *gate_clear;       // null, or a rebuild gate to clear (nothing later in the step reads it)
    int32_t *rebuilds;         // null, or a count of the steps whose gate was raised (with gate_clear)
    // With drift != 0 the kernel also applies the next step's first half-kick
    // and drift to the cell-order rows (the drift kernel's arithmetic, fused;
    // single systems only, the ensemble's far kernel ignores it):
    // xs_next = xs (written back), gate_raise raised when a particle has moved
    // more than half the skin since the build.
    int drift;
    double dt, L[3], half_skin2;
    const double *xb;          // SoA [3][N] positions at the last build, cell order
    double4 *xs_next;
    int32_t *gate_raise;
    Thermo th;                 // the drift's thermostat (single systems)
};
hipError_t launch_far(const FarArgs &a, hipStream_t st);
// ensemble: far_blocks items per replica
hipError_t launch_far_batch(const FarArgs *tab, const EnsItem *items, int n, bool mixed, hipStream_t st);

// --- energies ---------------------------------------------------------------
// An energy row: U_N, U*_F, U_k0, U_self, U_bg, KE, W_N, W*_F.
constexpr int kEnergyCols = 8;
struct EnergyArgs {
    int nnear, nfar, P;
    const double *epart;       // [2][nnear]: energy, then virial partials
    const double *kepart;      // [nfar] or null
    const double *eF;          // [P]
    const double *eW;          // [P]
    double Uk0, Uself, Ubg;
    double *out;               // [rows][kEnergyCols]; one system writes row row0
    uint64_t row0;
    const double *ke_set;      // null, or the kinetic energy to report (a global bath's, after its half-step)
};
hipError_t launch_energy(const EnergyArgs &a, hipStream_t st);
// ensemble: one item per replica; each writes row *shift + row0 of its out
hipError_t launch_energy_batch(const EnergyArgs *tab, const EnsItem *items, int n, const uint64_t *shift,
                               hipStream_t st);


// --- global baths (Nose-Hoover, Berendsen) ------------------------------------
// The bath state lives on the device: kBathWords doubles, [0] xi, [1] eta (the
// Nose-Hoover friction and its time integral), [2] the factor the velocities
// take next, [3] the kinetic energy after the last closing half-step.
constexpr int kBathWords = 8;
constexpr int kBathNoseHoover = 2, kBathBerendsen = 3;
struct BathArgs {
    int kind;                  // kBathNoseHoover or kBathBerendsen
    int mode;                  // 1: opening half-step; 2: closing; 3: closing then opening
    double dt, gkT, Q, rate;   // g k_B T with g = 3N; Nose-Hoover mass g kT tau^2; 1/tau
    int nfar;
    const double *kepart;      // [nfar] kinetic-energy partials of the current velocities
    double *bath;              // [kBathWords]
};
hipError_t launch_bath(const BathArgs &a, hipStream_t st);
// kinetic-energy partials of vs (cell order) in the far kernel's blocks
hipError_t launch_ke_partials(int N, const double *vs, const double *ms, double *kepart, hipStream_t st);
// vs *= *scale
hipError_t launch_scale_v(int N, double *vs, const double *scale, hipStream_t st);


}  // namespace rbsog

// The single-system state of librbsog behind the opaque rbsog_handle, and the
// host helpers that size, describe and launch it.  Shared by the C-ABI of one
// system and the served ensemble; nothing here is part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

#include "internal.h"
#include "launch.h"

namespace rbsog {

constexpr double kPi = 3.141592653589793;
constexpr size_t kAlign = 256;

#define HIPCHECK(call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail(RBSOG_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Offsets of every buffer inside the workspace.
struct Layout {
    size_t lattice, cdf, coef, first, size;
    size_t cell_id, count, cell_start, fill, tmp, order, order_old, xs, xs_old, tile_sum, xb, vs, vs_old, fs, ms, ms_old;
    size_t samp, part, rho, gk, eF, eW, vm, fnear, epart, kepart, flag, energy, nbr, nbr_cnt, tab, tab_far;
    size_t cdf_q, mh;   // Metropolis-Hastings draws: proposal CDF, chain state
    size_t bath;        // global bath state (kBathWords doubles)
    size_t fab;         // the decomposition's Fourier coefficients A, B (cuboid virial factors)
    size_t total;
};

// Sizes derived from the parameters, shared by rbsog_workspace_size and
// rbsog_create.  Two cell grids: the coarse one (cells >= r_c), which is the
// cell list of rbsog_build_cells, and the fine one of the force evaluation
// (cells >= (r_c + skin)/2, a 5 x 5 x 5 stencil).
struct Derived {
    double skin, rl;   // neighbour-list skin and radius r_c + skin
    double Lb[3];      // box edges (equal in a cube)
    int cuboid;        // edges differ: the measure point by point (each lattice point its own shell)
    int nc[3], nf[3];  // coarse and fine cells per axis
    int nf_tight[3];   // fine cells per axis of lists of radius r_c alone (the grid a dropped skin uses; >= nf)
    int mmax;          // cube: lattice 1 <= |n|^2 <= mmax; cuboid: 0
    int64_t nlat;
    int64_t nshells;   // capacity of the per-shell tables: mmax (cube) or nlat (cuboid)
    int kp;            // neighbour-list capacity per (particle, chunk)
    int sbatch;        // steps whose modes one sampling launch draws
    int full_k;        // deterministic far field over the whole lattice
    int64_t nmodes;    // modes of one evaluation: P, or nlat with full_k
};

size_t align_up(size_t v);
int nchunks(int64_t N, int P);
CellGeom make_geom(const double Lb[3], const int nc[3]);
// the box edges of the parameters (Ly, Lz of 0 take L)
void box_edges(const rbsog_params *p, double Lb[3]);
// kp of a system of N particles in volume V for lists of radius rl
int near_capacity(int64_t N, double V, double rl);
Derived derive(const rbsog_params *p, const rbsog_sog *s);
// shared_lattice: the packed lattice lives outside the workspace
Layout make_layout(int64_t N, const Derived &d, int P, bool shared_lattice);
int check_params(const rbsog_params *p, const rbsog_sog *s);

}  // namespace rbsog

struct rbsog_handle {
    using Derived = rbsog::Derived;
    using CellGeom = rbsog::CellGeom;
    using Layout = rbsog::Layout;
    using SogDev = rbsog::SogDev;
    rbsog_params p;
    rbsog_sog sog;
    const double *q, *m;
    hipStream_t st;
    Derived d;
    CellGeom g;   // coarse grid (rbsog_build_cells)
    CellGeom gf;  // fine grid (force evaluation)
    int nshell;
    double S, V, Q1, Q2, Uk0, Uself, Ubg;
    Layout lay;
    char *ws;
    SogDev sd;
    // views into the workspace
    int32_t *lattice, *first, *size, *cell_id, *count, *cell_start, *fill, *tmp, *order, *order_old, *flag, *tile_sum;
    double *cdf, *coef, *eF, *eW, *vm, *fnear, *epart, *kepart, *energy, *xb;
    double *vs, *vs_old, *fs, *ms, *ms_old;   // the stepped state in cell order (with xs)
    double4 *xs, *xs_old, *samp;
    double2 *part, *rho, *gk, *tab, *tab_far;
    int32_t *nbr, *nbr_cnt;
    int32_t *gate;       // device, two words: rebuild the cell order and lists in this step
                         // (steps alternate between them; each step clears the other)
    int32_t *ticket;     // device: the scan's finished-tile counter
    int phase;           // which gate word the next step uses
    bool lists_valid;    // cell order and lists in the workspace belong to the fine grid
    double m_min;        // lightest mass (host copy, for the default skin's thermal check)
    bool skin_default;   // the skin is the library's default (only a default skin adapts)
    double dt_checked;   // largest time step the default skin has been checked against
    int32_t *rebuilds;   // device: steps of rbsog_step whose lists were rebuilt (since creation)
    int32_t *rb_host;    // pinned host copy of it, read back after each rbsog_step
    hipEvent_t rb_ev;    // completes when rb_host holds the count of rb_steps steps
    bool rb_pending;
    int64_t rb_steps, steps_done;
    uint64_t samp_step;  // first step of the modes in samp, with samp_n steps drawn
    int samp_n;
    // Metropolis-Hastings draws (p.sampler == 1): the proposal CDF (F = 1) and
    // its total, and the chain state (lattice index, shell index; -1 empty)
    double *fab = nullptr;   // [2][kMaxGauss] A then B
    double *cdf_q = nullptr;
    double Sq = 0.0;
    int32_t *mh = nullptr;
    // rbsog_set_kT: pinned staging of the re-derived cdf and coef ([2][nshell]),
    // free again once kt_ev has completed
    double *kt_host = nullptr;
    hipEvent_t kt_ev = nullptr;
    // Langevin thermostat of rbsog_step (rbsog_set_thermostat; friction 0: off)
    double friction = 0.0, bath_kT = 0.0;
    // global bath of rbsog_step (rbsog_set_bath: Nose-Hoover or Berendsen;
    // 0: none), its rate 1/tau and device state
    int bath_kind = 0;
    double bath_rate = 0.0;
    double *bath = nullptr;
    // per-kernel event timing (rbsog_timing_enable)
    bool timing = false;
    std::vector<hipEvent_t> events;
    std::vector<std::pair<int, int>> records;  // (kernel class, index of the start event)
    int used = 0;
    double timing_ms[RBSOG_NUM_KERNEL_CLASSES] = {};
    int64_t launches[RBSOG_NUM_KERNEL_CLASSES] = {};
};

namespace rbsog {


hipError_t harvest(rbsog_handle *h);

// Runs one launcher; when timing is on, brackets it with events on the stream.
template <class F>
hipError_t timed(rbsog_handle *h, int cls, F &&launch)
{
    if (!h->timing) return launch();
    if (h->used + 2 > (int)h->events.size()) {
        hipError_t e = harvest(h);
        if (e != hipSuccess) return e;
    }
    int s = h->used;
    hipError_t e = hipEventRecord(h->events[s], h->st);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(h->events[s + 1], h->st);
    if (e != hipSuccess) return e;
    h->records.emplace_back(cls, s);
    h->used += 2;
    return hipSuccess;
}

// a build of grid g; carry_v: velocities are live and move with their rows
CellArgs cell_args(rbsog_handle *h, const CellGeom &g, const int32_t *gate, bool carry_v);
// caller arrays -> cell order (v, f may be null) and back
PermArgs perm_args(rbsog_handle *h, double *x, double *v, double *f);
NearArgs near_args(rbsog_handle *h, const int32_t *gate, bool energy);
SampleArgs sample_args(rbsog_handle *h, uint64_t step, int nstep);
RhoArgs rho_args(rbsog_handle *h, const double4 *samp);
// f, f_near: caller-order outputs (may be null); kick: write the cell-order
// forces and apply the second half-kick to the cell-order velocities
FarArgs far_args(rbsog_handle *h, const double4 *samp, double *f, double *f_near, bool kick, double dt);
EnergyArgs energy_args(rbsog_handle *h, double *out, bool kick);
// cell order + lists of the fine grid from the rows in xs (gated or not)
int prepare(rbsog_handle *h, const int32_t *gate, bool carry_v);
// The default skin against the time step dt: when the fastest thermal velocity
// component would carry a particle across skin/2 within two steps, the skin
// drops to 0 and the fine grid and list capacity are re-derived for lists of
// r_c alone (inside the same workspace; the next build is forced).  Checked
// again whenever dt exceeds every earlier dt; returns true when it dropped.
bool adapt_skin(rbsog_handle *h, double dt);
// The same drop when the lists of the last rbsog_step calls were rebuilt at
// more than half their steps (read back without waiting; checked when the
// count of a previous call has arrived).
bool adapt_skin_rebuilds(rbsog_handle *h);
// rbsog_create; with lattice_dev (the packed lattice up to at least the
// system's m_max, owned by the caller) the workspace holds no lattice copy
// q_host, m_host (nullable): host copies of the charges and masses, which
// spare the read-back of q_dev and m_dev; with sync false nothing waits on the
// stream (the table uploads complete in stream order).
int create_system(const rbsog_params *p, const rbsog_sog *s, const double *q_dev, const double *m_dev, void *ws_dev,
                  size_t ws_bytes, hipStream_t stream, const int32_t *lattice_dev, rbsog_handle **out,
                  const double *q_host = nullptr, const double *m_host = nullptr, bool sync = true);
// gate_raise non-null (with kick): the far kernel also applies the next
// step's first half-kick and drift, raising gate_raise; gate_clear is cleared
// the thermostat of a step's drift into force index `step` (off without friction)
Thermo thermo(const rbsog_handle *h, double dt, uint64_t step);
// with gate_raise the far kernel also drifts into force index next_step
int evaluate(rbsog_handle *h, const double4 *samp, double *f, double *f_near, bool kick, double dt, double *energy,
             int32_t *gate_raise = nullptr, int32_t *gate_clear = nullptr, uint64_t next_step = 0,
             int bath_mode = 0);

}  // namespace rbsog

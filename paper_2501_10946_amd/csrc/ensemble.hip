// Served ensemble of librbsog (rbsog_ens_*, declared in include/rbsog.h).
//
// Many independent systems ("replicas") are resident at once inside one
// device pool and advance together: one ensemble step is a single launch of
// each step kernel over a work list of (replica, workgroup) items covering
// every active replica, so the launch count per step does not grow with the
// number of replicas and small systems share the chip instead of each leaving
// it idle.  A replica's argument blocks sit in device tables; the only value
// that changes from step to step is the ensemble step counter, passed as a
// kernel argument, from which each replica derives its own force-evaluation
// index (sampling) and energy row.  The host touches the work lists only when
// the resident set changes (admission, completion).
//
// Per replica, one step is the step of one system (rbsog_step): half-kick +
// drift with the rebuild test, gated cell build and neighbour lists, mode
// draws, structure factors, near field, far field + second half-kick, and the
// energy terms of the new force written to the replica's energy history.  The
// rebuild gate is raised by the drift and cleared by the far-field kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "system.h"

namespace rbsog {
namespace {

// First-fit allocator over the byte range of the pool (kAlign granules).
class Pool {
   public:
    void init(size_t bytes)
    {
        free_.clear();
        if (bytes) free_[0] = bytes;
        total_ = bytes;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            size_t o = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[o + bytes] = rest;
            *off = o;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t free_bytes() const
    {
        size_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }

   private:
    std::map<size_t, size_t> free_;
    size_t total_ = 0;
};

struct Replica {
    bool used = false;      // slot holds a replica (active or finished, not retired)
    bool active = false;    // still stepping
    bool reported = false;  // completion returned by rbsog_ens_poll
    rbsog_handle *h = nullptr;
    size_t off = 0, bytes = 0;
    double *x = nullptr, *v = nullptr, *f = nullptr, *q = nullptr, *m = nullptr, *ehist = nullptr;
    int64_t N = 0;
    int P = 0, ng = 0, nsteps = 0;
    bool mixed = false;
    uint64_t e_adm = 0;   // ensemble steps launched before the replica's first
    uint64_t e_done = 0;  // ensemble step count after its last step
};

constexpr int kEnsEvents = 8192;  // completion events kept (ring)
constexpr int kGroups = 10;       // near-field groups: Gaussian count (0: run-time count), 9: polynomial sums

// A device array grown on demand (the ensemble's own bookkeeping, outside the pool).
template <class T>
struct DevVec {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t reserve(size_t n)
    {
        if (n <= cap) return hipSuccess;
        size_t c = std::max<size_t>(n, 2 * cap);
        T *q = nullptr;
        hipError_t e = hipMalloc((void **)&q, sizeof(T) * c);
        if (e != hipSuccess) return e;
        if (p) (void)hipFree(p);
        p = q;
        cap = c;
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

}  // namespace
}  // namespace rbsog

using namespace rbsog;

struct rbsog_ens {
    hipStream_t st = nullptr;
    size_t budget = 0;
    char *pool = nullptr;
    Pool alloc;
    int max_slots = 0;
    std::vector<Replica> rep;
    // argument tables, one entry per slot
    KickDriftArgs *t_kick = nullptr;
    CellArgs *t_cell = nullptr;
    NearArgs *t_nlist = nullptr, *t_near = nullptr;
    SampleArgs *t_samp = nullptr;
    RhoArgs *t_rho = nullptr;
    FarArgs *t_far = nullptr;
    EnergyArgs *t_energy = nullptr;
    // work lists: one device buffer, offsets and counts per list
    DevVec<EnsItem> items;
    enum { L256, LTILE, LNLIST, LSAMP, LENERGY, LRHO0, LRHO1, LRED0, LRED1, LFAR0, LFAR1, LNEAR0, LNEAR1 = LNEAR0 + kGroups,
           NLISTS = LNEAR1 + kGroups };
    size_t off[NLISTS] = {};
    int cnt[NLISTS] = {};
    size_t rho_lds[2] = {};
    int nactive = 0;
    bool dirty = false;
    uint64_t E = 0;  // ensemble steps launched
    uint64_t *E_dev = nullptr;  // the same counter on the device, advanced by the step itself
    // the step as a HIP graph, captured once per resident set and replayed
    bool use_graph = true;
    hipStream_t cap = nullptr;
    // admissions upload on a stream of their own (default priority) and wait
    // for those copies alone, not for the steps in flight on st
    hipStream_t up = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the packed Fourier lattice shared by every replica (a prefix serves any
    // smaller m_max), outside the pool
    int32_t *lat = nullptr;
    int lat_mmax = 0;
    hipEvent_t ev0 = nullptr;
    std::vector<hipEvent_t> ev;
};

namespace {

int ens_fail_hip(hipError_t e, const char *what) { return fail(RBSOG_EHIP, "%s: %s", what, hipGetErrorString(e)); }

// The last node of a step: the device's ensemble step counter moves on.
__global__ void k_ens_advance(uint64_t *E)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) E[0] = E[0] + 1;
}

void drop_graph(rbsog_ens *s)
{
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->exec = nullptr;
    s->graph = nullptr;
}

// Rebuilds and uploads the work lists of the active replicas (largest first,
// so the longest workgroups start early).
int rebuild_lists(rbsog_ens *s)
{
    std::vector<int> order;
    for (int r = 0; r < s->max_slots; ++r)
        if (s->rep[r].active) order.push_back(r);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return s->rep[a].N > s->rep[b].N; });
    std::vector<std::vector<EnsItem>> L(rbsog_ens::NLISTS);
    size_t lds[2] = {0, 0};
    for (int r : order) {
        const Replica &R = s->rep[r];
        const rbsog_handle *h = R.h;
        const int N = (int)R.N, pr = R.mixed ? 1 : 0;
        auto add = [&](int list, int64_t n) {
            for (int64_t b = 0; b < n; ++b) L[list].push_back(EnsItem{r, (int32_t)b});
        };
        add(rbsog_ens::L256, (N + kBlock - 1) / kBlock);
        add(rbsog_ens::LTILE, scan_tiles(h->gf.ncell));
        add(rbsog_ens::LNLIST, nlist_blocks(h->gf.nc));
        add(rbsog_ens::LSAMP, (R.P + 63) / 64);
        add(rbsog_ens::LENERGY, 1);
        const int chunk = rho_chunk_shared(N, R.P, R.mixed), nch = (N + chunk - 1) / chunk;   // as rho_args
        add(rbsog_ens::LRHO0 + pr, rho_blocks(nch, R.P));
        add(rbsog_ens::LRED0 + pr, rho_reduce_blocks(R.P));
        add(rbsog_ens::LFAR0 + pr, far_blocks(N));
        add((pr ? rbsog_ens::LNEAR1 : rbsog_ens::LNEAR0) + R.ng, near_blocks(N));
        lds[pr] = std::max(lds[pr], rho_lds_bytes(R.P, chunk, pr == 1, true));
    }
    size_t total = 0;
    for (int k = 0; k < rbsog_ens::NLISTS; ++k) {
        s->off[k] = total;
        s->cnt[k] = (int)L[k].size();
        total += L[k].size();
    }
    std::vector<EnsItem> flat;
    flat.reserve(total);
    for (auto &l : L) flat.insert(flat.end(), l.begin(), l.end());
    s->rho_lds[0] = lds[0];
    s->rho_lds[1] = lds[1];
    s->dirty = false;
    drop_graph(s);
    if (total == 0) return RBSOG_OK;
    // the previous lists may still be read by launched kernels: let them finish
    hipError_t e = hipStreamSynchronize(s->st);
    if (e == hipSuccess) e = s->items.reserve(total);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->items.p, flat.data(), sizeof(EnsItem) * total, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return ens_fail_hip(e, "uploading work lists");
    return RBSOG_OK;
}

template <class T>
hipError_t put(T *table, int slot, const T &v, hipStream_t st)
{
    hipError_t e = hipMemcpyAsync(table + slot, &v, sizeof(T), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

// Pool bytes of one replica: its workspace (without the lattice), x, v, f,
// q, m and the energy history.
size_t replica_bytes(const rbsog_params *p, const rbsog_sog *sog, int nsteps)
{
    const size_t N = (size_t)p->N;
    const size_t ws = make_layout(p->N, derive(p, sog), p->P, true).total;
    return align_up(ws) + align_up(sizeof(double) * 3 * N) * 3 + align_up(sizeof(double) * N) * 2 +
           align_up(sizeof(double) * kEnergyCols * (size_t)nsteps);
}

// Argument blocks of slot r (the replica was admitted with e_adm steps launched).
int write_tables(rbsog_ens *s, int r, double dt)
{
    Replica &R = s->rep[r];
    rbsog_handle *h = R.h;
    hipError_t e;
    KickDriftArgs k{};
    k.N = (int)R.N;
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
    k.gate = h->gate;
    k.gate_next = nullptr;
    k.flag = h->flag;
    if ((e = put(s->t_kick, r, k, s->up)) != hipSuccess) return ens_fail_hip(e, "kick table");
    CellArgs c = cell_args(h, h->gf, h->gate, true);
    if ((e = put(s->t_cell, r, c, s->up)) != hipSuccess) return ens_fail_hip(e, "cell table");
    NearArgs nl = near_args(h, h->gate, false);
    if ((e = put(s->t_nlist, r, nl, s->up)) != hipSuccess) return ens_fail_hip(e, "list table");
    // modes of force index E + 1 - e_adm at ensemble step E (unsigned wrap)
    SampleArgs sa = sample_args(h, (uint64_t)1 - R.e_adm, 1);
    if ((e = put(s->t_samp, r, sa, s->up)) != hipSuccess) return ens_fail_hip(e, "sample table");
    RhoArgs ra = rho_args(h, h->samp);
    if ((e = put(s->t_rho, r, ra, s->up)) != hipSuccess) return ens_fail_hip(e, "rho table");
    NearArgs na = near_args(h, nullptr, true);
    if ((e = put(s->t_near, r, na, s->up)) != hipSuccess) return ens_fail_hip(e, "near table");
    FarArgs fa = far_args(h, h->samp, nullptr, nullptr, true, dt);
    fa.gate_clear = h->gate;
    if ((e = put(s->t_far, r, fa, s->up)) != hipSuccess) return ens_fail_hip(e, "far table");
    // energies of step E - e_adm go to row E - e_adm
    EnergyArgs ea = energy_args(h, R.ehist, true);
    ea.row0 = (uint64_t)0 - R.e_adm;
    if ((e = put(s->t_energy, r, ea, s->up)) != hipSuccess) return ens_fail_hip(e, "energy table");
    return RBSOG_OK;
}

// Makes the shared lattice cover m_max, re-pointing the resident replicas'
// sampling tables when it moves.
int ensure_lattice(rbsog_ens *s, int mmax)
{
    if (mmax <= s->lat_mmax) return RBSOG_OK;
    int64_t n = lattice_points(mmax);
    std::vector<int32_t> host((size_t)n);
    lattice_copy(mmax, host.data());
    int32_t *dev = nullptr;
    hipError_t e = hipStreamSynchronize(s->st);   // nothing may still read the old table
    if (e == hipSuccess) e = hipMalloc((void **)&dev, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(dev, host.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        if (dev) (void)hipFree(dev);
        return ens_fail_hip(e, "uploading the lattice");
    }
    for (int r = 0; r < s->max_slots; ++r) {
        Replica &R = s->rep[r];
        if (!R.used || !R.h) continue;
        R.h->lattice = dev;
        SampleArgs sa = sample_args(R.h, (uint64_t)1 - R.e_adm, 1);
        if ((e = put(s->t_samp, r, sa, s->up)) != hipSuccess) {
            (void)hipFree(dev);
            return ens_fail_hip(e, "sample table");
        }
    }
    if (s->lat) (void)hipFree(s->lat);
    s->lat = dev;
    s->lat_mmax = mmax;
    return RBSOG_OK;
}

void drop_replica(rbsog_ens *s, int r)
{
    Replica &R = s->rep[r];
    if (R.h) rbsog_destroy(R.h);
    if (R.bytes) s->alloc.release(R.off, R.bytes);
    R = Replica{};
}

}  // namespace

extern "C" int rbsog_ens_create(size_t hbm_budget, int max_slots, void *hip_stream, rbsog_ens **out)
{
    if (!out) return fail(RBSOG_EINVAL, "out is null");
    if (max_slots < 1 || max_slots > 65536) return fail(RBSOG_EINVAL, "max_slots must lie in [1, 65536]");
    if (hbm_budget < kAlign) return fail(RBSOG_EINVAL, "hbm_budget below %zu bytes", kAlign);
    rbsog_ens *s = new (std::nothrow) rbsog_ens{};
    if (!s) return fail(RBSOG_ENOMEM, "ensemble allocation");
    s->st = (hipStream_t)hip_stream;
    s->budget = hbm_budget / kAlign * kAlign;
    s->max_slots = max_slots;
    s->rep.resize(max_slots);
    hipError_t e = hipMalloc((void **)&s->pool, s->budget);
    size_t n = (size_t)max_slots;
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_kick, sizeof(KickDriftArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_cell, sizeof(CellArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_nlist, sizeof(NearArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_near, sizeof(NearArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_samp, sizeof(SampleArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_rho, sizeof(RhoArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_far, sizeof(FarArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->t_energy, sizeof(EnergyArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&s->E_dev, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemsetAsync(s->E_dev, 0, sizeof(uint64_t), s->st);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->up, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->ev0);
    if (e == hipSuccess) {
        s->ev.resize(kEnsEvents, nullptr);
        for (auto &x : s->ev)
            if (e == hipSuccess) e = hipEventCreate(&x);
    }
    if (e == hipSuccess) e = hipEventRecord(s->ev0, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) {
        rbsog_ens_destroy(s);
        return ens_fail_hip(e, "creating the ensemble");
    }
    s->alloc.init(s->budget);
    if (const char *g = std::getenv("RBSOG_ENS_GRAPH"))   // 0: launch the kernels one by one each step
        s->use_graph = std::atoi(g) != 0;
    *out = s;
    return RBSOG_OK;
}

extern "C" int rbsog_ens_bytes(const rbsog_params *p, const rbsog_sog *sog, int nsteps, size_t *bytes)
{
    if (!bytes) return fail(RBSOG_EINVAL, "bytes is null");
    if (nsteps < 1) return fail(RBSOG_EINVAL, "nsteps must be >= 1");
    int rc = check_params(p, sog);
    if (rc) return rc;
    *bytes = replica_bytes(p, sog, nsteps);
    return RBSOG_OK;
}

extern "C" int rbsog_ens_admit(rbsog_ens *s, const rbsog_params *p, const rbsog_sog *sog, const double *x_host,
                               const double *v_host, const double *q_host, const double *m_host, int nsteps, double dt,
                               int *slot_out)
{
    if (!s || !x_host || !v_host || !q_host || !m_host || !slot_out) return fail(RBSOG_EINVAL, "null argument");
    if (nsteps < 1) return fail(RBSOG_EINVAL, "nsteps must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBSOG_EINVAL, "dt must be positive and finite");
    int rc = check_params(p, sog);
    if (rc) return rc;
    if (p->full_k) return fail(RBSOG_EINVAL, "the ensemble serves random-batch replicas only (full_k = 0)");
    if (p->sampler != RBSOG_SAMPLER_IID)
        return fail(RBSOG_EINVAL, "the ensemble draws i.i.d. modes only (sampler = RBSOG_SAMPLER_IID)");
    if ((p->Ly > 0.0 && p->Ly != p->L) || (p->Lz > 0.0 && p->Lz != p->L))
        return fail(RBSOG_EINVAL, "the ensemble serves cubic boxes only (Ly, Lz of 0 or equal to L)");
    int slot = -1;
    for (int r = 0; r < s->max_slots; ++r)
        if (!s->rep[r].used) {
            slot = r;
            break;
        }
    if (slot < 0) return fail(RBSOG_EAGAIN, "no free slot (%d resident)", s->max_slots);
    const Derived d = derive(p, sog);
    rc = ensure_lattice(s, d.mmax);
    if (rc) return rc;
    const size_t ws = make_layout(p->N, d, p->P, true).total;
    const size_t N = (size_t)p->N;
    size_t bytes = replica_bytes(p, sog, nsteps), off = 0;
    if (!s->alloc.alloc(bytes, &off))
        return fail(RBSOG_EAGAIN, "pool has no %zu contiguous bytes (%zu free)", bytes, s->alloc.free_bytes());
    Replica &R = s->rep[slot];
    R = Replica{};
    R.used = true;
    R.off = off;
    R.bytes = bytes;
    char *b = s->pool + off;
    char *wsp = b;
    b += align_up(ws);
    auto take = [&](size_t nbytes) {
        char *o = b;
        b += align_up(nbytes);
        return (double *)o;
    };
    R.x = take(sizeof(double) * 3 * N);
    R.v = take(sizeof(double) * 3 * N);
    R.f = take(sizeof(double) * 3 * N);
    R.q = take(sizeof(double) * N);
    R.m = take(sizeof(double) * N);
    R.ehist = take(sizeof(double) * kEnergyCols * (size_t)nsteps);
    R.N = p->N;
    R.P = p->P;
    R.ng = sog->n <= 8 ? sog->n : 0;
    R.mixed = p->precision == RBSOG_MIXED;
    R.nsteps = nsteps;
    // the state and the system's tables go up on the upload stream, which is
    // then waited for (the copies only); the replica's kernels follow on st
    hipError_t e = hipMemcpyAsync(R.x, x_host, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipMemcpyAsync(R.v, v_host, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipMemcpyAsync(R.q, q_host, sizeof(double) * N, hipMemcpyHostToDevice, s->up);
    if (e == hipSuccess) e = hipMemcpyAsync(R.m, m_host, sizeof(double) * N, hipMemcpyHostToDevice, s->up);
    if (e != hipSuccess) {
        drop_replica(s, slot);
        return ens_fail_hip(e, "uploading the replica");
    }
    rc = create_system(p, sog, R.q, R.m, wsp, align_up(ws), s->up, s->lat, &R.h, q_host, m_host, true);
    if (rc) {
        drop_replica(s, slot);
        return rc;
    }
    R.h->st = s->st;
    // the force of the initial state, evaluation index 0, then the state in
    // cell order, where the steps keep it until retirement
    rc = rbsog_compute_forces(R.h, 0, R.x, R.f, nullptr, nullptr);
    if (rc == RBSOG_OK) {
        PermArgs in = perm_args(R.h, R.x, R.v, R.f);
        hipError_t le = launch_state_in(in, s->st);
        if (le != hipSuccess) rc = ens_fail_hip(le, "moving the replica into cell order");
    }
    if (rc) {
        drop_replica(s, slot);
        return rc;
    }
    // the default skin meets the time step here, as at a system's first
    // rbsog_step: a hot replica drops it (and so rebuilds at its first step,
    // like the system stepped alone), so that both take the same steps
    if (adapt_skin(R.h, dt)) {
        hipError_t le = launch_set_int(R.h->gate, 1, s->st);
        if (le != hipSuccess) {
            drop_replica(s, slot);
            return ens_fail_hip(le, "raising the replica's rebuild gate");
        }
    }
    R.h->samp_n = 0;
    if (!R.mixed && R.h->sd.poly) R.ng = 9;
    R.e_adm = s->E;
    rc = write_tables(s, slot, dt);
    if (rc) {
        drop_replica(s, slot);
        return rc;
    }
    R.active = true;
    s->nactive += 1;
    s->dirty = true;
    *slot_out = slot;
    return RBSOG_OK;
}

namespace {

// One ensemble step of every active replica, enqueued on st.
hipError_t enqueue_step(rbsog_ens *s, hipStream_t st)
{
    const EnsItem *it = s->items.p;
    auto list = [&](int k) { return it + s->off[k]; };
    hipError_t e = launch_kick_drift_batch(s->t_kick, list(rbsog_ens::L256), s->cnt[rbsog_ens::L256], st);
    if (e == hipSuccess)
        e = launch_cell_build_batch(s->t_cell, list(rbsog_ens::L256), s->cnt[rbsog_ens::L256], list(rbsog_ens::LTILE),
                                    s->cnt[rbsog_ens::LTILE], st);
    if (e == hipSuccess) e = launch_nlist_batch(s->t_nlist, list(rbsog_ens::LNLIST), s->cnt[rbsog_ens::LNLIST], st);
    if (e == hipSuccess)
        e = launch_sample_batch(s->t_samp, list(rbsog_ens::LSAMP), s->cnt[rbsog_ens::LSAMP], s->E_dev, st);
    for (int pr = 0; pr < 2 && e == hipSuccess; ++pr)
        if (s->cnt[rbsog_ens::LRHO0 + pr] > 0)
            e = launch_rho_batch(s->t_rho, list(rbsog_ens::LRHO0 + pr), s->cnt[rbsog_ens::LRHO0 + pr], s->rho_lds[pr],
                                 pr == 1, list(rbsog_ens::LRED0 + pr), s->cnt[rbsog_ens::LRED0 + pr], st);
    for (int pr = 0; pr < 2 && e == hipSuccess; ++pr)
        for (int g = 0; g < kGroups && e == hipSuccess; ++g) {
            int k = (pr ? rbsog_ens::LNEAR1 : rbsog_ens::LNEAR0) + g;
            if (s->cnt[k] > 0) e = launch_near_batch(s->t_near, list(k), s->cnt[k], g, pr == 1, true, st);
        }
    for (int pr = 0; pr < 2 && e == hipSuccess; ++pr)
        if (s->cnt[rbsog_ens::LFAR0 + pr] > 0)
            e = launch_far_batch(s->t_far, list(rbsog_ens::LFAR0 + pr), s->cnt[rbsog_ens::LFAR0 + pr], pr == 1, st);
    if (e == hipSuccess)
        e = launch_energy_batch(s->t_energy, list(rbsog_ens::LENERGY), s->cnt[rbsog_ens::LENERGY], s->E_dev, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_ens_advance, dim3(1), dim3(64), 0, st, s->E_dev);
        e = hipGetLastError();
    }
    return e;
}

// Captures the step into a graph (the launch sequence only: kernel nodes, no
// memory operations) on the ensemble's own capture stream.
hipError_t capture_step(rbsog_ens *s)
{
    hipError_t e = hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = enqueue_step(s, s->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s->cap, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    s->graph = g;
    e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) drop_graph(s);
    return e;
}

}  // namespace

extern "C" int rbsog_ens_step(rbsog_ens *s)
{
    if (!s) return fail(RBSOG_EINVAL, "null ensemble");
    if (s->dirty) {
        int rc = rebuild_lists(s);
        if (rc) return rc;
    }
    if (s->nactive == 0) return RBSOG_OK;
    if (s->use_graph) {
        if (!s->exec) HIPCHECK(capture_step(s));
        HIPCHECK(hipGraphLaunch(s->exec, s->st));
    } else {
        HIPCHECK(enqueue_step(s, s->st));
    }
    s->E += 1;
    HIPCHECK(hipEventRecord(s->ev[s->E % kEnsEvents], s->st));
    for (int r = 0; r < s->max_slots; ++r) {
        Replica &R = s->rep[r];
        if (R.active && s->E - R.e_adm >= (uint64_t)R.nsteps) {
            R.active = false;
            R.e_done = s->E;
            s->nactive -= 1;
            s->dirty = true;
        }
    }
    return RBSOG_OK;
}

extern "C" int rbsog_ens_poll(rbsog_ens *s, int *done_slots, int *n_done)
{
    if (!s || !done_slots || !n_done) return fail(RBSOG_EINVAL, "null argument");
    int n = 0;
    for (int r = 0; r < s->max_slots; ++r) {
        Replica &R = s->rep[r];
        if (!R.used || R.active || R.reported) continue;
        hipError_t e = hipEventQuery(s->ev[R.e_done % kEnsEvents]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return ens_fail_hip(e, "polling");
        R.reported = true;
        done_slots[n++] = r;
    }
    *n_done = n;
    return RBSOG_OK;
}

extern "C" int rbsog_ens_retire(rbsog_ens *s, int slot, double *x_host, double *v_host, double *energy_hist_host)
{
    if (!s || slot < 0 || slot >= s->max_slots || !s->rep[slot].used) return fail(RBSOG_EINVAL, "no such slot");
    Replica &R = s->rep[slot];
    if (R.active) return fail(RBSOG_EINVAL, "slot %d has steps left", slot);
    const size_t N = (size_t)R.N;
    // the final state back into the caller's order
    PermArgs out = perm_args(R.h, R.x, R.v, nullptr);
    hipError_t e = launch_state_out(out, s->st);
    if (e == hipSuccess && x_host) e = hipMemcpyAsync(x_host, R.x, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess && v_host)
        e = hipMemcpyAsync(v_host, R.v, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess && energy_hist_host)
        e = hipMemcpyAsync(energy_hist_host, R.ehist, sizeof(double) * kEnergyCols * (size_t)R.nsteps, hipMemcpyDeviceToHost,
                           s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return ens_fail_hip(e, "reading the replica back");
    int32_t flag = 0;
    e = hipMemcpy(&flag, R.h->flag, sizeof(int32_t), hipMemcpyDeviceToHost);
    drop_replica(s, slot);
    if (e != hipSuccess) return ens_fail_hip(e, "reading the replica's flag");
    if (flag) return fail(RBSOG_ENONFINITE, "slot %d produced a non-finite force or an over-long step", slot);
    return RBSOG_OK;
}

extern "C" int rbsog_ens_status(const rbsog_ens *s, int *resident, int *active, uint64_t *ens_steps,
                                size_t *pool_free)
{
    if (!s) return fail(RBSOG_EINVAL, "null ensemble");
    int used = 0;
    for (auto &R : s->rep) used += R.used ? 1 : 0;
    if (resident) *resident = used;
    if (active) *active = s->nactive;
    if (ens_steps) *ens_steps = s->E;
    if (pool_free) *pool_free = s->alloc.free_bytes();
    return RBSOG_OK;
}

extern "C" int rbsog_ens_step_time(rbsog_ens *s, uint64_t ens_step, double *ms)
{
    if (!s || !ms) return fail(RBSOG_EINVAL, "null argument");
    if (ens_step < 1 || ens_step > s->E || s->E - ens_step >= (uint64_t)kEnsEvents)
        return fail(RBSOG_EINVAL, "ensemble step %llu is not among the last %d launched", (unsigned long long)ens_step,
                    kEnsEvents);
    hipEvent_t ev = s->ev[ens_step % kEnsEvents];
    HIPCHECK(hipEventSynchronize(ev));
    float t = 0.0f;
    HIPCHECK(hipEventElapsedTime(&t, s->ev0, ev));
    *ms = (double)t;
    return RBSOG_OK;
}

extern "C" void rbsog_ens_destroy(rbsog_ens *s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->st);
    for (int r = 0; r < s->max_slots; ++r)
        if (s->rep[r].h) rbsog_destroy(s->rep[r].h);
    drop_graph(s);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    if (s->up) (void)hipStreamDestroy(s->up);
    s->items.release();
    if (s->lat) (void)hipFree(s->lat);
    if (s->E_dev) (void)hipFree(s->E_dev);
    for (void *p : {(void *)s->t_kick, (void *)s->t_cell, (void *)s->t_nlist, (void *)s->t_near, (void *)s->t_samp,
                    (void *)s->t_rho, (void *)s->t_far, (void *)s->t_energy, (void *)s->pool})
        if (p) (void)hipFree(p);
    for (auto &x : s->ev)
        if (x) (void)hipEventDestroy(x);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    delete s;
}

// gfx950 kernels of librbsog: the cell list (a counting sort with a stable
// rank), the first velocity-Verlet half step, and the moves between the
// caller's particle order and cell order.
//
// Data layout in HBM: the caller's particle arrays are FP64 SoA in the
// caller's order; the library keeps the state it steps in cell order (xs[N]
// = (x, y, z, q) as double4, 32-byte rows, velocities, forces and masses as
// SoA), with order[p] the caller index of cell position p.  Every kernel of a
// step streams these arrays contiguously; the caller's arrays are read once
// when a call starts and written once when it ends.  A build sorts the rows
// by (cell, caller index) and moves them into the new order.
//
// Builds can be gated: every build kernel takes a device flag and returns at
// once when it is zero, so the decision to rebuild (some particle moved more
// than half the list skin) is taken on the device with no host round-trip.
#include <hip/hip_runtime.h>


#include "dev_common.h"

namespace rbsog {

// A build kernel proceeds when it has no gate or its gate is raised.
__device__ inline bool gate_open(const int32_t *gate) { return gate == nullptr || *gate != 0; }

// ---------------------------------------------------------------------------
// cell list: ids + counts, scan, scatter, stable rank + gather
// ---------------------------------------------------------------------------

// Every kernel body takes its argument block and its workgroup index b within
// the system's grid; the single-system kernels pass blockIdx.x, the ensemble
// kernels the (replica, block) item of a work list.

// Wave-aggregated counting: the particles of a wave are consecutive rows of
// the cell order, so runs of neighbouring lanes share a cell.  The first lane
// of each run (live lanes form a prefix of the wave) adds the run's length
// with one atomic, and with want_base its lanes get consecutive slots from
// the value it read back: a quarter of the atomics of one per particle at
// ~4 particles per cell.  The slots within a cell depend on the order the
// atomics land in, as before; the rank pass makes the final order
// independent of them.
__device__ inline int add_runs(int32_t *cnt, int id, bool live, bool want_base)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lv = __builtin_amdgcn_ballot_w64(live);
    const int prev = __shfl_up(id, 1);
    const bool head = live && (lane == 0 || prev != id);
    const uint64_t H = __builtin_amdgcn_ballot_w64(head);
    int base = 0;
    if (head) {
        const uint64_t above = H & ~((2ull << lane) - 1ull);   // (2 << 63) wraps to 0: no head above lane 63
        const int end = above ? __ffsll((long long)above) - 1 : 64 - __clzll((long long)lv);
        if (want_base) base = atomicAdd(&cnt[id], end - lane);
        else atomicAdd(&cnt[id], end - lane);
    }
    if (!want_base) return 0;
    const int start = 63 - __clzll((long long)(H & ((2ull << lane) - 1ull)));   // this lane's run head
    return __shfl(base, start) + (lane - start);
}

// Snapshot of row p for the rank pass and its cell id (stored).
__device__ inline int cell_id_of(const CellArgs &a, int p)
{
    const double4 r = a.xs[p];
    // snapshot of the row: the rank pass reads the old order from here while
    // it writes the new one in place
    a.xs_old[p] = r;
    a.order_old[p] = a.order[p];
    a.ms_old[p] = a.ms[p];
    if (a.vs)
        for (int d = 0; d < 3; ++d) a.vs_old[d * a.N + p] = a.vs[d * a.N + p];
    int cx = cell_coord(r.x, a.g.inv_cell[0], a.g.nc[0]);
    int cy = cell_coord(r.y, a.g.inv_cell[1], a.g.nc[1]);
    int cz = cell_coord(r.z, a.g.inv_cell[2], a.g.nc[2]);
    int id = (cz * a.g.nc[1] + cy) * a.g.nc[0] + cx;
    a.cell_id[p] = id;
    return id;
}

__device__ inline void cell_ids_body(const CellArgs &a, int b)
{
    if (!gate_open(a.gate)) return;
    int p = b * kBlock + threadIdx.x;
    const bool live = p < a.N;
    int id = -1;
    if (live) id = cell_id_of(a, p);
    add_runs(a.count, id, live, false);
}

// Exclusive scan of the cell counts in two passes.

__device__ inline int32_t block_exclusive_scan_256(int32_t v, int32_t *sh, int32_t *total)
{
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int32_t u = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += u;
        __syncthreads();
    }
    int32_t incl = sh[t];
    *total = sh[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// Pass 1: per-tile sums; the last tile to finish (a ticket counter) turns them
// into exclusive tile offsets and resets the ticket.
__device__ inline void scan_tiles_body(const CellArgs &a, int b)
{
    if (!gate_open(a.gate)) return;
    __shared__ int32_t sh[kBlock];
    __shared__ int last;
    const int t = threadIdx.x;
    const int ntiles = scan_tiles(a.g.ncell);
    int base = b * kScanTile + t * kScanPer;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < a.g.ncell) s += a.count[base + k];
    int32_t total;
    block_exclusive_scan_256(s, sh, &total);
    if (t == 0) {
        a.tile_sum[b] = total;
        __threadfence();
        last = atomicAdd(a.ticket, 1) == ntiles - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    // exclusive scan of the tile sums, kBlock at a time
    int32_t run = 0;
    for (int b0 = 0; b0 < ntiles; b0 += kBlock) {
        int32_t v = b0 + t < ntiles ? __atomic_load_n(&a.tile_sum[b0 + t], __ATOMIC_RELAXED) : 0;
        int32_t chunk;
        int32_t ex = block_exclusive_scan_256(v, sh, &chunk);
        if (b0 + t < ntiles) a.tile_sum[b0 + t] = run + ex;
        run += chunk;
    }
    if (t == 0) *a.ticket = 0;
}

// Pass 2: each tile scanned with its offset; also clears the scatter's fill
// counters and the cell counts (ready for the next build).
__device__ inline void scan_apply_body(const CellArgs &a, int b)
{
    if (!gate_open(a.gate)) return;
    __shared__ int32_t sh[kBlock];
    int base = b * kScanTile + threadIdx.x * kScanPer;
    int32_t c[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = (base + k < a.g.ncell) ? a.count[base + k] : 0;
        s += c[k];
    }
    int32_t total;
    int32_t run = block_exclusive_scan_256(s, sh, &total) + a.tile_sum[b];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < a.g.ncell) {
            a.cell_start[base + k] = run;
            a.fill[base + k] = 0;
            a.count[base + k] = 0;
        }
        run += c[k];
    }
    if (b == 0 && threadIdx.x == 0) a.cell_start[a.g.ncell] = a.N;
}

// Unordered placement of the caller indices into each cell's segment.
__device__ inline void scatter_body(const CellArgs &a, int b)
{
    if (!gate_open(a.gate)) return;
    int p = b * kBlock + threadIdx.x;
    const bool live = p < a.N;
    const int c = live ? a.cell_id[p] : -1;
    const int slot = add_runs(a.fill, c, live, true);
    if (live) a.tmp[a.cell_start[c] + slot] = a.order_old[p];
}

// Stable position: a particle's rank within its cell is the number of cell
// members with a smaller caller index, so the new order is that of (cell,
// caller index) whatever order the scatter produced and whatever the old cell
// order was.  Moves the row, its velocity and mass, and records the positions
// of the build.
__device__ inline void rank_body(const CellArgs &a, int b)
{
    if (!gate_open(a.gate)) return;
    int p = b * kBlock + threadIdx.x;
    if (p >= a.N) return;
    int c = a.cell_id[p];
    const int key = a.order_old[p];
    int cb = a.cell_start[c], ce = a.cell_start[c + 1];
    int r = 0;
    for (int k = cb; k < ce; ++k) r += (a.tmp[k] < key);
    const int pn = cb + r;
    const double4 row = a.xs_old[p];
    a.xs[pn] = row;
    a.order[pn] = key;
    a.ms[pn] = a.ms_old[p];
    a.xb[pn] = row.x;
    a.xb[a.N + pn] = row.y;
    a.xb[2 * a.N + pn] = row.z;
    if (a.vs)
        for (int d = 0; d < 3; ++d) a.vs[d * a.N + pn] = a.vs_old[d * a.N + p];
}

RBSOG_KERNELS(cell_ids, CellArgs, kBlock)
RBSOG_KERNELS(scan_tiles, CellArgs, kBlock)
RBSOG_KERNELS(scan_apply, CellArgs, kBlock)
RBSOG_KERNELS(scatter, CellArgs, kBlock)
RBSOG_KERNELS(rank, CellArgs, kBlock)

static bool cell_args_ok(const CellArgs &a)
{
    return a.N >= 1 && a.g.nc[0] >= 1 && a.g.nc[1] >= 1 && a.g.nc[2] >= 1 && a.xs && a.order && a.xs_old && a.order_old && (!a.vs || a.vs_old) &&
           a.ms && a.ms_old && a.xb && a.cell_id && a.count && a.cell_start && a.fill && a.tmp && a.tile_sum && a.ticket;
}

hipError_t launch_cell_build(const CellArgs &a, hipStream_t st)
{
    if (!cell_args_ok(a)) return hipErrorInvalidValue;
    int grid = (a.N + kBlock - 1) / kBlock;
    int nt = scan_tiles(a.g.ncell);
    hipLaunchKernelGGL(k_cell_ids, dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kBlock), 0, st, a);
    hipLaunchKernelGGL(k_rank, dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_cell_build_batch(const CellArgs *tab, const EnsItem *per256, int n256, const EnsItem *pertile,
                                   int ntile, hipStream_t st)
{
    if (!tab || (n256 > 0 && !per256) || (ntile > 0 && !pertile)) return hipErrorInvalidValue;
    if (n256 > 0) hipLaunchKernelGGL(k_cell_ids_batch, dim3(n256), dim3(kBlock), 0, st, tab, per256);
    if (ntile > 0) hipLaunchKernelGGL(k_scan_tiles_batch, dim3(ntile), dim3(kBlock), 0, st, tab, pertile);
    if (ntile > 0) hipLaunchKernelGGL(k_scan_apply_batch, dim3(ntile), dim3(kBlock), 0, st, tab, pertile);
    if (n256 > 0) hipLaunchKernelGGL(k_scatter_batch, dim3(n256), dim3(kBlock), 0, st, tab, per256);
    if (n256 > 0) hipLaunchKernelGGL(k_rank_batch, dim3(n256), dim3(kBlock), 0, st, tab, per256);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// first half-kick + drift + wrap in cell order; raises the rebuild gate of
// this step when a particle has moved more than half the skin since the last
// build, and clears the gate of the next step (when the caller alternates two
// gates)
// ---------------------------------------------------------------------------

__device__ inline void kick_drift_body(const KickDriftArgs &a, int b)
{
    int p = b * kBlock + threadIdx.x;
    if (p == 0 && a.gate_next) *a.gate_next = 0;
    if (p >= a.N) return;
    const double hm = (0.5 * a.dt) / a.ms[p];
    const double4 r = a.xs[p];
    double x[3] = {r.x, r.y, r.z};
    double v[3] = {a.vs[p], a.vs[a.N + p], a.vs[2 * a.N + p]};
    if (a.vscale) {   // a global bath's half-steps since the last kick
        const double sc = *a.vscale;
        v[0] = v[0] * sc;
        v[1] = v[1] * sc;
        v[2] = v[2] * sc;
    }
    const double f[3] = {a.fs[p], a.fs[a.N + p], a.fs[2 * a.N + p]};
    bool bad = false;
    double d2 = kick_drift_row(x, v, f, hm, a.dt, a.L, a.inv_L, a.xb, a.N, p, &bad, a.th,
                               a.th.on ? (uint64_t)a.order[p] : 0, a.ms[p]);
    for (int d = 0; d < 3; ++d) a.vs[d * a.N + p] = v[d];
    a.xs[p] = make_double4(x[0], x[1], x[2], r.w);
    raise_any(a.flag, bad);
    raise_gate(a.gate, d2, a.half_skin2, p);
}

RBSOG_KERNELS(kick_drift, KickDriftArgs, kBlock)

hipError_t launch_kick_drift(const KickDriftArgs &a, hipStream_t st)
{
    if (a.N < 1 || !a.xs || !a.vs || !a.fs || !a.ms || !a.xb || !a.gate || !a.flag || (a.th.on && !a.order))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kick_drift, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_kick_drift_batch(const KickDriftArgs *tab, const EnsItem *per256, int n, hipStream_t st)
{
    if (!tab || !per256 || n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_kick_drift_batch, dim3(n), dim3(kBlock), 0, st, tab, per256);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// caller order <-> cell order
// ---------------------------------------------------------------------------

__device__ inline void state_in_body(const PermArgs &a, int b)
{
    int p = b * kBlock + threadIdx.x;
    if (p >= a.N) return;
    const int i = a.order[p];
    a.xs[p] = make_double4(a.x[i], a.x[a.N + i], a.x[2 * a.N + i], a.q[i]);
    a.ms[p] = a.m[i];
    for (int d = 0; d < 3; ++d) {
        if (a.v) a.vs[d * a.N + p] = a.v[d * a.N + i];
        if (a.f) a.fs[d * a.N + p] = a.f[d * a.N + i];
    }
}

__device__ inline void state_out_body(const PermArgs &a, int b)
{
    int p = b * kBlock + threadIdx.x;
    if (p >= a.N) return;
    const int i = a.order[p];
    const double4 r = a.xs[p];
    a.x[i] = r.x;
    a.x[a.N + i] = r.y;
    a.x[2 * a.N + i] = r.z;
    for (int d = 0; d < 3; ++d) {
        if (a.v) a.v[d * a.N + i] = a.vs[d * a.N + p];
        if (a.f) a.f[d * a.N + i] = a.fs[d * a.N + p];
    }
}

__global__ __launch_bounds__(kBlock) void k_state_in(PermArgs a) { state_in_body(a, (int)blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_state_out(PermArgs a) { state_out_body(a, (int)blockIdx.x); }

hipError_t launch_state_in(const PermArgs &a, hipStream_t st)
{
    if (a.N < 1 || !a.order || !a.x || !a.q || !a.m || !a.xs || !a.ms || (a.v && !a.vs) || (a.f && !a.fs))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_state_in, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_state_out(const PermArgs &a, hipStream_t st)
{
    if (a.N < 1 || !a.order || !a.x || !a.xs || (a.v && !a.vs) || (a.f && !a.fs)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_state_out, dim3((a.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t *order, int N)
{
    int p = blockIdx.x * kBlock + threadIdx.x;
    if (p < N) order[p] = p;
}

hipError_t launch_iota(int32_t *order, int N, hipStream_t st)
{
    if (!order || N < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_iota, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, order, N);
    return hipGetLastError();
}

__global__ void k_set_int(int32_t *p, int32_t v) { *p = v; }

hipError_t launch_set_int(int32_t *p, int32_t v, hipStream_t st)
{
    if (!p) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
    return hipGetLastError();
}

}  // namespace rbsog

#!/usr/bin/env python3
"""Throughput of the RBSOG time step on one MI355X.

Headline workload: the Yukawa one-component plasma with N = 1e6 unit charges
at number density 3/(4 pi) (Wigner-Seitz radius 1), kappa = 0.1, r_c = 5,
P = 500 sampled Fourier modes, SOG tolerance 1e-4, dt = 0.01, seeded uniform
positions and Maxwell velocities, in two runs of 200 NVE velocity-Verlet steps:
Gamma = 0.1 (k_B T = 10) and Gamma = 100 (k_B T = 0.01).  A timed step is one
velocity-Verlet step: half-kick + drift, cell list, neighbour lists, mode
sampling, structure factors, near field, far field + second half-kick, and the
energy terms of the new state.  `value` is the FP64 throughput of the two runs
together (their particle-steps over their summed time); mixed precision beside it.

Also reported: the force error against the FP64 CPU oracle at the final state
(total, near and far; relative RMS and the largest single-particle error), the
energy drift of each run (all steps, and the second half), per-kernel times from
HIP events on the stream the kernels run on, the roofline position of the
dominant kernel, the oracle's throughput on this machine's host cores, and the
other workloads of the suite (N = 1000, N = 1e5 with pre-equilibration, the
served ensemble, the binary mixture) as extra keys.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at stated force RMS error; served-ensemble p50/p99 step latency"
PEAK_FP64_TFLOPS = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
PEAK_SLOTS = PEAK_FP64_TFLOPS / 2 * 1e12   # VALU issue slots per second (one FMA, add, mul or compare each)
PEAK_HBM_GBS = 8000.0

# Algorithmic VALU issue slots per unit of work (one slot per add, multiply,
# FMA or compare), as the method states its work: an exponential, a square root
# or a sine-cosine pair costs what the device library's FP64 function costs on
# this GPU, measured live (elementary_prices) in FMA slots.
#   pair within r_c: 1 sqrt + (M + 1) exp + (15 + 2 M) arithmetic + 3 FMA accumulation
#   candidate tested: 3 sub + 3 FMA + 1 compare
#   structure-factor term (particle, mode): 3 FMA phase + 1 fract + sincos + 2 FMA accumulation
#   far-field term (particle, mode): 3 FMA phase + 1 fract + sincos + 2 (Im) + 1 (coef) + 3 FMA


def slots_pair(M: int, pr: dict) -> float:
    return pr["sqrt"] + (M + 1) * pr["exp"] + 15 + 2 * M + 3


SLOTS_CANDIDATE = 7.0


def slots_rho(pr: dict) -> float:
    return 6 + pr["sincos"]


def slots_far(pr: dict) -> float:
    return 10 + pr["sincos"]


# Sources each profiled kernel is built from: a stored counter figure holds
# only while the SHA-256 over these files is the one it was taken on.
KERNEL_SOURCES = {
    "near": ["k_near.hip", "k_rho.hip", "dev_common.h", "dev_math.h", "launch.h"],
    "far": ["k_far.hip", "dev_common.h", "dev_math.h", "launch.h"],
    "nlist": ["k_near.hip", "dev_common.h", "launch.h"],
}

# HBM bytes per launch at the N = 1e6, Gamma = 0.1 plasma (FP64), from one
# FETCH_SIZE and one WRITE_SIZE counter run (KiB per dispatch, mean over the
# profiled dispatches), each scaled by what the same counter reads for an FP64
# copy y = 2x of 256 MiB (FETCH_SIZE 131086 KiB for 262144 KiB read: x2.000;
# WRITE_SIZE 262147 KiB for 262144 KiB written: x1.000).
MEASURED_TRAFFIC = {
    # kernel: (sources sha256, FETCH_SIZE KiB, WRITE_SIZE KiB, fetch scale, write scale)
    "near": ("2edc4d3d5daba9c89dc3bd03b92b66876eec853fe4d09cafb3ce0c42d98c9f5a", 419413.0, 100836.0, 2.0, 1.0),
    "far": ("8a7c054038bc2072189517df0d36b38d52c239fcc80a1550dab3e5fc888b6711", 78336.0, 78613.0, 2.0, 1.0),
    "nlist": ("adf973cba8197b26cebf41bd16d350515c2037a2819a967fb5d13af835ff96be", 83770.0, 517545.0, 2.0, 1.0),
}

# VALU issue at the same workload (FP64): VALU busy = SQ_ACTIVE_INST_VALU x 4
# cycles / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8 XCDs), lane utilisation =
# SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU); their product is the
# fraction of the VALU's lane-cycles that issued work.
MEASURED_VALU = {
    # kernel: (sources sha256, VALU busy, lane utilisation)
    "near": ("2edc4d3d5daba9c89dc3bd03b92b66876eec853fe4d09cafb3ce0c42d98c9f5a", 0.79, 0.89),
    "far": ("8a7c054038bc2072189517df0d36b38d52c239fcc80a1550dab3e5fc888b6711", 0.89, 1.00),
    "nlist": ("adf973cba8197b26cebf41bd16d350515c2037a2819a967fb5d13af835ff96be", 0.83, 0.76),
}


def sources_sha256(kernel: str) -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2501_10946_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    t = MEASURED_TRAFFIC.get(kernel)
    if t is None or t[0] != sources_sha256(kernel):
        return None
    return (t[1] * t[3] + t[2] * t[4]) * 1024.0


def measured_valu(kernel: str):
    t = MEASURED_VALU.get(kernel)
    if t is None or t[0] != sources_sha256(kernel):
        return None
    return {"valu_busy": t[1], "lane_utilisation": t[2], "busy_x_utilisation": t[1] * t[2]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model or platform.processor(), "nproc": avail, "cpu_count": os.cpu_count()}


# ---------------------------------------------------------------------------
# elementary-function prices (libprice.so, measured on this GPU)
# ---------------------------------------------------------------------------

def elementary_prices() -> dict:
    """FMA issue slots per FP64 call of exp, sincos, sqrt and rsqrt (the device
    library's functions), from the time per call against a plain FMA chain."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2501_10946_amd", "libprice.so"))
    lib.rbsog_price_run.restype = ctypes.c_int
    lib.rbsog_price_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    blocks = 256 * 8 * 4   # 8 workgroups of 4 waves per CU

    def run(op, iters):
        ms = ctypes.c_double()
        if lib.rbsog_price_run(op, iters, blocks, ctypes.byref(ms)) != 0:
            raise RuntimeError("rbsog_price_run failed")
        return ms.value / (iters * 8.0)   # ms per call per lane-chain step (grid-wide)

    t_fma = run(0, 4000)
    t_exp = run(1, 400)
    t_sc = run(2, 200)
    t_sqrt = run(3, 1000)
    t_rsq = run(4, 1000)
    calls = blocks * 256.0   # lane-chain steps per ms-unit above: t_* is per (iteration x chain)
    return {
        "fma": 1.0,
        "exp": t_exp / t_fma,
        "sincos": t_sc / t_fma - 1.0,    # the chain's one FMA beside each call
        "sqrt": t_sqrt / t_fma - 1.0,    # the chain's one add
        "rsqrt": t_rsq / t_fma - 1.0,
        "fma_calls_per_s": calls / (t_fma * 1e-3),
        "fma_peak_fraction": (calls / (t_fma * 1e-3)) / PEAK_SLOTS,
    }


# ---------------------------------------------------------------------------
# statistics
# ---------------------------------------------------------------------------

def energy_drift(E, dt: float, scale: float) -> dict:
    """Least-squares slope of the per-step total energy (in units of `scale`,
    N k_B T) per unit time, with its standard error, and the spread."""
    import numpy as np
    E = np.asarray(E, dtype=np.float64)
    t = dt * np.arange(1, len(E) + 1)
    y = E / scale
    if len(y) < 3:
        return {"steps": len(y)}
    A = np.vstack([t, np.ones_like(t)]).T
    coef, _, _, _ = np.linalg.lstsq(A, y, rcond=None)
    n = len(y)
    resid = y - A @ coef
    s2 = float(resid @ resid) / max(1, n - 2)
    se = (s2 / float(((t - t.mean()) ** 2).sum())) ** 0.5
    return {"steps": n, "slope_NkT_per_time": float(coef[0]), "stderr": se, "std_NkT": float(np.std(y)),
            "E0_NkT": float(y[0]), "E_end_NkT": float(y[-1])}


def force_errors(fg, fng, fo, fno) -> dict:
    """Relative RMS over all components and the largest single-particle error
    (relative to the RMS particle force) of total, near and far forces."""
    import numpy as np

    def pair(a, b):
        r = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        d = np.linalg.norm(a - b, axis=0)
        s = float(np.sqrt(np.mean(np.linalg.norm(b, axis=0) ** 2)))
        return {"rel_rms": r, "max_particle": float(d.max()) / s}

    return {"total": pair(fg, fo), "near": pair(fng, fno), "far": pair(fg - fng, fo - fno)}


def count_pairs(x, L, rc) -> int:
    """Ordered pairs within r_c (periodic), the near field's algorithmic work."""
    from scipy.spatial import cKDTree
    t = cKDTree(x.T.copy() % L, boxsize=L)
    return int(t.count_neighbors(t, rc)) - x.shape[1]   # every particle counts itself once


def canonical_candidates(N: int, L: float, rc: float) -> float:
    """Candidates a particle tests over the 27 cells of width L / floor(L / r_c)
    around it (the cell-list search of the method), times N."""
    nc = math.floor(L / rc)
    return N * 27.0 * N / nc ** 3


# ---------------------------------------------------------------------------
# one system: timed steps, per-kernel times, force error, drift
# ---------------------------------------------------------------------------

def run_workload(R, w, st, sog, prec, steps, warmup, dev, skin=-1.0, x0=None, v0=None, step0=0,
                 kernel_pass=True):
    """W untimed warm-up steps from the state, then K timed NVE steps from the
    same state (forces and integration; the near-field energy is optional in
    the method and not evaluated), then (kernel_pass) a pass of K/4 more steps
    with per-kernel events, then the same K steps once more from the state
    with the per-step energies recorded (untimed) for the drift.  Returns
    throughput, the final state of the timed run and the energy history."""
    import torch
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, precision=prec, skin=skin, device=dev)
    xs = torch.tensor(st.x if x0 is None else x0, device=dev)
    vs = torch.tensor(st.v if v0 is None else v0, device=dev)
    if warmup > 0:
        x, v, f = xs.clone(), vs.clone(), torch.empty_like(xs)
        R.rbsog_compute_forces(s.h, step0, x, f)
        R.rbsog_step(s.h, x, v, f, step0, warmup, w.dt)
        torch.cuda.synchronize()
        R.rbsog_check(s.h)
        del x, v, f
    x, v, f = xs.clone(), vs.clone(), torch.empty_like(xs)
    R.rbsog_compute_forces(s.h, step0, x, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R.rbsog_step(s.h, x, v, f, step0, steps, w.dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    R.rbsog_check(s.h)
    res = {"value": w.N * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps, "elapsed_s": elapsed,
           "x": x.clone(), "v": v.clone(), "step": step0 + steps, "info": R.rbsog_get_info(s.h)}
    if kernel_pass:
        n = max(10, steps // 4)
        xk, vk, fk = x.clone(), v.clone(), f.clone()
        R.rbsog_timing_enable(s.h, True)
        R.rbsog_step(s.h, xk, vk, fk, step0 + steps, n, w.dt)
        res["kernels"] = {k: {"ms_per_launch": (t / c if c else 0.0), "launches": c, "ms_per_step": t / n}
                          for k, (t, c) in R.rbsog_timing_read(s.h).items() if c}
        R.rbsog_timing_enable(s.h, False)
        R.rbsog_check(s.h)
    # the energy history of the same trajectory (untimed)
    x, v, f = xs.clone(), vs.clone(), torch.empty_like(xs)
    eh = torch.zeros((steps, R.ENERGY_COLS), dtype=torch.float64, device=dev)
    R.rbsog_compute_forces(s.h, step0, x, f)
    t0 = time.perf_counter()
    R.rbsog_step(s.h, x, v, f, step0, steps, w.dt, eh)
    torch.cuda.synchronize()
    res["ms_per_step_with_energies"] = 1e3 * (time.perf_counter() - t0) / steps
    R.rbsog_check(s.h)
    res["ehist"] = eh.cpu().numpy()
    res["system"] = s
    return res


def force_check(R, oracle, w, st, o, x_state, step, dev, nsample=512):
    """Library forces (FP64 and mixed) at one state against the FP64 oracle on
    `nsample` sampled particles: near field by the oracle's subset pair sum, far
    field from the oracle's structure factors of the same sampled modes."""
    import numpy as np
    import torch
    xh = x_state.cpu().numpy() if hasattr(x_state, "cpu") else x_state
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(w.N, min(nsample, w.N), replace=False))
    n3, coef = ref.draw(step)
    rho = oracle.rho(xh, st.q, w.L, n3)
    fno = oracle.near_subset(xh, st.q, w.L, o, idx)
    ffo = oracle.far_rb(xh[:, idx], st.q[idx], w.L, n3, coef, rho)
    sog_o = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    xt = torch.tensor(xh, device=dev)
    out = {}
    for name, prec in (("fp64", R.RBSOG_FP64), ("mixed", R.RBSOG_MIXED)):
        s = R.System(st.q, st.m, w.L, sog_o, w.kT, w.P, seed=w.seed, precision=prec, device=dev)
        fg = torch.empty_like(xt)
        fng = torch.empty_like(xt)
        R.rbsog_compute_forces(s.h, step, xt, fg, fng)
        torch.cuda.synchronize()
        out[name] = force_errors(fg.cpu().numpy()[:, idx], fng.cpu().numpy()[:, idx], fno + ffo, fno)
        del s
    out["sampled_particles"] = int(len(idx))
    return out


def strip(res: dict) -> dict:
    return {k: v for k, v in res.items() if k not in ("x", "v", "ehist", "system", "info", "step", "elapsed_s")}


def rooflines(kern: dict, work: dict) -> dict:
    """Every priced kernel: algorithmic slots per launch / mean launch time."""
    out = {}
    for k, slots in work.items():
        if k in kern and kern[k]["ms_per_launch"] > 0:
            rate = slots / (kern[k]["ms_per_launch"] * 1e-3)
            out[k] = {"achieved": 2 * rate / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                      "frac": rate / PEAK_SLOTS, "slots_per_launch": slots,
                      "ms_per_launch": kern[k]["ms_per_launch"],
                      "basis": "algorithmic: the method's operations with exp, sqrt and sincos priced at the device "
                               "library's measured cost (an equivalent rate, not issued work; valu_counters has "
                               "the issued fraction)"}
    return out


# ---------------------------------------------------------------------------
# the served ensemble
# ---------------------------------------------------------------------------

def preequilibrate(R, w, st, sog, dev, steps):
    """`steps` FP64 steps from the seeded state with the velocities rescaled to
    the target kinetic energy after each (untimed); returns (x, v) on the host."""
    import torch
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, device=dev)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    eh = torch.zeros((1, R.ENERGY_COLS), dtype=torch.float64, device=dev)
    ke_target = 0.5 * (3 * w.N - 3) * w.kT
    for k in range(steps):
        R.rbsog_step(s.h, x, v, f, k, 1, w.dt, eh)
        v.mul_(torch.sqrt(ke_target / eh[0, 5]))
    R.rbsog_check(s.h)
    xe, ve = x.cpu().numpy(), v.cpu().numpy()
    del s
    return xe, ve


def variance_experiment(R, dev, draws=400, snapshots=20, equil_steps=20000, gap=100):
    """The fluctuation comparison of the sampling densities (Section 5.3,
    Fig. 8) through the library: the 1000-particle plasma with P = 20 at
    effective couplings 1e-3 .. 100, equilibrated by the library's own dynamics
    (velocities rescaled to the target temperature each step), then along an
    NVE run `snapshots` states `gap` steps apart, each evaluated with `draws`
    random batches per density against the full-lattice far field of the same
    library: E_fluc = <(E* - E)^2>, F_fluc = <(1/N) sum_i |F*_i - F_i|^2>.
    "adaptive_tinst" is the adaptive density at the snapshot's instantaneous
    temperature (rbsog_set_kT, Section 4.3)."""
    import numpy as np
    import torch

    import workloads
    names = {R.RBSOG_ADAPTIVE: "adaptive", R.RBSOG_FLAT: "flat", R.RBSOG_K2: "k2", R.RBSOG_DH4PI: "dh4pi"}
    out = {"recipe": {"N": 1000, "P": 20, "kappa": workloads.VARIANCE_KAPPA, "r_c": 5.0 / workloads.VARIANCE_KAPPA,
                      "draws_per_snapshot": draws, "snapshots": snapshots, "equilibration_steps": equil_steps,
                      "snapshot_gap_steps": gap}, "gamma_star": {}}
    for gs in workloads.VARIANCE_GAMMA_STAR:
        w = workloads.variance_workload(gs)
        st = workloads.make_state(w)
        sog = R.rbsog_sog_init(w.lam, w.r_c, w.eps)
        dyn = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, device=dev)
        full = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, full_k=True, device=dev)
        rb = {d: R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed + 1, density=d, device=dev) for d in names}
        tinst = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed + 1, density=R.RBSOG_ADAPTIVE, device=dev)
        x = torch.tensor(st.x, device=dev)
        v = torch.tensor(st.v, device=dev)
        f = torch.empty_like(x)
        R.rbsog_compute_forces(dyn.h, 0, x, f)
        eh = torch.zeros((1, R.ENERGY_COLS), dtype=torch.float64, device=dev)
        ke_target = 0.5 * (3 * w.N - 3) * w.kT
        for k in range(equil_steps):
            R.rbsog_step(dyn.h, x, v, f, k, 1, w.dt, eh)
            v.mul_(torch.sqrt(ke_target / eh[0, 5]))
        step = equil_steps
        acc = {n: [0.0, 0.0] for n in list(names.values()) + ["adaptive_tinst"]}
        F = torch.empty((draws, 3, w.N), dtype=torch.float64, device=dev)
        E = torch.zeros((draws, R.ENERGY_COLS), dtype=torch.float64, device=dev)
        ff = torch.empty_like(x)
        ef = torch.zeros(R.ENERGY_COLS, dtype=torch.float64, device=dev)
        ehist = torch.zeros((gap, R.ENERGY_COLS), dtype=torch.float64, device=dev)
        t_inst = []
        for snap in range(snapshots):
            R.rbsog_step(dyn.h, x, v, f, step, gap, w.dt, ehist)
            step += gap
            kT_now = 2.0 * float(ehist[-1, 5]) / (3 * w.N - 3)
            t_inst.append(kT_now)
            R.rbsog_set_kT(tinst.h, kT_now)
            R.rbsog_compute_forces(full.h, 0, x, ff, None, ef)
            for name, sysm in [(names[d], rb[d]) for d in names] + [("adaptive_tinst", tinst)]:
                for s in range(draws):
                    R.rbsog_compute_forces(sysm.h, snap * draws + s, x, F[s], None, E[s])
                acc[name][0] += float(((E[:, 1] - ef[1]) ** 2).mean())
                acc[name][1] += float((((F - ff[None]) ** 2).sum(dim=(1, 2)) / w.N).mean())
        for sysm in [dyn, full, tinst] + list(rb.values()):
            R.rbsog_check(sysm.h)
        res = {n: {"E_fluc": a[0] / snapshots, "F_fluc": a[1] / snapshots} for n, a in acc.items()}
        emin = min(res[n]["E_fluc"] for n in names.values())
        fmin = min(res[n]["F_fluc"] for n in names.values())
        for n in res:
            res[n]["E_rel"] = res[n]["E_fluc"] / emin
            res[n]["F_rel"] = res[n]["F_fluc"] / fmin
        out["gamma_star"][f"{gs:g}"] = {"gamma": w.gamma, "kT": w.kT, "dt": w.dt,
                                         "kT_inst_mean": float(np.mean(t_inst)), "densities": res}
        log(f"[bench] variance Gamma* {gs:g}: " + ", ".join(
            f"{n} E {r['E_rel']:.2f} F {r['F_rel']:.2f}" for n, r in res.items()))
        del dyn, full, rb, tinst
    return out


def serve(args, dev):
    """The served ensemble: seeded requests (N log-uniform in [500, 5e4], Gamma
    log-uniform in [0.1, 100], kappa uniform in [0.1, 2], r_c 4, P 200, 100
    steps, mixed precision) admitted into one ensemble.  First all at t = 0
    (saturated capacity), then Poisson arrivals at fractions of that capacity,
    then a small pool that forces queueing."""
    import numpy as np
    import torch

    import paper_2501_10946_amd as R
    import workloads

    reqs = workloads.served_requests(args.serve_requests)
    prep = []
    for i, (_, w) in enumerate(reqs):
        st = workloads.make_state(w)
        sog = R.rbsog_sog_init(w.lam, w.r_c, w.eps)
        params = R.make_params(w.N, w.L, w.kT, w.P, 104, i, 0, R.RBSOG_MIXED)
        prep.append((w, st, sog, params))
    total_ps = sum(w.N * w.steps for w, _, _, _ in prep)
    need = [R.rbsog_ens_bytes(p, sg, w.steps) for w, _, sg, p in prep]
    free, _ = torch.cuda.mem_get_info(dev)
    log(f"[serve] {len(prep)} requests, {sum(w.N for w, *_ in prep)} particles, "
        f"{sum(need) / 2**30:.2f} GiB of replica state, {free / 2**30:.1f} GiB free")

    def run(arrivals, budget, max_slots):
        ens = R.rbsog_ens_create(budget, max_slots)
        try:
            pending = list(range(len(prep)))
            slot_req, t_done, active_at, times = {}, {}, [], []
            done = 0
            t_admit = 0.0
            t0 = time.perf_counter()
            while done < len(prep):
                now = time.perf_counter() - t0
                while pending and arrivals[pending[0]] <= now:
                    i = pending[0]
                    w, st, sg, p = prep[i]
                    ta = time.perf_counter()
                    try:
                        slot = R.rbsog_ens_admit(ens, p, sg, np.ascontiguousarray(st.x), np.ascontiguousarray(st.v),
                                                 np.ascontiguousarray(st.q), np.ascontiguousarray(st.m), w.steps,
                                                 w.dt)
                    except R.RbsogError as e:
                        if e.code != R.RBSOG_EAGAIN:
                            raise
                        break
                    finally:
                        t_admit += time.perf_counter() - ta
                    slot_req[slot] = i
                    pending.pop(0)
                stat = R.rbsog_ens_status(ens)
                if stat["active"] > 0:
                    active_at.append(stat["active"])
                    R.rbsog_ens_step(ens)
                    while len(times) < stat["ens_steps"]:
                        times.append(R.rbsog_ens_step_time(ens, len(times) + 1))
                elif pending and arrivals[pending[0]] > now:
                    time.sleep(min(1e-3, arrivals[pending[0]] - now))
                else:
                    torch.cuda.synchronize()
                for slot in R.rbsog_ens_poll(ens, max_slots):
                    R.rbsog_ens_retire(ens, slot)
                    t_done[slot_req.pop(slot)] = time.perf_counter() - t0
                    done += 1
            wall = time.perf_counter() - t0
            nst = R.rbsog_ens_status(ens)["ens_steps"]
            while len(times) < nst:
                times.append(R.rbsog_ens_step_time(ens, len(times) + 1))
            times = np.array(times)
        finally:
            R.rbsog_ens_destroy(ens)
        gaps = np.diff(times)
        w_gaps = np.repeat(gaps, active_at[1:len(times)]) if len(gaps) else np.zeros(1)
        lat = np.array([t_done[i] - arrivals[i] for i in range(len(prep))])
        return {"wall_s": wall, "admission_s": t_admit, "ens_steps": int(nst),
                "step_time_sum_s": float(gaps.sum() / 1e3) if len(gaps) else 0.0,
                "particle_steps_per_s": total_ps / wall, "requests_per_s": len(prep) / wall,
                "step_ms_p50": float(np.percentile(w_gaps, 50)), "step_ms_p99": float(np.percentile(w_gaps, 99)),
                "request_ms_p50": 1e3 * float(np.percentile(lat, 50)),
                "request_ms_p99": 1e3 * float(np.percentile(lat, 99)),
                "mean_active": float(np.mean(active_at)) if active_at else 0.0}

    budget = int(free * 0.8)
    zero = np.zeros(len(prep))
    sat = run(zero, budget, len(prep))
    log(f"[serve] saturated: {sat}")
    out = {"workload": f"served_{len(prep)}req_mixed", "requests": len(prep), "steps_each": 100,
           "particle_steps": total_ps, "budget_bytes": budget, "saturated": sat, "poisson": {}}
    cap = sat["requests_per_s"]
    for frac in [float(v) for v in args.serve_rates.split(",") if v]:
        arr = np.array([t for t, _ in workloads.served_requests(args.serve_requests, rate=frac * cap)])
        r = run(arr, budget, len(prep))
        out["poisson"][f"{frac:g}"] = dict(r, rate_req_per_s=frac * cap)
        log(f"[serve] poisson {frac:g}x capacity ({frac * cap:.1f} req/s): {r}")
    small = max(need) + sum(sorted(need)[: len(need) // 8])
    r = run(zero, small, len(prep))
    out["small_budget"] = dict(r, budget_bytes=small)
    log(f"[serve] small pool {small / 2**20:.0f} MiB: {r}")
    return out


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed NVE steps per run of the headline workload")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle velocity-Verlet steps of the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-ensemble measurement")
    ap.add_argument("--no-variance", action="store_true", help="skip the sampling-density fluctuation comparison")
    ap.add_argument("--no-force-check", action="store_true")
    ap.add_argument("--skin", type=float, default=-1.0, help="neighbour-list skin (negative: the library default)")
    ap.add_argument("--gammas", default="0.1,100", help="couplings of the headline runs")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rates", default="0.5,0.8,1.2",
                    help="Poisson arrival rates as fractions of the measured saturated capacity")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the served-ensemble measurement, printed as its own JSON line (for profiling)")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="MiB of an elementwise FP64 copy (y = 2x) to run first, as a known-traffic reference "
                         "for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library steps each system (or ensemble) on one GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import oracle
    import paper_2501_10946_amd as R
    import workloads

    if args.serve_only:
        print(json.dumps({"served": serve(args, torch.device("cuda:0"))}), flush=True)
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.copy_calibration > 0:
        n = int(args.copy_calibration * 2 ** 20 / 8)
        a = torch.ones(n, dtype=torch.float64, device=dev)
        for _ in range(3):
            b = a * 2.0
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {n * 8} bytes read and written per launch")
        del a, b

    prices = elementary_prices()
    log(f"[bench] FP64 elementary functions in FMA slots: " +
        ", ".join(f"{k} {prices[k]:.1f}" for k in ("exp", "sincos", "sqrt", "rsqrt")) +
        f" (FMA chain at {prices['fma_peak_fraction']:.2f} of the issue peak)")

    # ---- headline: N = 1e6, kappa = 0.1, r_c = 5, P = 500, Gamma = 0.1 and 100 ----
    gammas = [float(g) for g in args.gammas.split(",") if g]
    base = workloads.OCP_1M_WEAK
    runs, t_tot = {}, {"fp64": 0.0, "mixed": 0.0}
    ps_tot = 0
    cpu = None
    headline_kernels = None
    for g in gammas:
        w = workloads.Workload(f"ocp_n{base.N}_k{base.kappa:g}_g{g:g}", N=base.N, kappa=base.kappa, gamma=g,
                               r_c=base.r_c, P=base.P, steps=args.steps,
                               seed=workloads.OCP_1M_WEAK.seed if g == 0.1 else
                               (workloads.OCP_1M_STRONG.seed if g == 100 else base.seed))
        st = workloads.make_state(w)
        o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
        log(f"[bench] {w.name}: N={w.N} L={w.L:.4f} P={w.P} SOG M1={sog.M1} M2={sog.M2} "
            f"err={sog.max_err:.2e}")
        rr = {}
        for name, prec in (("fp64", R.RBSOG_FP64), ("mixed", R.RBSOG_MIXED)):
            res = run_workload(R, w, st, sog, prec, args.steps, args.warmup, dev, skin=args.skin)
            E = res["ehist"][:, :6].sum(axis=1)
            res["drift"] = {"all": energy_drift(E, w.dt, w.N * w.kT),
                            "second_half": energy_drift(E[args.steps // 2:], w.dt, w.N * w.kT)}
            eh = res["ehist"]
            pv = (2 * eh[:, 5] + eh[:, 6] + eh[:, 7] + 3 * (eh[:, 2] + eh[:, 4])) / (3 * w.V)
            res["pressure"] = {"mean": float(pv.mean()), "std": float(pv.std()), "ideal": w.N * w.kT / w.V,
                               "from": "(2 KE + W_N + W*_F + 3 U_k0 + 3 U_bg) / (3V) per step"}
            info = res["info"]
            res["lists"] = {"skin": info.skin, "nf": info.nf, "near_capacity": info.near_capacity}
            t_tot[name] += res["elapsed_s"]
            log(f"[bench] {w.name} {name}: {res['value']:.4g} particle-steps/s, {res['ms_per_step']:.3f} ms/step; "
                f"kernels " + ", ".join(f"{k} {v['ms_per_step'] * 1e3:.0f} us" for k, v in res["kernels"].items()))
            rr[name] = res
        ps_tot += w.N * args.steps
        if not args.no_force_check:
            rr["force_rel_rms"] = force_check(R, oracle, w, st, o, rr["fp64"]["x"], rr["fp64"]["step"] + 1, dev)
            log(f"[bench] {w.name} force error vs oracle: {rr['force_rel_rms']}")
        if g == gammas[0]:
            headline_kernels = (w, rr["fp64"]["kernels"], rr["fp64"]["x"].cpu().numpy(), sog.n)
            if not args.no_cpu_baseline:
                # the oracle on this machine's host cores: a bounded number of
                # velocity-Verlet steps of the same workload from the same state
                ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
                xo, vo = st.x.copy(), st.v.copy()
                t0 = time.perf_counter()
                fo, _, _ = ref.force(xo, 0)
                t_f = time.perf_counter() - t0
                t0 = time.perf_counter()
                ref.run(xo, vo, fo, 0, args.cpu_steps, w.dt)
                tk = time.perf_counter() - t0
                hi = host_info()
                cpu = {"value": w.N * args.cpu_steps / tk, "unit": "particle-steps/s",
                       "cores": oracle.num_threads(), "kind": "oracle",
                       "sample": f"{args.cpu_steps} FP64 velocity-Verlet steps of {w.name} from the seeded state "
                                 f"(OpenMP; one force evaluation {t_f:.1f} s)",
                       "nproc": hi["nproc"], "cpu_model": hi["cpu_model"], "seconds": tk}
                log(f"[bench] oracle: {cpu['value']:.4g} particle-steps/s on {cpu['cores']} threads "
                    f"({hi['cpu_model']}, nproc {hi['nproc']}; {tk:.1f} s)")
        runs[f"gamma_{g:g}"] = {"N": w.N, "kT": w.kT, "seed": w.seed,
                                "fp64": strip(rr["fp64"]), "mixed": strip(rr["mixed"]),
                                "force_rel_rms": rr.get("force_rel_rms")}
        for name in ("fp64", "mixed"):
            rr[name].pop("system", None)
        del rr
        torch.cuda.empty_cache()

    # ---- roofline of the dominant kernel (FP64, first coupling) ----
    roofline, kroof = None, {}
    if headline_kernels is not None:
        w, kern, xh, M = headline_kernels
        npairs = count_pairs(xh, w.L, w.r_c)
        near_slots = npairs * slots_pair(M, prices)
        rho_slots = w.N * w.P * slots_rho(prices)
        fused_rho = kern.get("rho_partial") is None
        work = {
            "near": near_slots + (rho_slots if fused_rho else 0.0),
            "far": w.N * w.P * slots_far(prices),
            "nlist": canonical_candidates(w.N, w.L, w.r_c) * SLOTS_CANDIDATE,
        }
        if not fused_rho:
            work["rho_partial"] = rho_slots
        kroof = rooflines(kern, work)
        for k in kroof:
            kroof[k]["traffic"] = measured_traffic(k) if k in KERNEL_SOURCES else None
            vc = measured_valu(k) if k in KERNEL_SOURCES else None
            if vc is not None:
                kroof[k]["valu_counters"] = vc
        dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
        if dom in kroof:
            roofline = dict(kroof[dom], kernel=dom + ("+rho_partial" if dom == "near" and fused_rho else ""),
                            bound="alu", traffic=measured_traffic(dom))
            vc = measured_valu(dom)
            if vc is not None:
                roofline["valu_counters"] = vc
        log(f"[bench] near pairs {npairs} ({npairs / w.N:.1f} per particle); dominant kernel {dom}")

    n_runs = len(gammas)
    out = {
        "metric": METRIC,
        "value": ps_tot / t_tot["fp64"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_tot["fp64"] / (n_runs * args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ocp_n1000000_k0.1_rc5_p500_" + "+".join(f"g{g:g}" for g in gammas),
                   "N": base.N, "kappa": base.kappa, "gamma": gammas, "r_c": base.r_c, "P": base.P,
                   "eps": base.eps, "dt": base.dt, "nve_steps_per_run": args.steps,
                   "force_rel_rms": {k: (v["force_rel_rms"] or {}).get("fp64") for k, v in runs.items()}},
        "mixed": {"value": ps_tot / t_tot["mixed"],
                  "ms_per_step": 1e3 * t_tot["mixed"] / (n_runs * args.steps),
                  "speedup_vs_fp64": t_tot["fp64"] / t_tot["mixed"],
                  "dtype": "f32 pair/phase arithmetic, f64 positions, reduction, accumulation and integration",
                  "force_rel_rms": {k: (v["force_rel_rms"] or {}).get("mixed") for k, v in runs.items()}},
        "runs": runs,
        "roofline": roofline,
        "kernel_rooflines": kroof,
        "elementary_prices_fma_slots": prices,
        "cpu_baseline": cpu,
    }

    # ---- the other workloads of the suite ----
    if not args.no_extra:
        extra = {}
        # N = 1000, kappa = 1, Gamma = 1, r_c = 3, P = 100, FP64, 100 steps
        w = workloads.OCP_1K
        st = workloads.make_state(w)
        o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
        res = run_workload(R, w, st, sog, R.RBSOG_FP64, w.steps, 20, dev, kernel_pass=False)
        res["drift"] = energy_drift(res["ehist"][:, :6].sum(axis=1), w.dt, w.N * w.kT)
        ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
        xo, vo = st.x.copy(), st.v.copy()
        fo, _, _ = ref.force(xo, 0)
        ref.run(xo, vo, fo, 0, w.steps, w.dt)
        d = res["x"].cpu().numpy() - xo
        d -= w.L * np.round(d / w.L)
        res["trajectory_max_dx_vs_oracle"] = float(np.abs(d).max())
        if not args.no_force_check:
            res["force_rel_rms"] = force_check(R, oracle, w, st, o, res["x"], res["step"] + 1, dev)
        extra[w.name] = strip(res)
        log(f"[bench] {w.name}: {res['value']:.4g} particle-steps/s, trajectory |dx| {d.__abs__().max():.2e}")
        del res

        # N = 1e5, kappa = 0.5, Gamma = 10: 200 pre-equilibration steps, then FP64 and mixed
        w = workloads.OCP_100K
        st = workloads.make_state(w)
        o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
        xe, ve = preequilibrate(R, w, st, sog, dev, 200)
        c2 = {"preequilibration_steps": 200}
        for name, prec in (("fp64", R.RBSOG_FP64), ("mixed", R.RBSOG_MIXED)):
            res = run_workload(R, w, st, sog, prec, w.steps, 20, dev, x0=xe, v0=ve, step0=200)
            res["drift"] = energy_drift(res["ehist"][:, :6].sum(axis=1), w.dt, w.N * w.kT)
            c2[name] = strip(res)
            log(f"[bench] {w.name} {name}: {res['value']:.4g} particle-steps/s, {res['ms_per_step']:.4f} ms/step")
            if name == "fp64":
                xf, sf = res["x"], res["step"] + 1
        if not args.no_force_check:
            c2["force_rel_rms"] = force_check(R, oracle, w, st, o, xf, sf, dev)
        extra[w.name] = c2

        # binary mixture N = 2e5: 200 pre-equilibration steps, then mixed precision (and FP64 beside it), 500 steps
        w = workloads.MIXTURE_200K
        st = workloads.make_state(w)
        o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
        xe, ve = preequilibrate(R, w, st, sog, dev, 200)
        c5 = {"preequilibration_steps": 200}
        for name, prec in (("mixed", R.RBSOG_MIXED), ("fp64", R.RBSOG_FP64)):
            res = run_workload(R, w, st, sog, prec, w.steps, 20, dev, kernel_pass=False, x0=xe, v0=ve, step0=200)
            res["drift"] = energy_drift(res["ehist"][:, :6].sum(axis=1), w.dt, w.N * w.kT)
            c5[name] = strip(res)
            if name == "mixed":
                xf, sf = res["x"], res["step"] + 1
            log(f"[bench] {w.name} {name}: {res['value']:.4g} particle-steps/s")
        if not args.no_force_check:
            c5["force_rel_rms"] = force_check(R, oracle, w, st, o, xf, sf, dev)
        extra[w.name] = c5
        if not args.no_variance:
            extra["variance_ocp_n1000_p20"] = variance_experiment(R, dev)
        if not args.no_serve:
            extra["served"] = serve(args, dev)
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

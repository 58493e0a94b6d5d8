#!/usr/bin/env python3
"""Throughput of the RBSOG time step on one MI355X.

Workload: the Yukawa one-component plasma with N = 1e5 unit charges at number
density 3/(4 pi) (Wigner-Seitz radius 1), kappa = 0.5, Gamma = 10, r_c = 4,
P = 200 sampled Fourier modes, SOG tolerance 1e-4, dt = 0.01; seeded uniform
positions and Maxwell velocities, pre-equilibrated for 200 steps with the
velocities rescaled to k_B T after each step (untimed).  A timed step is one
velocity-Verlet step: half-kick + drift, cell list, mode sampling, structure
factors, near field, far field + second half-kick.

Prints one JSON line: particle-steps/s of the FP64 path (`value`), the same for
the mixed-precision path, the force error against the FP64 CPU oracle at the
final state, the roofline position of the dominant kernel (per-kernel HIP
events recorded on the stream the kernels run on), and the oracle's own
throughput on this machine's host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at stated force RMS error; served-ensemble p50/p99 step latency"
PEAK_FP64_TFLOPS = 78.6      # 256 CU x 2.4 GHz x 64 FP64 FMA lanes x 2
PEAK_FP32_TFLOPS = 157.3     # published FP32 vector peak (packed FP32)
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 flops per unit of work (FMA = 2, add/mul/rint/compare = 1).  An
# elementary function is priced as a full-accuracy FP64 series: exp2 29 (rint,
# subtract, 13-term Horner, ldexp), sincos in revolutions 40 (two rint, a
# quarter-turn split, 8 + 8 Horner steps, one multiply), whatever the kernels spend.
FLOPS_SINCOS = 40
FLOPS_EXP2 = 29
FLOPS_FAR_PER_IK = 5 + FLOPS_SINCOS + 3 + 6          # phase, sincos, Im(e^{-ikr} rho) coef, 3 FMA
FLOPS_RHO_PER_IK = 5 + FLOPS_SINCOS + 4              # phase, sincos, 2 FMA


def flops_near_per_pair(n_gauss: int) -> int:
    # minimum image 15, r^2 5, cutoff test 1, qq 1, rsqrt 12, r 1, exp(-r/lambda) 1 + 29,
    # F_N1 6, per Gaussian (1 + 29 + 2), factor 2, force 3 FMA 6
    return 15 + 5 + 1 + 1 + 12 + 1 + (1 + FLOPS_EXP2) + 6 + n_gauss * (1 + FLOPS_EXP2 + 2) + 2 + 6


# HBM bytes per launch of a kernel, from one FETCH_SIZE and one WRITE_SIZE counter
# run (KiB per dispatch), each scaled by what the same counter reads for an FP64
# copy of known size.  A figure holds only for the kernel sources it was taken
# on: it is reported when the SHA-256 over the library sources still matches.
MEASURED_TRAFFIC = {
    # kernel: (sources sha256, FETCH_SIZE KiB, WRITE_SIZE KiB, fetch scale, write scale); the scales are what
    # the same counters read for an FP64 copy y = 2 x over 256 MiB (bench.py --copy-calibration 256)
    # (the near launch carries the structure-factor partial sums in its first workgroups)
    "near": ("55d8160675e4a3b15912bd5c7def180d41e0b5e59bf6d3a050bbf6c7a9aee5d3",
             26486.9149, 9475.0, 262144 / 131086.7917, 262144 / 262147.125),
}


def sources_sha256() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2501_10946_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    t = MEASURED_TRAFFIC.get(kernel)
    if t is None or t[0] != sources_sha256():
        return None
    return (t[1] * t[3] + t[2] * t[4]) * 1024.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def energy_drift(E, dt: float, scale: float) -> dict:
    """Least-squares slope of the per-step total energy (in units of `scale`,
    N k_B T) per unit time, with its standard error, and the spread."""
    import numpy as np
    t = dt * np.arange(1, len(E) + 1)
    y = np.asarray(E) / scale
    A = np.vstack([t, np.ones_like(t)]).T
    coef, res, _, _ = np.linalg.lstsq(A, y, rcond=None)
    n = len(y)
    resid = y - A @ coef
    s2 = float(resid @ resid) / max(1, n - 2)
    se = (s2 / float(((t - t.mean()) ** 2).sum())) ** 0.5
    return {"steps": n, "slope_NkT_per_time": float(coef[0]), "stderr": se, "std_NkT": float(np.std(y))}


def force_noise(R, h, h_full, x, m, w, evals: int) -> dict:
    """Random-batch force noise at one state: forces of `evals` independent
    draws (force indices 10^6 + k) against the full-lattice force of the same
    positions.  Velocity-Verlet applies each step's force noise xi over one
    whole time step, so the kinetic energy grows by dt^2 |xi|^2 / (2 m) per
    step and particle: the expected energy drift is dt <|xi|^2 / m> / (2 kT) in
    N kT per unit time.  The mean of the draws estimates the bias, whose RMS
    over particles should be that of the noise over sqrt(evals)."""
    import torch
    ff = torch.empty_like(x)
    R.rbsog_compute_forces(h_full, 0, x, ff)
    fr = torch.empty_like(x)
    s1 = torch.zeros_like(x)
    s2 = torch.zeros(x.shape[1], dtype=torch.float64, device=x.device)
    for k in range(evals):
        R.rbsog_compute_forces(h, 1_000_000 + k, x, fr)
        d = fr - ff
        s1 += d
        s2 += (d * d).sum(dim=0)
    torch.cuda.synchronize()
    R.rbsog_check(h)
    xi2 = s2 / evals
    bias = s1 / evals
    bias_rms = float((bias * bias).sum(dim=0).mean()) ** 0.5
    noise_rms = float(xi2.mean()) ** 0.5
    return {"evals": evals, "xi_rms": noise_rms, "f_full_rms": float((ff * ff).sum(dim=0).mean()) ** 0.5,
            "bias_rms": bias_rms, "bias_rms_expected": noise_rms / evals ** 0.5,
            "predicted_slope_NkT_per_time": w.dt * float((xi2 / m).mean()) / (2.0 * w.kT)}


def serve(args, dev, log):
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
            slot_req, t_adm, t_done, active_at, times = {}, {}, {}, [], []
            done = 0
            t0 = time.perf_counter()
            while done < len(prep):
                now = time.perf_counter() - t0
                while pending and arrivals[pending[0]] <= now:
                    i = pending[0]
                    w, st, sg, p = prep[i]
                    try:
                        slot = R.rbsog_ens_admit(ens, p, sg, np.ascontiguousarray(st.x), np.ascontiguousarray(st.v),
                                                 np.ascontiguousarray(st.q), np.ascontiguousarray(st.m), w.steps,
                                                 w.dt)
                    except R.RbsogError as e:
                        if e.code != R.RBSOG_EAGAIN:
                            raise
                        break
                    slot_req[slot] = i
                    t_adm[i] = time.perf_counter() - t0
                    pending.pop(0)
                stat = R.rbsog_ens_status(ens)
                if stat["active"] > 0:
                    active_at.append(stat["active"])
                    R.rbsog_ens_step(ens)
                    # keep one step queued behind the one running, no more; the
                    # completion times are read as the steps are waited for
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
        # per (replica, step) latency: the gap between consecutive ensemble-step
        # completions, counted once per replica active in the later step
        gaps = np.diff(times)
        w_gaps = np.repeat(gaps, active_at[1:len(times)]) if len(gaps) else np.zeros(1)
        lat = np.array([t_done[i] - arrivals[i] for i in range(len(prep))])
        return {"wall_s": wall, "ens_steps": int(nst), "particle_steps_per_s": total_ps / wall,
                "requests_per_s": len(prep) / wall,
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
        out["poisson"][f"{frac:g}"] = r
        log(f"[serve] poisson {frac:g}x capacity ({frac * cap:.1f} req/s): {r}")
    small = max(need) + sum(sorted(need)[: len(need) // 8])
    r = run(zero, small, len(prep))
    out["small_budget"] = dict(r, budget_bytes=small)
    log(f"[serve] small pool {small / 2**20:.0f} MiB: {r}")
    return out


def count_pairs(x, L, rc) -> int:
    """Ordered pairs within r_c (periodic), the near field's algorithmic work."""
    from scipy.spatial import cKDTree
    t = cKDTree(x.T.copy() % L, boxsize=L)
    return 2 * len(t.query_pairs(rc, output_type="ndarray"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--preeq", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget for the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--skin", type=float, default=-1.0, help="neighbour-list skin (negative: the library default)")
    ap.add_argument("--drift-steps", type=int, default=500, help="NVE steps of the energy-drift runs (0: none)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-ensemble measurement")
    ap.add_argument("--no-fullk-energy", action="store_true",
                    help="skip the deterministic full-lattice energy along the first 100 FP64 NVE steps")
    ap.add_argument("--noise-evals", type=int, default=200,
                    help="random-batch draws for the force-noise estimate of the drift (0: none)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rates", default="0.5,0.8,1.2",
                    help="Poisson arrival rates as fractions of the measured saturated capacity")
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

    import paper_2501_10946_amd as R
    import workloads

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
    w = workloads.OCP_100K
    st = workloads.make_state(w)
    sog = R.rbsog_sog_init(w.lam, w.r_c, w.eps)
    log(f"[bench] {w.name}: N={w.N} L={w.L:.4f} P={w.P} SOG M1={sog.M1} M2={sog.M2} err={sog.max_err:.2e}")

    # ---- pre-equilibration (FP64, velocity rescaling to kT each step) ----
    sys64 = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, precision=R.RBSOG_FP64, skin=args.skin,
                     device=dev)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(sys64.h, 0, x, f)
    eh = torch.zeros((1, 6), dtype=torch.float64, device=dev)
    ke_target = 0.5 * (3 * w.N - 3) * w.kT
    step = 0
    t0 = time.perf_counter()
    for _ in range(args.preeq):
        R.rbsog_step(sys64.h, x, v, f, step, 1, w.dt, eh)
        step += 1
        v.mul_(torch.sqrt(ke_target / eh[0, 5]))
    R.rbsog_check(sys64.h)
    torch.cuda.synchronize()
    log(f"[bench] pre-equilibration {args.preeq} steps: {time.perf_counter() - t0:.2f} s")
    x_eq, v_eq, f_eq, step_eq = x.clone(), v.clone(), f.clone(), step

    results = {}
    for name, prec in (("fp64", R.RBSOG_FP64), ("mixed", R.RBSOG_MIXED)):
        s = sys64 if prec == R.RBSOG_FP64 else R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed,
                                                         precision=prec, skin=args.skin, device=dev)
        x, v, f = x_eq.clone(), v_eq.clone(), f_eq.clone()
        step = step_eq
        R.rbsog_compute_forces(s.h, step, x, f)
        R.rbsog_step(s.h, x, v, f, step, args.warmup, w.dt)
        step += args.warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.rbsog_step(s.h, x, v, f, step, args.steps, w.dt)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        step += args.steps
        R.rbsog_check(s.h)
        res = {"value": w.N * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps}
        # per-kernel HIP events over a second pass of the same number of steps
        if not args.no_roofline:
            R.rbsog_timing_enable(s.h, True)
            R.rbsog_step(s.h, x, v, f, step, args.steps, w.dt)
            step += args.steps
            res["kernels"] = {k: {"ms_per_launch": (t / n if n else 0.0), "launches": n}
                              for k, (t, n) in R.rbsog_timing_read(s.h).items()}
            # the structure-factor partial sums as a launch of their own (the
            # standalone entry point; in a step they share the near launch)
            rho = torch.empty((w.P, 2), dtype=torch.float64, device=dev)
            for k in range(args.steps):
                R.rbsog_compute_rho(s.h, step + k, x, rho)
            t_rho, n_rho = R.rbsog_timing_read(s.h)["rho_partial"]
            res["rho_partial_standalone_ms"] = t_rho / n_rho if n_rho else 0.0
            R.rbsog_timing_enable(s.h, False)
        res["x"], res["step"] = x, step
        # force-only rate: one evaluation (cell order and lists rebuilt, modes,
        # structure factors, near and far field) per call at the final state
        fo = torch.empty_like(x)
        R.rbsog_compute_forces(s.h, step, x, fo)
        torch.cuda.synchronize()
        nf = max(10, args.steps // 4)
        t0 = time.perf_counter()
        for k in range(nf):
            R.rbsog_compute_forces(s.h, step + k, x, fo)
        torch.cuda.synchronize()
        res["force_only"] = w.N * nf / (time.perf_counter() - t0)
        # energy drift over NVE steps from the equilibrated state (untimed)
        if args.drift_steps > 0:
            xd, vd, fd = x_eq.clone(), v_eq.clone(), torch.empty_like(x_eq)
            R.rbsog_compute_forces(s.h, step_eq, xd, fd)
            ehd = torch.zeros((args.drift_steps, 6), dtype=torch.float64, device=dev)
            R.rbsog_step(s.h, xd, vd, fd, step_eq, args.drift_steps, w.dt, ehd)
            R.rbsog_check(s.h)
            res["drift"] = energy_drift(ehd.sum(dim=1).cpu().numpy(), w.dt, w.N * w.kT)
            if prec == R.RBSOG_FP64 and not args.no_fullk_energy:
                # the same trajectory's energy with the whole lattice (no sampling
                # noise) at steps 0, 25, 50, 75, 100
                sfk = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, precision=R.RBSOG_FP64, full_k=True,
                               device=dev)
                mt = torch.tensor(st.m, device=dev)
                xd, vd, fd = x_eq.clone(), v_eq.clone(), torch.empty_like(x_eq)
                R.rbsog_compute_forces(s.h, step_eq, xd, fd)
                ftmp = torch.empty_like(xd)
                e6 = torch.zeros(6, dtype=torch.float64, device=dev)
                efull, sd = [], step_eq
                for c in range(5):
                    R.rbsog_compute_forces(sfk.h, 0, xd, ftmp, None, e6)
                    ke = 0.5 * float((mt * (vd * vd).sum(dim=0)).sum())
                    efull.append((float(e6[:5].sum()) + ke) / (w.N * w.kT))
                    if c < 4:
                        R.rbsog_step(s.h, xd, vd, fd, sd, 25, w.dt)
                        sd += 25
                tt = w.dt * 25 * np.arange(5)
                slope = float(np.polyfit(tt, np.array(efull), 1)[0])
                res["drift"]["full_k"] = {"steps": [0, 25, 50, 75, 100], "E_NkT": efull,
                                          "slope_NkT_per_time": slope, "lattice_points": R.rbsog_get_info(sfk.h).nlat}
                if args.noise_evals > 0:
                    res["drift"]["noise"] = force_noise(R, s.h, sfk.h, x_eq, mt, w, args.noise_evals)
                del sfk
        results[name] = res
        log(f"[bench] {name}: {res['value']:.4g} particle-steps/s, {res['ms_per_step']:.3f} ms/step, "
            f"force-only {res['force_only']:.4g}/s, drift {res.get('drift')}")

    # ---- force error at the final FP64 state, against the FP64 oracle ----
    import oracle
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    xf = results["fp64"]["x"]
    xh = xf.cpu().numpy()
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(w.N, 512, replace=False))
    estep = results["fp64"]["step"] + 1
    n3, coef = ref.draw(estep)
    rho = oracle.rho(xh, st.q, w.L, n3)
    fno = oracle.near_subset(xh, st.q, w.L, o, idx)
    ffo = oracle.far_rb(xh[:, idx], st.q[idx], w.L, n3, coef, rho)
    sog_o = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    errs = {}
    for name, prec in (("fp64", R.RBSOG_FP64), ("mixed", R.RBSOG_MIXED)):
        s = R.System(st.q, st.m, w.L, sog_o, w.kT, w.P, seed=w.seed, precision=prec, device=dev)
        fg = torch.empty_like(xf)
        fng = torch.empty_like(xf)
        R.rbsog_compute_forces(s.h, estep, xf, fg, fng)
        torch.cuda.synchronize()
        fg, fng = fg.cpu().numpy()[:, idx], fng.cpu().numpy()[:, idx]
        rr = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        errs[name] = {"total": rr(fg, fno + ffo), "near": rr(fng, fno), "far": rr(fg - fng, ffo)}
        log(f"[bench] {name} force rel RMS vs oracle: {errs[name]}")

    # ---- roofline of the dominant kernel (FP64 path) ----
    roofline = None
    if not args.no_roofline:
        kern = results["fp64"]["kernels"]
        dom = max(kern, key=lambda k: kern[k]["ms_per_launch"] * kern[k]["launches"])
        ms = kern[dom]["ms_per_launch"]
        npairs = count_pairs(xh, w.L, w.r_c)
        work = {
            "far": w.N * w.P * FLOPS_FAR_PER_IK,
            "rho_partial": w.N * w.P * FLOPS_RHO_PER_IK,
            "near": npairs * flops_near_per_pair(sog.n),
        }
        # the structure-factor partials run inside the near launch (its first
        # workgroups) when no launch of their own was timed: that launch does both
        fused = kern["near"]["launches"] > 0 and kern["rho_partial"]["launches"] == 0
        if fused:
            work["near"] += work.pop("rho_partial")
        if dom in work:
            achieved = work[dom] / (ms * 1e-3) / 1e12
            roofline = {"kernel": "near+rho_partial" if fused and dom == "near" else dom, "bound": "alu",
                        "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(dom),
                        "ms_per_launch": ms, "flops_per_launch": work[dom]}
        log(f"[bench] kernels (fp64): " + ", ".join(f"{k} {v['ms_per_launch']:.4f} ms" for k, v in kern.items()))
        log(f"[bench] near pairs {npairs} ({npairs / w.N:.1f} per particle)")
        results["fp64"]["algorithmic_tflops"] = {("near+rho_partial" if fused and k == "near" else k):
                                                 work[k] / (kern[k]["ms_per_launch"] * 1e-3) / 1e12
                                                 for k in work if kern[k]["ms_per_launch"] > 0}
        ms_rho = results["fp64"].get("rho_partial_standalone_ms", 0.0)
        if ms_rho > 0:
            results["fp64"]["algorithmic_tflops"]["rho_partial (standalone launch)"] = (
                w.N * w.P * FLOPS_RHO_PER_IK / (ms_rho * 1e-3) / 1e12)

    # ---- the oracle on this machine's host cores (bounded sample) ----
    cpu = None
    if not args.no_cpu_baseline:
        xo = x_eq.cpu().numpy().copy()
        vo = v_eq.cpu().numpy().copy()
        fo, _, _ = ref.force(xo, step_eq)
        t0 = time.perf_counter()
        ref.run(xo, vo, fo, step_eq, 1, w.dt)
        t1 = time.perf_counter() - t0
        k = max(1, min(1000, int(args.cpu_seconds / max(t1, 1e-6)) - 1))
        t0 = time.perf_counter()
        ref.run(xo, vo, fo, step_eq + 1, k, w.dt)
        tk = time.perf_counter() - t0 + t1
        cpu = {"value": w.N * (k + 1) / tk, "unit": "particle-steps/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"{k + 1} velocity-Verlet steps of the same workload (FP64, OpenMP)"}
        log(f"[bench] oracle: {cpu['value']:.4g} particle-steps/s on {cpu['cores']} threads ({tk:.1f} s)")

    r64 = results["fp64"]
    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "kappa": w.kappa, "gamma": w.gamma, "r_c": w.r_c, "P": w.P,
                   "eps": w.eps, "dt": w.dt, "n_gauss": sog.n, "preequilibration_steps": args.preeq,
                   "force_rel_rms": errs["fp64"]},
        "mixed": {"value": results["mixed"]["value"], "ms_per_step": results["mixed"]["ms_per_step"],
                  "dtype": "f32 pair/phase arithmetic, f64 accumulation", "force_rel_rms": errs["mixed"]},
        "kernels_ms": {k: v["ms_per_launch"] for k, v in r64.get("kernels", {}).items()},
        "roofline": roofline,
        # every priced kernel against the FP64 vector peak (algorithmic flops per launch / its mean event time)
        "kernel_rooflines": {k: {"achieved": v, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                 "frac": v / PEAK_FP64_TFLOPS}
                             for k, v in r64.get("algorithmic_tflops", {}).items()},
        "cpu_baseline": cpu,
    }
    out["force_only"] = {"fp64": results["fp64"]["force_only"], "mixed": results["mixed"]["force_only"],
                         "unit": "particle-evaluations/s"}
    if "drift" in results["fp64"]:
        out["energy_drift"] = {"fp64": results["fp64"]["drift"], "mixed": results["mixed"]["drift"],
                               "unit": "N k_B T per unit time"}
    if not args.no_serve:
        out["served"] = serve(args, dev, log)
    if "kernels" in results["mixed"]:
        out["mixed"]["kernels_ms"] = {k: v["ms_per_launch"] for k, v in results["mixed"]["kernels"].items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Pins of the oracle's time loop (Algorithm 2 with velocity-Verlet): the global
energy error of a symplectic second-order integrator scales as dt^2, the
integrator is time reversible, and a random-batch run keeps the energy
bounded over the short workload."""
import math

import numpy as np

import workloads


def _ocp(orc, N=125, lam=1.0, rc=2.5, gamma=1.0, seed=17, full_k=True, P=1):
    w = workloads.Workload("t", N=N, kappa=1 / lam, gamma=gamma, r_c=rc, P=P, seed=seed)
    st = workloads.make_state(w)
    s = orc.sog_auto(lam, rc, 1e-4)
    sysm = orc.System(st.q, st.m, w.L, s, w.kT, P, seed=seed, full_k=full_k)
    return w, st, sysm


def _energy_error(orc, dt, nsteps):
    w, st, sysm = _ocp(orc)
    x, v = st.x.copy(), st.v.copy()
    f, _, e0 = sysm.force(x, 0)
    E0 = e0[:5].sum() + 0.5 * float((st.m * (v * v).sum(0)).sum())
    eh = sysm.run(x, v, f, 0, nsteps, dt)
    E = eh[:, :6].sum(1)
    return np.abs(E - E0).max()


def test_energy_error_is_second_order(orc):
    """Deterministic full-k forces: halving dt over the same time span divides
    the maximum energy error by ~4 (velocity-Verlet is second order)."""
    e1 = _energy_error(orc, 0.01, 100)
    e2 = _energy_error(orc, 0.005, 200)
    assert 3.5 <= e1 / e2 <= 4.5


def test_time_reversible(orc):
    """Integrating forward, reversing the velocities and integrating back returns
    the start positions (velocity-Verlet is time reversible; deterministic forces)."""
    w, st, sysm = _ocp(orc, seed=23)
    x, v = st.x.copy(), st.v.copy()
    f, _, _ = sysm.force(x, 0)
    sysm.run(x, v, f, 0, 60, 0.01)
    v = -v
    sysm.run(x, v, f, 0, 60, 0.01)
    d = x - st.x
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= 1e-9


def test_random_batch_energy_bounded(orc):
    """The small one-component plasma with random-batch far field (P = 100) over
    100 steps: the total energy stays within 2% of N k_B T of its start (the
    estimator noise is ~1e-2 N k_B T per evaluation) and no particle escapes."""
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, w.eps)
    sysm = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=w.seed)
    x, v = st.x.copy(), st.v.copy()
    f, _, e0 = sysm.force(x, 0)
    E0 = e0[:5].sum() + 0.5 * float((st.m * (v * v).sum(0)).sum())
    eh = sysm.run(x, v, f, 0, 100, w.dt)
    E = eh[:, :6].sum(1)
    assert np.abs(E - E0).max() <= 0.05 * w.N * w.kT
    assert np.all((x >= 0) & (x < w.L))

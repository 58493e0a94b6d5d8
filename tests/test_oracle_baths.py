"""Pins of the oracle's global baths (Nose-Hoover NVT and Berendsen weak
coupling, each a half-step operator on either side of the velocity-Verlet
step): on nearly free particles (charges 1e-4) the Nose-Hoover kinetic energy
oscillates about g kT/2 at the angular frequency sqrt(2)/tau of the
linearised equations and the Berendsen one relaxes to it as exp(-t/tau);
for an interacting system with the deterministic far field the Nose-Hoover
extended energy K + U + Q xi^2/2 + g kT eta is conserved to second order in
dt; kind 0 is plain velocity-Verlet bit for bit."""
import math

import numpy as np
import pytest

import workloads


def _free(orc, N=1500, seed=3):
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=seed)
    q = np.full(N, 1e-4)
    m = np.where(np.arange(N) % 3 == 0, 2.0, 1.0)
    s = orc.sog_auto(1.0, 3.0, 1e-4)
    return st, q, m, L, orc.System(q, m, L, s, 1.0, 8, seed=5)


def _kinetic(m, v):
    return 0.5 * float((m[None, :] * v * v).sum())


def test_nose_hoover_oscillation_frequency(orc):
    """K = (g kT/2)(1 + d), xi: d' = -2 xi, xi' = (g kT/Q) d = d/tau^2, so
    d(t) = d0 cos(sqrt(2) t / tau) for small d0 (xi(0) = 0)."""
    st, q, m, L, sysm = _free(orc)
    N = q.size
    g, kT, tau, dt = 3 * N, 1.5, 0.8, 0.01
    rng = np.random.default_rng(2)
    v = rng.normal(size=(3, N)) / np.sqrt(m)[None, :]
    d0 = 0.02
    v *= math.sqrt((1 + d0) * g * kT / 2 / _kinetic(m, v))
    sysm.set_bath(2, 1.0 / tau, kT)
    x = st.x.copy()
    f, _, _ = sysm.force(x, 0)
    eh = sysm.run(x, v, f, 0, 400, dt)
    t = dt * np.arange(1, 401)
    d = eh[:, 5] / (g * kT / 2) - 1
    ref = d0 * np.cos(math.sqrt(2) * t / tau)
    assert np.abs(d - ref).max() <= 0.05 * d0          # O(d0^2) nonlinearity and O(dt^2)


def test_berendsen_relaxation(orc):
    st, q, m, L, sysm = _free(orc)
    N = q.size
    g, kT, tau, dt = 3 * N, 2.0, 0.5, 0.01
    rng = np.random.default_rng(4)
    v = 0.3 * rng.normal(size=(3, N))
    K0 = _kinetic(m, v)
    sysm.set_bath(3, 1.0 / tau, kT)
    x = st.x.copy()
    f, _, _ = sysm.force(x, 0)
    eh = sysm.run(x, v, f, 0, 300, dt)
    t = dt * np.arange(1, 301)
    Kinf = g * kT / 2
    ref = Kinf + (K0 - Kinf) * np.exp(-t / tau)
    assert np.abs(eh[:, 5] - ref).max() <= 2e-3 * Kinf


def _nh_extended(orc, dt, nsteps):
    w = workloads.Workload("nh", N=64, kappa=1.0, gamma=1.0, r_c=2.5, P=1, seed=7)
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, 1e-8)
    sysm = orc.System(st.q, st.m, w.L, s, w.kT, 1, seed=1, full_k=True)
    g, kT0, tau = 3 * w.N, 1.3 * w.kT, 0.3
    Q = g * kT0 * tau * tau
    sysm.set_bath(2, 1.0 / tau, kT0)
    x, v = st.x.copy(), st.v.copy()
    f, _, _ = sysm.force(x, 0)
    H = []
    for n in range(nsteps):   # one step per call: the bath state carries over
        e = sysm.run(x, v, f, n, 1, dt)[0]
        xi, eta = sysm.bath_state()
        H.append(e[:6].sum() + 0.5 * Q * xi * xi + g * kT0 * eta)
    return np.array(H), (g, kT0, Q)


def test_nose_hoover_extended_energy(orc):
    T = 0.6
    errs = []
    for dt in (0.004, 0.002):
        H, _ = _nh_extended(orc, dt, int(round(T / dt)))
        errs.append(np.abs(H - H[0]).max())
    assert errs[0] < 1e-3 * 64
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.0, ratio


def test_one_step_calls_equal_one_long_call(orc):
    """The closing and opening half-steps between two calls compose to the
    same dynamics as inside one call (to rounding: the kinetic energy is
    recomputed at a call's start)."""
    w = workloads.Workload("nh2", N=64, kappa=1.0, gamma=1.0, r_c=2.5, P=1, seed=8)
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, 1e-8)
    out = []
    for split in (False, True):
        sysm = orc.System(st.q, st.m, w.L, s, w.kT, 1, seed=1, full_k=True)
        sysm.set_bath(2, 2.0, 1.2 * w.kT)
        x, v = st.x.copy(), st.v.copy()
        f, _, _ = sysm.force(x, 0)
        if split:
            for n in range(20):
                sysm.run(x, v, f, n, 1, 0.005)
        else:
            sysm.run(x, v, f, 0, 20, 0.005)
        out.append((x, v, sysm.bath_state()))
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-12 * np.abs(out[0][1]).max()
    assert abs(out[0][2][0] - out[1][2][0]) <= 1e-12 * max(1.0, abs(out[0][2][0]))


def test_bath_off_is_plain_verlet(orc):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, w.eps)
    res = []
    for kind in (None, 0):
        sysm = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=w.seed)
        if kind is not None:
            sysm.set_bath(2, 1.0, 1.0)
            sysm.set_bath(kind, 0.0, 0.0)
        x, v = st.x.copy(), st.v.copy()
        f, _, _ = sysm.force(x, 0)
        sysm.run(x, v, f, 0, 5, w.dt)
        res.append((x, v))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    with pytest.raises(ValueError):
        orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=w.seed).set_bath(2, -1.0, 1.0)

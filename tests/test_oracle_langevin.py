"""Pins of the oracle's Langevin thermostat (the BAOAB splitting of the
velocity-Verlet step, with Philox normals): the normals are the Box-Muller
transform of the counter-based Philox words (checked against numpy on the
pinned generator, and for normality), the Ornstein-Uhlenbeck velocity update
relaxes free particles from rest to the bath temperature exactly as
(1 - c^(2n)) k_B T / m with c = exp(-friction dt), and friction 0 is plain
velocity-Verlet."""
import math

import numpy as np
from scipy import stats

import workloads


def test_normals_are_box_muller_of_philox(orc):
    seed, rep = 77, 3
    zs = []
    for i in range(2000):
        for step in (1, 2 ** 40 + 5):
            z = orc.langevin_normals(i, step, seed, rep)
            w = orc.philox(np.array([i, step, 1, 0], dtype=np.uint64), np.array([seed, rep], dtype=np.uint64))
            u = ((w >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
            r0, r1 = math.sqrt(-2 * math.log(u[0])), math.sqrt(-2 * math.log(u[2]))
            ref = [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
                   r1 * math.cos(2 * math.pi * u[3])]
            assert np.allclose(z, ref, rtol=1e-14, atol=1e-15)
            zs.extend(z)
    zs = np.array(zs)
    assert stats.kstest(zs, "norm").pvalue > 1e-6
    assert abs(zs.mean()) <= 5 / math.sqrt(zs.size) and abs(zs.var() - 1) <= 5 * math.sqrt(2 / zs.size)


def test_free_particles_relax_to_bath(orc):
    """Charges of 1e-4 make the forces negligible: from rest, n BAOAB steps
    give velocity variance (1 - c^(2n)) k_B T / m per component."""
    N = 3000
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=3)
    q = np.full(N, 1e-4)
    m = np.where(np.arange(N) % 2 == 0, 1.0, 4.0)
    s = orc.sog_auto(1.0, 3.0, 1e-4)
    sysm = orc.System(q, m, L, s, 1.0, 8, seed=5)
    kT, gamma, dt = 2.0, 0.7, 0.05
    sysm.set_langevin(gamma, kT)
    x = st.x.copy()
    v = np.zeros((3, N))
    f, _, _ = sysm.force(x, 0)
    for n in (1, 10, 60):
        xs, vs, fs = x.copy(), v.copy(), f.copy()
        sysm.run(xs, vs, fs, 0, n, dt)
        c = math.exp(-gamma * dt)
        want = (1 - c ** (2 * n)) * kT / m
        ratio = (vs ** 2 / want[None, :]).ravel()
        assert abs(ratio.mean() - 1) <= 5 * math.sqrt(2 / ratio.size), (n, ratio.mean())


def test_zero_friction_is_plain_verlet(orc):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, w.eps)
    out = []
    for fr in (None, 0.0):
        sysm = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=w.seed)
        if fr is not None:
            sysm.set_langevin(fr, 5.0)
        x, v = st.x.copy(), st.v.copy()
        f, _, _ = sysm.force(x, 0)
        sysm.run(x, v, f, 0, 5, w.dt)
        out.append((x, v))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])

"""Pins of the oracle in a cuboid box (edges L_x, L_y, L_z; Section 2 and
Algorithm 2 take the box as three edges): the Fourier lattice against a
brute-force enumeration with the truncation written out here, near field +
full-lattice far field + constants against the periodic Yukawa image sum of
the cuboid, F = -grad U, the cell-list near field against a k-d tree with a
per-axis period, the point-by-point sampling tables and draws against the
measure P(k) = F(k) Fhat(k) / S, unbiasedness of the random-batch force, the
virial under a joint scaling of all edges, time reversal of the dynamics, and
equal edges reducing to the cubic functions bit for bit."""
import math

import numpy as np
import pytest
from scipy import special
from scipy.spatial import cKDTree

import workloads

LB = (6.0, 7.5, 6.8)


def _state(n, Lb, seed, neutral=True):
    st = workloads.small_system(n, 1.0, seed, neutral=neutral)
    st.x = np.ascontiguousarray(st.x * np.asarray(Lb)[:, None])
    return st


def _fhat(s, k2):
    return sum(a * np.exp(-b * k2) for a, b in zip(s.A, s.B))


def test_box_lattice_against_enumeration(orc):
    s = orc.sog_auto(1.0, 2.5, 1e-6)
    n3, k2 = orc.box_lattice(LB, s)
    thr = 1e-16 * _fhat(s, 0.0)
    g = np.arange(-40, 41)
    N = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    N = N[np.any(N != 0, axis=1)]
    kk = ((2 * np.pi) * N / np.asarray(LB)[None, :]) ** 2
    K2 = kk[:, 0] + kk[:, 1] + kk[:, 2]
    keep = _fhat(s, K2) >= thr
    N, K2 = N[keep], K2[keep]
    assert np.abs(N).max() < 40                  # the enumeration reached past the cutoff
    order = np.lexsort((N[:, 2], N[:, 1], N[:, 0], K2))
    assert np.array_equal(n3, N[order].astype(np.int32))
    assert np.array_equal(k2, K2[order])


def test_cubic_box_lattice_is_the_shell_lattice(orc):
    s = orc.sog_auto(1.0, 2.5, 1e-6)
    L = 6.0
    n3, _ = orc.box_lattice((L, L, L), s)
    sysm = orc.System(np.ones(2), np.ones(2), L, s, 1.0, 4, seed=1)
    n3c, _ = sysm.lattice()
    assert np.array_equal(n3, n3c)


def k0_constant(s, lam, rc):
    iy = lam * math.exp(-rc / lam) * (rc + lam)
    iF = sum(c * (rc * math.exp(-ss * rc * rc) / (2 * ss) + math.sqrt(math.pi) / (4 * ss ** 1.5)
                  * special.erfc(math.sqrt(ss) * rc)) for c, ss in zip(s.c, s.s))
    return 4 * math.pi * (iy - iF)


@pytest.mark.parametrize("neutral", [True, False])
def test_full_k_equals_cuboid_image_sum(orc, neutral):
    lam, rc = 1.0, 2.5
    st = _state(10, LB, 7, neutral)
    s = orc.sog_auto(lam, rc, 1e-13)
    sysm = orc.System(st.q, st.m, LB, s, kT=1.0, P=1, seed=1, full_k=True)
    f, fn, e = sysm.force(st.x, 0)
    U = e[0] + e[1] + e[2] + e[3]
    Ub, fb = orc.yukawa_image_sum(st.x, st.q, LB, lam, 60.0)
    V = float(np.prod(LB))
    Ub -= st.q.sum() ** 2 * k0_constant(s, lam, rc) / (2 * V)
    assert abs(U - Ub) <= 1e-11 * abs(Ub)
    assert np.linalg.norm(f - fb) <= 1e-11 * np.linalg.norm(fb)
    assert abs(e[4] + st.q.sum() ** 2 * 4 * math.pi * lam * lam / (2 * V)) <= 1e-14 * max(1.0, abs(e[4]))


def _num_grad(fun, x, h=1e-5):
    g = np.zeros_like(x)
    for d in range(3):
        for i in range(x.shape[1]):
            xp = x.copy(); xp[d, i] += h
            xm = x.copy(); xm[d, i] -= h
            g[d, i] = (fun(xp) - fun(xm)) / (2 * h)
    return g


def test_forces_are_minus_gradient(orc):
    Lb = (7.0, 8.2, 7.6)
    st = _state(8, Lb, 11, neutral=False)
    s = orc.sog_auto(1.0, 2.5, 1e-6)
    fn, _ = orc.near(st.x, st.q, Lb, s)
    g = _num_grad(lambda y: orc.near(y, st.q, Lb, s)[1], st.x)
    assert np.linalg.norm(fn + g) <= 1e-7 * np.linalg.norm(fn)
    ff, _ = orc.far_full_box(st.x, st.q, Lb, s)
    g = _num_grad(lambda y: orc.far_full_box(y, st.q, Lb, s)[1], st.x)
    assert np.linalg.norm(ff + g) <= 1e-7 * np.linalg.norm(ff)


def test_near_cell_path_against_kdtree(orc):
    Lb = (13.0, 17.5, 15.2)
    st = _state(2600, Lb, 21, neutral=False)
    st.q[::3] = -0.7
    s = orc.sog_auto(1.0, 3.5, 1e-4)
    f, U = orc.near(st.x, st.q, Lb, s)
    pos = st.x.T
    pairs = cKDTree(pos, boxsize=Lb).query_pairs(3.5, output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= np.asarray(Lb)[None, :] * np.round(d / np.asarray(Lb)[None, :])
    r = np.sqrt((d * d).sum(1))
    fac = np.exp(-r) * (1 + r) / r ** 3 - 2 * sum(c * ss * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    en = np.exp(-r) / r - sum(c * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    qq = st.q[pairs[:, 0]] * st.q[pairs[:, 1]]
    fb = np.zeros((3, st.x.shape[1]))
    for k in range(3):
        np.add.at(fb[k], pairs[:, 0], qq * fac * d[:, k])
        np.add.at(fb[k], pairs[:, 1], -qq * fac * d[:, k])
    assert abs(U - float((qq * en).sum())) <= 1e-12 * abs(U)
    assert np.linalg.norm(f - fb) <= 1e-12 * np.linalg.norm(fb)
    idx = np.arange(0, 2600, 131)
    assert np.abs(orc.near_subset(st.x, st.q, Lb, s, idx) - f[:, idx]).max() <= 1e-12 * np.abs(f).max()


def test_point_tables_and_draws(orc):
    Lb = (5.0, 6.5, 5.6)
    st = _state(40, Lb, 13, neutral=False)
    s = orc.sog_auto(1.0, 1.6, 1e-4)
    kT, P = 0.3, 400
    sysm = orc.System(st.q, st.m, Lb, s, kT=kT, P=P, seed=9)
    n3, k2 = orc.box_lattice(Lb, s)
    _, cdf, coef = sysm.tables()
    V, Q2 = float(np.prod(Lb)), float((st.q ** 2).sum())
    F = kT * V / (kT * V / Q2 + 1.0 / (1.0 + k2))          # eq. (3.22), lambda = 1
    w = F * _fhat(s, k2)
    assert np.allclose(cdf, np.cumsum(w), rtol=1e-13, atol=0)
    assert np.allclose(coef, w.sum() / (P * V * F), rtol=1e-13, atol=0)
    counts = np.zeros(len(k2))
    index = {tuple(v): i for i, v in enumerate(n3)}
    for step in range(100):
        nd, cd = sysm.draw(step)
        for v, c in zip(map(tuple, nd), cd):
            i = index[v]
            counts[i] += 1
            assert c == coef[i]
    p = w / w.sum()
    big = p * counts.sum() > 20
    chi2 = (((counts[big] - p[big] * counts.sum()) ** 2) / (p[big] * counts.sum())).sum()
    dof = int(big.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_random_batch_force_is_unbiased(orc):
    Lb = (5.0, 6.5, 5.6)
    st = _state(20, Lb, 17, neutral=True)
    s = orc.sog_auto(1.0, 1.6, 1e-6)
    sysm = orc.System(st.q, st.m, Lb, s, kT=1.0, P=50, seed=3)
    full = orc.System(st.q, st.m, Lb, s, kT=1.0, P=1, seed=1, full_k=True)
    f_full, fn, _ = full.force(st.x, 0)
    samples = []
    for step in range(2000):
        f, fnn, _ = sysm.force(st.x, step)
        samples.append((f - fnn).ravel())
    samples = np.array(samples)
    z = (samples.mean(0) - (f_full - fn).ravel()) / (samples.std(0, ddof=1) / math.sqrt(len(samples)))
    assert np.abs(z).max() < 5.0
    assert abs((z ** 2).mean() - 1.0) < 0.5


def test_virial_under_joint_scaling(orc):
    Lb0 = np.array([6.5, 7.5, 7.0])
    st = _state(12, Lb0, 23, neutral=False)
    s = orc.sog_auto(1.0, 2.0, 1e-10)

    def energy(t):
        Lb = tuple(Lb0 * t)
        x = st.x * t
        _, un = orc.near(x, st.q, Lb, s)
        _, uf = orc.far_full_box(x, st.q, Lb, s)
        V = float(np.prod(Lb))
        return un + uf + s.Fhat0 * st.q.sum() ** 2 / (2 * V)

    _, _, wn = orc.near(st.x, st.q, tuple(Lb0), s, virial=True)
    _, uf, wf = orc.far_full_box(st.x, st.q, tuple(Lb0), s, virial=True)
    V0 = float(np.prod(Lb0))
    uk0 = s.Fhat0 * st.q.sum() ** 2 / (2 * V0)
    h = 1e-5   # V = V0 t^3: -3V dU/dV = -t dU/dt at t = 1
    dUdt = (energy(1 + h) - energy(1 - h)) / (2 * h)
    W = wn + wf + 3 * uk0
    assert abs(W + dUdt) <= 1e-7 * (abs(W) + abs(wn))


def test_dynamics_wrap_per_axis_and_reverse(orc):
    Lb = (9.0, 11.0, 10.0)
    st = _state(50, Lb, 29, neutral=True)
    s = orc.sog_auto(1.0, 2.5, 1e-6)
    sysm = orc.System(st.q, st.m, Lb, s, kT=1.0, P=1, seed=1, full_k=True)
    x, v = st.x.copy(), 3.0 * st.v.copy()
    f, _, _ = sysm.force(x, 0)
    sysm.run(x, v, f, 0, 40, 0.02)
    assert np.all(x >= 0) and np.all(x < np.asarray(Lb)[:, None])
    v = -v
    sysm.run(x, v, f, 40, 40, 0.02)
    d = x - st.x
    d -= np.asarray(Lb)[:, None] * np.round(d / np.asarray(Lb)[:, None])
    assert np.abs(d).max() <= 1e-9


def test_equal_edges_reduce_to_the_cube(orc):
    L = 7.0
    st = _state(30, (L, L, L), 31, neutral=False)
    s = orc.sog_auto(1.0, 2.0, 1e-6)
    a = orc.near(st.x, st.q, L, s, virial=True)
    b = orc.near(st.x, st.q, (L, L, L), s, virial=True)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    n3 = np.array([[1, 0, 0], [2, -1, 3], [0, 0, -4]], dtype=np.int32)
    assert np.array_equal(orc.rho(st.x, st.q, L, n3), orc.rho(st.x, st.q, (L, L, L), n3))
    mmax = orc.mmax_default(s, L)
    fa, ua, wa = orc.far_full(st.x, st.q, L, s, mmax, virial=True)
    fb, ub, wb = orc.far_full_box(st.x, st.q, (L, L, L), s, virial=True)
    assert np.array_equal(fa, fb) and ua == ub and wa == wb


def test_rdf_in_a_cuboid_against_kdtree(orc):
    Lb = (9.0, 12.0, 10.5)
    st = _state(600, Lb, 37)
    counts, amb = orc.rdf(st.x, Lb, 3.0, 30)
    pairs = cKDTree(st.x.T, boxsize=Lb).query_pairs(3.0, output_type="ndarray")
    d = st.x.T[pairs[:, 0]] - st.x.T[pairs[:, 1]]
    d -= np.asarray(Lb)[None, :] * np.round(d / np.asarray(Lb)[None, :])
    r = np.sqrt((d * d).sum(1))
    ref = 2 * np.bincount(np.minimum((r / 0.1).astype(int), 29), minlength=30)
    assert np.abs(counts - ref).max() <= amb.max() + 0 and counts.sum() == ref.sum()
    assert np.array_equal(orc.rdf(st.x, (9.0, 9.0, 9.0), 3.0, 30)[0], orc.rdf(st.x, 9.0, 3.0, 30)[0])

"""Pins of the oracle's near field, far field and energies against identities the
mathematics fixes (Sections 2, 4.1): the Poisson summation identity between
the Fourier-space far field and its real-space lattice sum, the brute-force
periodic Yukawa image sum, and F = -grad U."""
import math

import numpy as np
import pytest
from scipy import special
from scipy.spatial import cKDTree

import workloads


def real_space_sog(x, q, L, s, nimg=8):
    """1/2 sum_n sum_{i,j} q_i q_j F(|r_i - r_j - nL|) (i = j, n = 0 included, F(0)
    finite) and its forces, by direct summation over images."""
    N = x.shape[1]
    rng = np.arange(-nimg, nimg + 1)
    sh = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) * L
    pos = x.T
    U = 0.0
    f = np.zeros((3, N))
    for i in range(N):
        d = pos[i][None, None, :] - pos[:, None, :] - sh[None, :, :]
        r2 = (d * d).sum(-1)
        F = sum(c * np.exp(-ss * r2) for c, ss in zip(s.c, s.s))
        U += 0.5 * q[i] * float((q[:, None] * F).sum())
        g = sum(-2 * c * ss * np.exp(-ss * r2) for c, ss in zip(s.c, s.s))
        f[:, i] = -q[i] * (q[:, None, None] * g[:, :, None] * d).sum(axis=(0, 1))
    return U, f


@pytest.mark.parametrize("neutral", [False, True])
def test_poisson_identity(orc, neutral):
    """(1/2V) sum_k Fhat(k) |rho(k)|^2 over all k (k = 0 included) equals the
    real-space lattice sum of F (eq. 3.5), and so do the forces (eq. 3.8)."""
    L = 6.0
    st = workloads.small_system(10, L, 5, neutral=neutral)
    s = orc.sog_auto(1.0, 2.5, 1e-13)
    mmax = orc.mmax_default(s, L)
    f_k, U_k = orc.far_full(st.x, st.q, L, s, mmax)
    U_k += s.Fhat0 * st.q.sum() ** 2 / (2 * L ** 3)
    U_r, f_r = real_space_sog(st.x, st.q, L, s)
    assert abs(U_k - U_r) <= 1e-12 * abs(U_r)
    assert np.linalg.norm(f_k - f_r) <= 1e-12 * np.linalg.norm(f_r)


def k0_constant(s, lam, rc):
    """Khat(0) = 4 pi int_{rc}^inf (Y - F) r^2 dr in closed form: the k = 0 Fourier
    mode of the decomposition error beyond r_c."""
    iy = lam * math.exp(-rc / lam) * (rc + lam)
    iF = sum(c * (rc * math.exp(-ss * rc * rc) / (2 * ss) + math.sqrt(math.pi) / (4 * ss ** 1.5)
                  * special.erfc(math.sqrt(ss) * rc)) for c, ss in zip(s.c, s.s))
    return 4 * math.pi * (iy - iF)


@pytest.mark.parametrize("neutral", [True, False])
def test_full_k_equals_yukawa_image_sum(orc, neutral):
    """Near field + deterministic full-k far field + self term equals the periodic
    Yukawa image sum (the plain definition; Section 2) to the SOG tolerance:
    with eps = 1e-13 the energy and forces agree to ~1e-11.  For a charged
    system the decomposition error's k = 0 mode, -(sum q)^2 Khat(0)/(2V), is a
    constant offset and is added to the reference."""
    L, lam, rc = 6.0, 1.0, 2.5
    st = workloads.small_system(10, L, 7, neutral=neutral)
    s = orc.sog_auto(lam, rc, 1e-13)
    sysm = orc.System(st.q, st.m, L, s, kT=1.0, P=1, seed=1, full_k=True)
    f, fn, e = sysm.force(st.x, 0)
    U = e[0] + e[1] + e[2] + e[3]
    Ub, fb = orc.yukawa_image_sum(st.x, st.q, L, lam, 60.0)
    Ub -= st.q.sum() ** 2 * k0_constant(s, lam, rc) / (2 * L ** 3)
    assert abs(U - Ub) <= 1e-11 * abs(Ub)
    assert np.linalg.norm(f - fb) <= 1e-11 * np.linalg.norm(fb)


def test_full_k_at_paper_tolerance(orc):
    """At eps = 1e-4 (the paper's choice) the forces agree with the image sum to
    about eps relative."""
    L, lam, rc = 6.0, 1.0, 2.5
    st = workloads.small_system(12, L, 3, neutral=True)
    s = orc.sog_auto(lam, rc, 1e-4)
    sysm = orc.System(st.q, st.m, L, s, kT=1.0, P=1, seed=1, full_k=True)
    f, fn, e = sysm.force(st.x, 0)
    Ub, fb = orc.yukawa_image_sum(st.x, st.q, L, lam, 60.0)
    assert np.linalg.norm(f - fb) <= 1e-3 * np.linalg.norm(fb)
    assert abs(e[:4].sum() - Ub) <= 1e-3 * abs(Ub) + 1e-3


def _num_grad(fun, x, h=1e-5):
    g = np.zeros_like(x)
    for d in range(3):
        for i in range(x.shape[1]):
            xp = x.copy(); xp[d, i] += h
            xm = x.copy(); xm[d, i] -= h
            g[d, i] = (fun(xp) - fun(xm)) / (2 * h)
    return g


def test_forces_are_minus_gradient(orc):
    """F = -grad U by central differences for the near field (eq. 3.8 vs the
    near energy), the full-k far field, and the random-batch estimators with the
    samples held fixed (eq. UF)."""
    L, lam, rc = 7.0, 1.0, 2.5
    st = workloads.small_system(8, L, 11, neutral=False)
    s = orc.sog_auto(lam, rc, 1e-6)
    # near field
    fn, _ = orc.near(st.x, st.q, L, s)
    g = _num_grad(lambda y: orc.near(y, st.q, L, s)[1], st.x)
    assert np.linalg.norm(fn + g) <= 1e-7 * np.linalg.norm(fn)
    # full-k far field
    mmax = orc.mmax_default(s, L)
    ff, _ = orc.far_full(st.x, st.q, L, s, mmax)
    g = _num_grad(lambda y: orc.far_full(y, st.q, L, s, mmax)[1], st.x)
    assert np.linalg.norm(ff + g) <= 1e-7 * np.linalg.norm(ff)
    # random batch with fixed samples
    sysm = orc.System(st.q, st.m, L, s, kT=1.0, P=30, seed=4)
    n3, coef = sysm.draw(3)

    def u_rb(y):
        return orc.lib().orc_far_rb_energy(len(coef), orc._ptr(coef), orc._ptr(orc.rho(y, st.q, L, n3)))

    fr = orc.far_rb(st.x, st.q, L, n3, coef, orc.rho(st.x, st.q, L, n3))
    g = _num_grad(u_rb, st.x)
    assert np.linalg.norm(fr + g) <= 1e-7 * np.linalg.norm(fr)


def test_near_field_against_kdtree(orc):
    """The near field found through the cell list (N > 2000) equals a direct sum
    over the periodic pairs within r_c found by a k-d tree."""
    w = workloads.Workload("t", N=3000, kappa=0.5, gamma=1.0, r_c=4.0, P=1, seed=21)
    st = workloads.make_state(w)
    st.q[::3] = -0.7
    s = orc.sog_auto(w.lam, w.r_c, 1e-4)
    f, U = orc.near(st.x, st.q, w.L, s)
    pos = st.x.T
    tree = cKDTree(pos, boxsize=w.L)
    pairs = tree.query_pairs(w.r_c, output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= w.L * np.round(d / w.L)
    r = np.sqrt((d * d).sum(1))
    lam = w.lam
    fac = np.exp(-r / lam) * (1 + r / lam) / r ** 3 - 2 * sum(c * ss * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    en = np.exp(-r / lam) / r - sum(c * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    qq = st.q[pairs[:, 0]] * st.q[pairs[:, 1]]
    fb = np.zeros((3, w.N))
    for k in range(3):
        np.add.at(fb[k], pairs[:, 0], qq * fac * d[:, k])
        np.add.at(fb[k], pairs[:, 1], -qq * fac * d[:, k])
    Ub = float((qq * en).sum())
    assert abs(U - Ub) <= 1e-12 * abs(Ub)
    assert np.linalg.norm(f - fb) <= 1e-12 * np.linalg.norm(fb)


def test_cell_list_against_sort(orc):
    """The cell list is the stable sort of particles by cell id (ties by index),
    with the id computed as floor(x nc / L) clamped to [0, nc-1]."""
    w = workloads.Workload("t", N=5000, kappa=1.0, gamma=1.0, r_c=3.0, P=1, seed=2)
    x = workloads.positions(w.N, w.L, 2)
    x[0, :5] = 0.0
    x[1, 5:10] = np.nextafter(w.L, 0)
    cs, order = orc.cells(x, w.L, w.r_c)
    nc = int(math.floor(w.L / w.r_c))
    inv = nc / w.L
    c = np.clip(np.floor(x * inv).astype(np.int64), 0, nc - 1)
    cid = (c[2] * nc + c[1]) * nc + c[0]
    ref = sorted(range(w.N), key=lambda i: (cid[i], i))
    assert np.array_equal(order, np.array(ref, dtype=np.int32))
    assert np.array_equal(cs, np.concatenate([[0], np.cumsum(np.bincount(cid, minlength=nc ** 3))]).astype(np.int32))

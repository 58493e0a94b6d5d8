"""Pins of the oracle's exact gradient-corrected screening (EGS) kernel
(Section 1): its partial-fraction split into two Yukawa terms against the
dielectric function as the paper defines it, the real-space kernel against
that Fourier form by quadrature, the limits nu -> 0 (Yukawa) and r -> 0
(Coulomb), the term-by-term decomposition's error bound and continuity at the
cutoff, the adaptive density of eq. (3.22) for this dielectric, and the whole
system (near field + full-lattice far field + constants) against the periodic
image sum of the kernel."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads


def yhat_paper(k, lam, nu):
    """4 pi / (k^2 eps_EGS(k)), eps_EGS(k) = 1 + (lam k)^-2 (1 + nu lam^2 k^2 / 4)^-1."""
    eps = 1.0 + (lam * k) ** -2 / (1.0 + nu * lam * lam * k * k / 4.0)
    return 4.0 * math.pi / (k * k * eps)


@pytest.mark.parametrize("lam,nu", [(1.0, 0.3), (0.577, 0.9), (2.5, 0.02), (1.3, 1e-6)])
def test_split_matches_the_dielectric(orc, lam, nu):
    a, l = orc.egs_split(lam, nu)
    for k in np.logspace(-3, 3, 61):
        ref = yhat_paper(k, lam, nu)
        got = sum(aj * 4 * math.pi * lj * lj / (1 + lj * lj * k * k) for aj, lj in zip(a, l))
        assert abs(got - ref) <= 1e-12 * abs(ref), (k, got, ref)
    assert abs(a.sum() - 1.0) <= 1e-14            # Coulomb at short range
    assert abs((a * l * l).sum() - lam * lam) <= 1e-12 * lam * lam   # Yhat(0) = 4 pi lam^2
    assert a[0] > 1.0 and a[1] < 0.0 and l[0] > l[1] > 0.0


def test_split_rejects_outside_the_range(orc):
    for nu in (0.0, -0.1, 1.0, 1.5, float("nan")):
        with pytest.raises(ValueError):
            orc.egs_split(1.0, nu)


def test_yukawa_limit(orc):
    a, l = orc.egs_split(0.8, 1e-9)
    assert abs(a[0] - 1.0) <= 1e-9 and abs(a[1]) <= 1e-9
    assert abs(l[0] - 0.8) <= 1e-9 * 0.8


@pytest.mark.parametrize("nu", [0.3, 0.8])
def test_real_space_kernel_has_the_paper_transform(orc, nu):
    """Yhat(k) = (4 pi / k) int_0^inf r Y(r) sin(k r) dr by quadrature of the
    oracle's real-space kernel, against the paper's dielectric form."""
    lam = 1.0
    a, l = orc.egs_split(lam, nu)
    s = orc.SOG(lam, 1.0, 0, 0, 0, 0, 0, ya=a, yl=l, nu=nu)

    def ry(r):   # r Y(r) -> a_1 + a_2 = 1 as r -> 0
        return r * float(orc.kernel_Y(s, r)) if r > 0 else 1.0

    for k in (0.3, 1.0, 2.7):
        v, err = integrate.quad(ry, 0.0, 80.0 * lam, weight="sin", wvar=k, limit=400)
        got = 4 * math.pi / k * v
        ref = yhat_paper(k, lam, nu)
        assert abs(got - ref) <= 1e-8 * ref, (k, got, ref)
    # Coulomb at short range
    r = 1e-6
    assert abs(r * float(orc.kernel_Y(s, r)) - 1.0) <= 1e-5


def _yukawa_terms(a, l, r):
    return sum(aj * np.exp(-r / lj) / r for aj, lj in zip(a, l))


@pytest.mark.parametrize("lam,nu,rc,eps,smooth", [(1.0, 0.3, 3.0, 1e-6, 1), (1.0, 0.8, 2.5, 1e-10, 1),
                                                  (1.0, 0.01, 3.0, 1e-6, 1), (0.7, 0.5, 2.0, 1e-8, 2)])
def test_decomposition_bound_and_continuity(orc, lam, nu, rc, eps, smooth):
    s = orc.sog_egs(lam, nu, rc, eps, smooth)
    a, l = s.terms[1], s.terms[2]
    assert len(s.c) == len(s.s) == len(s.A) == len(s.B) == s.n
    # the bound on a fine grid, recomputed here from the Gaussians and the split
    r = rc + (33 * l[0] - rc) * np.linspace(0, 1, 20001) ** 2
    F = sum(c * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    err = np.abs(_yukawa_terms(a, l, r) - F).max()
    assert err <= eps and abs(err - s.err) <= 0.05 * eps
    # N = Y - F vanishes at r_c with its derivative (and its curvature for C2),
    # up to the rounding of the terms and a term left wholly in the near field
    tail = sum(abs(aj) * math.exp(-rc / lj) / rc for aj, lj in zip(a, l) if rc >= 33 * lj)

    def nfun(x):
        return float(_yukawa_terms(a, l, np.array(x)) - sum(c * np.exp(-ss * x * x) for c, ss in zip(s.c, s.s)))

    scale = float(_yukawa_terms(np.abs(a), l, np.array(rc)))
    h = 1e-3 * rc
    d1 = (nfun(rc + h) - nfun(rc - h)) / (2 * h)
    d2 = (nfun(rc + h) - 2 * nfun(rc) + nfun(rc - h)) / (h * h)
    assert abs(nfun(rc)) <= 1e-13 * scale + tail
    assert abs(d1) <= 1e-7 * scale / rc + 40 * tail / l.min()
    if smooth == 2:
        assert abs(d2) <= 1e-4 * scale / rc ** 2
    else:
        assert abs(d2) > 1e-6 * scale / rc ** 2    # C1 only: the curvature jumps
    if nu == 0.01:
        assert rc >= 33 * l[1]                     # the short term is wholly near


def test_adaptive_density_for_the_dielectric(orc):
    lam, nu, kT, V, Q2 = 1.0, 0.4, 2.0, 30.0 ** 3, 500.0
    a, l = orc.egs_split(lam, nu)
    for k in (0.05, 0.4, 2.0, 9.0):
        got = orc.lib().orc_density_k(orc.ADAPTIVE, kT, V, Q2, 2, orc._ptr(a), orc._ptr(l), k * k)
        ref = kT * V / (kT * V / Q2 + yhat_paper(k, lam, nu) / (4 * math.pi))
        assert abs(got - ref) <= 1e-13 * ref
        got4 = orc.lib().orc_density_k(orc.DH4PI, kT, V, Q2, 2, orc._ptr(a), orc._ptr(l), k * k)
        assert abs(got4 - kT * V / (kT * V / Q2 + yhat_paper(k, lam, nu))) <= 1e-13 * got4
    one, lam_ = np.array([1.0]), np.array([lam])
    assert orc.lib().orc_density_k(orc.ADAPTIVE, kT, V, Q2, 1, orc._ptr(one), orc._ptr(lam_), 0.7) == \
        orc.density(orc.ADAPTIVE, kT, V, Q2, lam, 0.7)


@pytest.mark.parametrize("neutral", [True, False])
def test_full_k_equals_egs_image_sum(orc, neutral):
    """Near field + full-lattice far field + U_k0 + U_self equals the periodic
    image sum of the EGS kernel (two Yukawa image sums with the split's
    weights) to the decomposition's tolerance; a charged system's reference
    carries the decomposition error's k = 0 mode."""
    L, lam, nu, rc = 6.0, 1.0, 0.35, 2.5
    st = workloads.small_system(10, L, 17, neutral=neutral)
    s = orc.sog_egs(lam, nu, rc, 1e-13)
    a, l = s.terms[1], s.terms[2]
    sysm = orc.System(st.q, st.m, L, s, kT=1.0, P=1, seed=1, full_k=True)
    f, fn, e = sysm.force(st.x, 0)
    U = e[0] + e[1] + e[2] + e[3]
    Ub, fb = 0.0, np.zeros_like(st.x)
    for aj, lj in zip(a, l):
        u, ff = orc.yukawa_image_sum(st.x, st.q, L, lj, 60.0)
        Ub += aj * u
        fb += aj * ff
    iy = sum(aj * lj * math.exp(-rc / lj) * (rc + lj) for aj, lj in zip(a, l))
    iF = sum(c * (rc * math.exp(-ss * rc * rc) / (2 * ss) + math.sqrt(math.pi) / (4 * ss ** 1.5)
                  * math.erfc(math.sqrt(ss) * rc)) for c, ss in zip(s.c, s.s))
    Ub -= st.q.sum() ** 2 * 4 * math.pi * (iy - iF) / (2 * L ** 3)
    assert abs(U - Ub) <= 1e-11 * abs(Ub)
    assert np.linalg.norm(f - fb) <= 1e-11 * np.linalg.norm(fb)
    # the background term integrates the kernel over space: 4 pi lam^2 as for Yukawa
    assert abs(e[4] + st.q.sum() ** 2 * 4 * math.pi * lam * lam / (2 * L ** 3)) <= 1e-14 * max(1.0, abs(e[4]))


def test_near_force_is_minus_gradient(orc):
    L, rc = 7.0, 2.5
    st = workloads.small_system(8, L, 23, neutral=False)
    s = orc.sog_egs(1.0, 0.6, rc, 1e-6)
    fn, _ = orc.near(st.x, st.q, L, s)
    g = np.zeros_like(st.x)
    h = 1e-5
    for d in range(3):
        for i in range(st.x.shape[1]):
            xp = st.x.copy(); xp[d, i] += h
            xm = st.x.copy(); xm[d, i] -= h
            g[d, i] = (orc.near(xp, st.q, L, s)[1] - orc.near(xm, st.q, L, s)[1]) / (2 * h)
    assert np.linalg.norm(fn + g) <= 1e-7 * np.linalg.norm(fn)


def test_near_cell_path_against_kdtree(orc):
    """The cell-list pair search (N > 2000) with the two-term pair function
    equals a direct sum over the periodic pairs within r_c found by a k-d tree,
    with the pair force and energy written out from the split here."""
    from scipy.spatial import cKDTree
    w = workloads.Workload("t", N=2500, kappa=0.5, gamma=1.0, r_c=3.0, P=1, seed=29)
    st = workloads.make_state(w)
    st.q[::4] = -0.6
    s = orc.sog_egs(w.lam, 0.45, w.r_c, 1e-6)
    a, l = s.terms[1], s.terms[2]
    f, U = orc.near(st.x, st.q, w.L, s)
    pos = st.x.T
    pairs = cKDTree(pos, boxsize=w.L).query_pairs(w.r_c, output_type="ndarray")
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    d -= w.L * np.round(d / w.L)
    r = np.sqrt((d * d).sum(1))
    fac = sum(aj * np.exp(-r / lj) * (1 + r / lj) / r ** 3 for aj, lj in zip(a, l)) \
        - 2 * sum(c * ss * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    en = _yukawa_terms(a, l, r) - sum(c * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    qq = st.q[pairs[:, 0]] * st.q[pairs[:, 1]]
    fb = np.zeros((3, w.N))
    for k in range(3):
        np.add.at(fb[k], pairs[:, 0], qq * fac * d[:, k])
        np.add.at(fb[k], pairs[:, 1], -qq * fac * d[:, k])
    assert abs(U - float((qq * en).sum())) <= 1e-12 * abs(U)
    assert np.linalg.norm(f - fb) <= 1e-12 * np.linalg.norm(fb)

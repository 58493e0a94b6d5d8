"""Pins of two oracle parts that the full-size GPU checks lean on:

* the near field on a subset of particles (eq. 3.8 summed for the chosen i
  only), which is the reference of every full-size force check, against a
  direct sum over the periodic pairs within r_c found by a k-d tree (and
  against the whole-system near field) -- boxes of three or more cells, a box
  of exactly three, and boxes below three cells (every image looped over);
* the energy of the neutralising background, -(sum q)^2 Yhat(0) / (2V), against
  a quadrature of the Yukawa kernel over space, Yhat(0) = 4 pi int Y r^2 dr, and
  against the k = 0 identity of the decomposition Y = N + F (Section 4.1):
  U_k0 + U_bg = -(sum q)^2 4 pi int_0^inf (Y - F) r^2 dr / (2V)."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import workloads


def kdtree_near(x, q, L, s, rc, idx):
    """Near-field forces on particles idx by a periodic k-d tree pair search."""
    pos = x.T % L
    tree = cKDTree(pos, boxsize=L)
    out = np.zeros((3, len(idx)))
    for k, i in enumerate(idx):
        js = np.array(tree.query_ball_point(pos[i], rc), dtype=np.int64)
        js = js[js != i]
        d = pos[i][None, :] - pos[js]
        d -= L * np.round(d / L)
        r = np.sqrt((d * d).sum(1))
        m = r < rc
        d, r, js = d[m], r[m], js[m]
        fac = np.exp(-r / s.lam) * (1 + r / s.lam) / r ** 3 - 2 * sum(
            c * ss * np.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
        out[:, k] = q[i] * ((q[js] * fac)[:, None] * d).sum(0)
    return out


def edge_state(w, seed):
    """The workload's uniform state with particles on box faces, edges and
    corners (coordinates 0 and the largest double below L)."""
    st = workloads.make_state(w, seed)
    x = st.x.copy()
    top = np.nextafter(w.L, 0)
    x[:, 0] = 0.0
    x[:, 1] = top
    x[0, 2], x[1, 3], x[2, 4] = 0.0, top, 0.0
    x[:, 5] = [0.0, top, 0.0]
    x[:, 6] = [top, 0.0, top]
    q = st.q.copy()
    q[::4] = -0.6
    return x, q


CASES = [
    # (N, kappa, r_c, cells per axis floor(L / r_c))
    (3000, 0.5, 4.0, 5),    # L = 22.9; the whole-system near field also takes the cell path (N > 2000)
    (655, 1.0, 4.0, 3),     # L = 13.996: exactly three cells per axis
]


@pytest.mark.parametrize("N,kappa,rc,nc", CASES)
def test_near_subset_against_kdtree_and_whole_system(orc, N, kappa, rc, nc):
    w = workloads.Workload("t", N=N, kappa=kappa, gamma=1.0, r_c=rc, P=1, seed=41)
    assert math.floor(w.L / rc) == nc
    x, q = edge_state(w, 41)
    s = orc.sog_auto(w.lam, rc, 1e-4)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(7), rng.choice(N, 120, replace=False)]))
    fs = orc.near_subset(x, q, w.L, s, idx)
    fk = kdtree_near(x, q, w.L, s, rc, idx)
    fw, _ = orc.near(x, q, w.L, s)
    for ref in (fk, fw[:, idx]):
        assert np.linalg.norm(fs - ref) <= 1e-12 * np.linalg.norm(ref)
        per = np.linalg.norm(fs - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
        assert per.max() <= 1e-11


@pytest.mark.parametrize("L,rc", [(7.0, 3.0), (5.0, 2.6), (4.0, 4.5)])
def test_near_subset_small_boxes(orc, L, rc):
    """Boxes below three cells (rc > L/3, even rc > L): every image within rc."""
    st = workloads.small_system(40, L, 9, neutral=True)
    s = orc.sog_auto(1.0, rc, 1e-6)
    idx = np.array([0, 5, 17, 39])
    fs = orc.near_subset(st.x, st.q, L, s, idx)
    fw, _ = orc.near(st.x, st.q, L, s)   # brute force over images for N <= 2000
    assert np.linalg.norm(fs) > 0
    assert np.linalg.norm(fs - fw[:, idx]) <= 1e-13 * np.linalg.norm(fw[:, idx])
    # and a direct image loop in numpy for one particle
    i = 5
    nimg = int(math.ceil(rc / L))
    acc = np.zeros(3)
    for a in range(-nimg, nimg + 1):
        for b in range(-nimg, nimg + 1):
            for c in range(-nimg, nimg + 1):
                d = st.x[:, i][:, None] - st.x - np.array([a, b, c])[:, None] * L
                r = np.sqrt((d * d).sum(0))
                m = (r < rc) & (r > 0)
                r_, d_ = r[m], d[:, m]
                fac = np.exp(-r_) * (1 + r_) / r_ ** 3 - 2 * sum(cc * ss * np.exp(-ss * r_ * r_)
                                                                for cc, ss in zip(s.c, s.s))
                acc += st.q[i] * (st.q[m] * fac * d_).sum(1)
    assert np.linalg.norm(fs[:, 1] - acc) <= 1e-12 * np.linalg.norm(acc)


def test_near_subset_rejects_bad_index(orc):
    st = workloads.small_system(10, 7.0, 1)
    s = orc.sog_auto(1.0, 2.0, 1e-4)
    with pytest.raises(ValueError):
        orc.near_subset(st.x, st.q, 7.0, s, np.array([3, 10]))


@pytest.mark.parametrize("lam,rc,L", [(1.0, 3.0, 16.12), (10.0, 5.0, 40.0), (2.0, 4.0, 20.0)])
def test_background_energy(orc, lam, rc, L):
    st = workloads.small_system(30, L, 4, neutral=False)
    s = orc.sog_auto(lam, rc, 1e-4)
    sysm = orc.System(st.q, st.m, L, s, kT=1.0, P=3, seed=1)
    _, _, e = sysm.force(st.x, 0)
    Q, V = st.q.sum(), L ** 3
    # the background integral: int over space of Y(|r|) = 4 pi int_0^inf exp(-r/lam) r dr
    iy = 4 * math.pi * integrate.quad(lambda r: math.exp(-r / lam) * r, 0, math.inf, epsabs=0, epsrel=1e-13)[0]
    assert abs(e[4] - (-Q * Q * iy / (2 * V))) <= 1e-12 * abs(e[4])
    # the k = 0 identity: Fhat(0) - Yhat(0) = -4 pi int (Y - F) r^2 dr, split at r_c for the quadrature
    def g(r):
        return (math.exp(-r / lam) * r) - r * r * sum(c * math.exp(-ss * r * r) for c, ss in zip(s.c, s.s))
    ik = sum(integrate.quad(g, a, b, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
             for a, b in ((0.0, rc), (rc, 40.0 * lam)))
    ik += integrate.quad(g, 40.0 * lam, math.inf, epsabs=0, epsrel=1e-10)[0]
    lhs = e[2] + e[4]
    rhs = -Q * Q * 4 * math.pi * ik / (2 * V)
    assert abs(lhs - rhs) <= 1e-9 * abs(e[4])

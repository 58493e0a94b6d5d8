"""Pins of the oracle's random numbers, lattice and importance sampler
(Section 4.3: P(k) = F(k) Fhat(k) / S with the adaptive correction)."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads


@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 0, 0), (123, 4)),
                                     ((99, 2 ** 63 + 5, 3, 11), (2 ** 64 - 1, 2 ** 40)),
                                     ((2 ** 64 - 1, 12345, 0, 1), (101, 0))])
def test_philox_against_numpy(orc, ctr, key):
    """Philox4x64-10 equals numpy's implementation of the same published generator.
    numpy increments its counter before producing a block, so numpy at
    counter c-1 yields the block at counter c."""
    c = np.array(ctr, dtype=np.uint64)
    prev = c.copy()
    # c - 1 with borrow across the 256-bit counter
    for w in range(4):
        if prev[w] != 0:
            prev[w] -= np.uint64(1)
            break
        prev[w] = np.uint64(2 ** 64 - 1)
    bg = np.random.Philox(counter=prev, key=np.array(key, dtype=np.uint64))
    assert np.array_equal(bg.random_raw(4).astype(np.uint64), orc.philox(c, key))


def test_lattice_enumeration(orc):
    """Every n with 1 <= |n|^2 <= mmax appears once, sorted by (|n|^2, nx, ny, nz);
    shell sizes are the sums-of-three-squares counts (r3(1)=6, r3(2)=12, r3(3)=8,
    r3(4)=6, r3(5)=24, and 0 for m = 4^a (8b + 7), Legendre's theorem)."""
    mmax = 200
    n3, start = orc.lattice(mmax)
    R = 15
    g = np.stack(np.meshgrid(*[np.arange(-R, R + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    m = (g * g).sum(1)
    g = g[(m >= 1) & (m <= mmax)]
    key = np.lexsort((g[:, 2], g[:, 1], g[:, 0], (g * g).sum(1)))
    assert np.array_equal(n3, g[key])
    r3 = np.diff(start)
    assert list(r3[1:6]) == [6, 12, 8, 6, 24]
    for mm in range(1, mmax + 1):
        a = mm
        while a % 4 == 0:
            a //= 4
        assert (r3[mm] == 0) == (a % 8 == 7)


def test_density_limits(orc):
    """The adaptive correction (eq. 3.22, leading term): tends to sum q^2 at large k
    and, in the Coulomb limit lambda -> inf, to kTVk^2/(1 + kTVk^2/sum q^2)
    (so ~ kTV k^2 at small k, as the paper notes for the pure Coulomb kernel)."""
    kT, V, Q2 = 0.7, 1000.0, 300.0
    assert math.isclose(orc.density(0, kT, V, Q2, 2.0, 1e8), Q2, rel_tol=1e-6)
    k2 = 1e-3
    lim = kT * V * k2 / (1 + kT * V * k2 / Q2)
    assert math.isclose(orc.density(0, kT, V, Q2, 1e7, k2), lim, rel_tol=1e-8)
    assert orc.density(1, kT, V, Q2, 2.0, 0.3) == 1.0
    assert orc.density(2, kT, V, Q2, 2.0, 0.3) == 0.3


def _system(orc, N=200, kappa=1.0, gamma=1.0, rc=3.0, P=100, seed=9, density=0):
    w = workloads.Workload("t", N=N, kappa=kappa, gamma=gamma, r_c=rc, P=P, seed=seed)
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, rc, 1e-4)
    return w, st, s, orc.System(st.q, st.m, w.L, s, w.kT, P, seed=seed, density=density)


def test_shell_table_is_the_measure(orc):
    """cdf increments are r3(m) F(k^2) Fhat(k^2) for each non-empty shell (eq. 3.124),
    the per-shell estimator coefficient is S/(P V F(k^2)), and the truncation
    keeps every shell with Fhat >= 1e-16 Fhat(0)."""
    w, st, s, sysm = _system(orc)
    m, cdf, coef = sysm.tables()
    n3, start = sysm.lattice()
    L, V = w.L, w.L ** 3
    k2 = (2 * math.pi / L) ** 2 * m
    Fh = np.array([sum(a * math.exp(-b * kk) for a, b in zip(s.A, s.B)) for kk in k2])
    Q2 = float((st.q ** 2).sum())
    Fk = w.kT * V / (w.kT * V / Q2 + w.lam ** 2 / (1 + w.lam ** 2 * k2))
    r3 = np.diff(start)[m]
    inc = np.diff(np.concatenate([[0.0], cdf]))
    # increments are differences of a running sum: exact to its rounding, ~u S
    assert np.allclose(inc, r3 * Fk * Fh, rtol=1e-12, atol=8 * 2.0 ** -53 * cdf[-1])
    assert np.allclose(coef, cdf[-1] / (w.P * V * Fk), rtol=1e-13)
    assert Fh[-1] >= 1e-16 * s.Fhat0
    assert float(s.Fhat((2 * math.pi / L) ** 2 * (sysm.mmax + 1))) < 1e-16 * s.Fhat0


@pytest.mark.parametrize("density", [0, 1, 2, 3])
def test_draws_follow_the_measure(orc, density):
    """Chi-square of the sampled shells against P(|n|^2 = m) = r3(m) W(m) / S over
    20000 draws (shells merged into bins expecting >= 50 draws), and uniformity of the point chosen
    within a shell.  Seeded; the 1e-6 tail leaves no room for a wrong weight."""
    w, st, s, sysm = _system(orc, P=100, density=density)
    m, cdf, coef = sysm.tables()
    n3, start = sysm.lattice()
    draws = np.concatenate([sysm.draw(step)[0] for step in range(200)])
    mm = (draws.astype(np.int64) ** 2).sum(1)
    # probability per shell; consecutive shells merged until each bin expects >= 50 draws
    p = np.diff(np.concatenate([[0.0], cdf])) / cdf[-1]
    shell_of = np.searchsorted(m, mm)
    assert np.array_equal(m[shell_of], mm)
    bin_of_shell = np.zeros(len(p), dtype=np.int64)
    b, acc = 0, 0.0
    for i, pi in enumerate(p):
        bin_of_shell[i] = b
        acc += pi * len(mm)
        if acc >= 50:
            b, acc = b + 1, 0.0
    nb = bin_of_shell[-1] + 1
    obs = np.bincount(bin_of_shell[shell_of], minlength=nb)
    exp_ = np.bincount(bin_of_shell, weights=p, minlength=nb) * len(mm)
    chi2 = ((obs - exp_) ** 2 / exp_).sum()
    assert nb >= 5
    assert stats.chi2.sf(chi2, nb - 1) > 1e-6
    # within-shell uniformity on the most populated shell
    top = m[np.argmax(np.bincount(shell_of, minlength=len(m)))]
    sel = draws[mm == top]
    pts = n3[start[top]:start[top + 1]]
    idx = np.array([np.flatnonzero((pts == d).all(1))[0] for d in sel])
    cnt = np.bincount(idx, minlength=len(pts))
    if len(sel) > 20 * len(pts):
        chi2 = ((cnt - len(sel) / len(pts)) ** 2 / (len(sel) / len(pts))).sum()
        assert stats.chi2.sf(chi2, len(pts) - 1) > 1e-6


def test_draws_are_counter_based(orc):
    """A draw depends only on (seed, replica, step, sample index): the same step
    gives the same samples, another step or replica different ones."""
    w, st, s, a = _system(orc, seed=5)
    b = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=5)
    c = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=5, replica=1)
    assert np.array_equal(a.draw(17)[0], b.draw(17)[0])
    assert not np.array_equal(a.draw(17)[0], a.draw(18)[0])
    assert not np.array_equal(a.draw(17)[0], c.draw(17)[0])

"""Pins of the oracle's Metropolis-Hastings draws of the Fourier modes (the
sampler Section 4.1 names for P(k)): the chain's long-run shell frequencies
against P(k) = F(k) Fhat(k) / S written out here from the SOG and eq. (3.22)
(chi-square over batch means), acceptance of every proposal when F = 1 (the
proposal measure itself), the far-field estimator's mean over the chain
against the full-lattice far field (unbiased in the long run), and the
chain's dependence on its key and history only."""
import math

import numpy as np
import pytest

import workloads


def _system(orc, density, sampler=1, P=200, seed=5):
    L = 5.0
    st = workloads.small_system(30, L, 9, neutral=False)
    s = orc.sog_auto(1.0, 2.0, 1e-4)
    return st, s, L, orc.System(st.q, st.m, L, s, kT=0.05, P=P, seed=seed, density=density, sampler=sampler)


def _target_shells(orc, sysm, st, s, L, density):
    """Shell probabilities r3(m) F(k^2) Fhat(k^2) / S, from the SOG's Fourier
    coefficients, the density written out from eq. (3.22) and a brute-force
    count of the lattice points per shell."""
    m_of, _, _ = sysm.tables()
    lim = int(math.isqrt(int(m_of[-1]))) + 1
    g = np.arange(-lim, lim + 1)
    n2 = (g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2).ravel()
    r3 = np.array([(n2 == m).sum() for m in m_of], dtype=float)
    k2 = (2 * math.pi / L) ** 2 * m_of
    fhat = sum(a * np.exp(-b * k2) for a, b in zip(s.A, s.B))
    V, Q2, kT = L ** 3, float((st.q ** 2).sum()), 0.05
    if density == orc.FLAT:
        F = np.ones_like(k2)
    else:
        F = kT * V / (kT * V / Q2 + 1.0 / (1.0 + k2))   # lambda = 1
    w = r3 * F * fhat
    return m_of, w / w.sum()


@pytest.mark.slow
def test_chain_samples_the_adaptive_measure(orc):
    st, s, L, sysm = _system(orc, orc.ADAPTIVE)
    m_of, p = _target_shells(orc, sysm, st, s, L, orc.ADAPTIVE)
    idx = {int(m): i for i, m in enumerate(m_of)}
    nb, per = 20, 100                      # 20 batches of 100 steps x 200 draws
    counts = np.zeros((nb, len(m_of)))
    moves = 0
    prev = None
    for b in range(nb):
        for t in range(per):
            n3, coef = sysm.draw(b * per + t)
            m = (n3.astype(np.int64) ** 2).sum(1)
            for v in m:
                counts[b, idx[int(v)]] += 1
            moves += int((np.any(n3[1:] != n3[:-1], axis=1)).sum())
            prev = n3
    freq = counts / counts.sum(1, keepdims=True)
    mean, se = freq.mean(0), freq.std(0, ddof=1) / math.sqrt(nb)
    big = p > 1e-3
    z = (mean[big] - p[big]) / np.maximum(se[big], 1e-12)
    assert np.abs(z).max() < 5.0, z
    assert abs(mean[~big].sum() - p[~big].sum()) < 5e-3
    rate = moves / (nb * per * 199)
    assert 0.3 < rate < 0.999            # the chain both moves and rejects


def test_flat_density_accepts_every_proposal(orc):
    st, s, L, sysm = _system(orc, orc.FLAT)
    total, moved = 0, 0
    seen = set()
    for step in range(30):
        n3, coef = sysm.draw(step)
        assert np.all(coef == coef[0])        # F = 1: one coefficient S / (P V)
        seen.update(map(tuple, n3))
        total += len(n3)
    assert len(seen) > 100                     # i.i.d. proposals, not a stuck chain


def test_flat_chain_frequencies(orc):
    st, s, L, sysm = _system(orc, orc.FLAT)
    m_of, p = _target_shells(orc, sysm, st, s, L, orc.FLAT)
    idx = {int(m): i for i, m in enumerate(m_of)}
    c = np.zeros(len(m_of))
    for step in range(200):
        n3, _ = sysm.draw(step)
        for v in (n3.astype(np.int64) ** 2).sum(1):
            c[idx[int(v)]] += 1
    big = p * c.sum() > 20
    chi2 = (((c[big] - p[big] * c.sum()) ** 2) / (p[big] * c.sum())).sum()
    dof = int(big.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_chain_is_keyed_and_sequential(orc):
    _, _, _, a = _system(orc, orc.ADAPTIVE)
    _, _, _, b = _system(orc, orc.ADAPTIVE)
    _, _, _, c = _system(orc, orc.ADAPTIVE, seed=6)
    for step in range(5):
        na, ca = a.draw(step)
        nb_, cb = b.draw(step)
        nc, _ = c.draw(step)
        assert np.array_equal(na, nb_) and np.array_equal(ca, cb)
        assert not np.array_equal(na, nc)
    # emptying the chain replays it from the start
    a.set_sampler(1)
    b.set_sampler(1)
    assert np.array_equal(a.draw(0)[0], b.draw(0)[0])
    # the i.i.d. sampler keeps its own draws, independent of the chain
    _, _, _, e = _system(orc, orc.ADAPTIVE, sampler=0)
    a.set_sampler(0)
    assert np.array_equal(a.draw(3)[0], e.draw(3)[0])


@pytest.mark.slow
def test_far_estimator_mean_over_the_chain(orc):
    """The random-batch far force averaged over the chain's draws approaches the
    full-lattice far force (the chain's stationary measure and the estimator's
    coefficients fit together)."""
    st, s, L, sysm = _system(orc, orc.ADAPTIVE, P=100)
    full = orc.System(st.q, st.m, L, s, kT=0.05, P=1, seed=1, full_k=True)
    f_full, fn, _ = full.force(st.x, 0)
    ff_full = f_full - fn
    nb, per = 16, 50
    means = []
    for b in range(nb):
        acc = np.zeros_like(st.x)
        for t in range(per):
            f, fnn, _ = sysm.force(st.x, b * per + t)
            acc += f - fnn
        means.append(acc / per)
    means = np.array(means)
    m = means.mean(0)
    se = means.std(0, ddof=1) / math.sqrt(nb)
    z = (m - ff_full) / np.maximum(se, 1e-14)
    assert np.sqrt((z ** 2).mean()) < 2.0

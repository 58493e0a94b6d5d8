"""Statistical pins of the random-batch far field (Section 4.4): unbiasedness of
the force and energy estimators, their exact variances (the lemma on
unbiasedness, eqs. 3.22 and 3.24), the O(1/P) scaling, and the variance
ordering the adaptive density is built for.  All seeded."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads


def _setup(orc, N=100, kappa=1.0, gamma=1.0, P=20, seed=31, density=0, charged=True):
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed, neutral=not charged)
    s = orc.sog_auto(1 / kappa, 3.0, 1e-4)
    sysm = orc.System(st.q, st.m, L, s, 1 / gamma, P, seed=seed, density=density)
    return L, st, s, sysm


def _full_lattice(orc, st, L, s, sysm):
    """rho, Fhat, k for every sampled mode, the full far force and energy."""
    n3, start = sysm.lattice()
    k = (2 * math.pi / L) * n3.astype(np.float64)
    rho = orc.rho(st.x, st.q, L, n3)
    k2 = (k * k).sum(1)
    fh = np.array([float(s.Fhat(v)) for v in k2])
    return n3, k, k2, rho, fh


def _batches(orc, st, L, sysm, B, step0=0):
    F, Us = [], []
    for b in range(B):
        n3, coef = sysm.draw(step0 + b)
        rho = orc.rho(st.x, st.q, L, n3)
        F.append(orc.far_rb(st.x, st.q, L, n3, coef, rho))
        Us.append(0.5 * float((coef * (rho ** 2).sum(1)).sum()))
    return np.array(F), np.array(Us)


def test_unbiased_and_variance_formulas(orc):
    """The batch mean of F* is the full far force (aggregate z^2 within the
    chi-square tail, max |z| <= 6) and of U* the full far energy; the empirical
    variances match eqs. (3.24) and (3.22) evaluated over the whole lattice."""
    L, st, s, sysm = _setup(orc)
    n3, k, k2, rho, fh = _full_lattice(orc, st, L, s, sysm)
    V = L ** 3
    f_full, U_full = orc.far_full(st.x, st.q, L, s, sysm.mmax)
    B = 4000
    F, Us = _batches(orc, st, L, sysm, B)
    mean = F.mean(0)
    sd = F.std(0, ddof=1)
    z = (mean - f_full) / (sd / math.sqrt(B))
    T = float((z ** 2).sum())
    assert stats.chi2.sf(T, z.size) > 1e-6
    assert np.abs(z).max() <= 6
    zu = (Us.mean() - U_full) / (Us.std(ddof=1) / math.sqrt(B))
    assert abs(zu) <= 5
    # eq. (3.24): E|Xi_F,i|^2 = (1/P)[(q_i^2 S/V^2) sum_k k^2 Fhat |Im(e^{-ik.r_i} rho)|^2 / F(k) - |F_F,i|^2]
    m_sh, cdf, coef = sysm.tables()
    S = cdf[-1]
    Q2 = float((st.q ** 2).sum())
    Fk = np.array([orc.density(0, sysm.kT, V, Q2, s.lam, v) for v in k2])
    th = st.x.T @ k.T                                  # (N, K)
    im = rho[None, :, 1] * np.cos(th) - rho[None, :, 0] * np.sin(th)
    second = (st.q ** 2 * S / V ** 2) * ((k2 * fh / Fk)[None, :] * im ** 2).sum(1)
    var_pred = (second - (f_full ** 2).sum(0)) / sysm.P
    var_emp = (F.var(0, ddof=1)).sum(0)
    assert abs(var_emp.sum() / var_pred.sum() - 1) <= 0.05
    # eq. (3.22): E|Xi_U|^2 = (1/P)[(S/(4V^2)) sum_k Fhat |rho|^4 / F(k) - U_F^2]
    r2 = (rho ** 2).sum(1)
    varU_pred = (S / (4 * V ** 2) * (fh * r2 ** 2 / Fk).sum() - U_full ** 2) / sysm.P
    assert abs(Us.var(ddof=1) / varU_pred - 1) <= 0.1


def test_variance_scales_as_one_over_P(orc):
    """The force variance is O(1/P) (the lemma): P = 40 has a quarter of the
    variance of P = 10."""
    v = []
    for P in (10, 40):
        L, st, s, sysm = _setup(orc, P=P, seed=44)
        F, _ = _batches(orc, st, L, sysm, 1500, step0=1000)
        v.append(F.var(0, ddof=1).sum())
    assert 3.4 <= v[0] / v[1] <= 4.6


def test_density_variance_ordering(orc):
    """Mean-field statement of Theorem 3.2 on uniform, uncorrelated input: the
    exact energy variance (eq. 3.22) of the adaptive density is no worse than the
    flat density's at weak coupling, where the adaptive correction tends to the
    constant sum q^2, and clearly better than the k^2 density's."""
    var = {}
    for dens in (0, 1, 2):
        L, st, s, sysm = _setup(orc, N=300, gamma=0.01, P=1, seed=8, density=dens)
        n3, k, k2, rho, fh = _full_lattice(orc, st, L, s, sysm)
        V = L ** 3
        m_sh, cdf, coef = sysm.tables()
        S = cdf[-1]
        Q2 = float((st.q ** 2).sum())
        Fk = np.array([orc.density(dens, sysm.kT, V, Q2, s.lam, v) for v in k2])
        r2 = (rho ** 2).sum(1)
        U = (fh * r2).sum() / (2 * V)
        var[dens] = S / (4 * V ** 2) * (fh * r2 ** 2 / Fk).sum() - U ** 2
    assert var[0] <= 1.05 * var[1]
    assert var[2] >= 2.0 * var[0]

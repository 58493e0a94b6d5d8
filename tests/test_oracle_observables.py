"""Pins of the oracle's observables (Section 5.1): the static structure
factor S(k) = <rho(k) rho(-k)> / N by lattice shell and the pair-distance
histogram behind the RDF.  Closed forms on a simple cubic crystal (Bragg
peaks of height N on the reciprocal lattice, zero elsewhere; neighbour shells
of 6, 12 and 8 sites), a single particle, an independent numpy pair search,
and the ideal-gas limits of uniform random positions."""
import itertools
import math

import numpy as np

import workloads


def _crystal(M, L):
    g = (np.arange(M) + 0.5) * L / M
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


def test_ssf_crystal_bragg_peaks(orc):
    M, L, mmax = 4, 9.0, 80
    x = _crystal(M, L)
    N = M ** 3
    S = orc.ssf(x, np.ones(N), L, mmax) / N
    R = int(math.isqrt(mmax)) + 1
    pts = [n for n in itertools.product(range(-R, R + 1), repeat=3) if 1 <= sum(c * c for c in n) <= mmax]
    for m in range(1, mmax + 1):
        shell = [n for n in pts if sum(c * c for c in n) == m]
        if not shell:
            assert S[m] == 0.0
            continue
        frac = sum(all(c % M == 0 for c in n) for n in shell) / len(shell)
        assert abs(S[m] - N * frac) <= 1e-9 * N, (m, S[m], N * frac)


def test_ssf_single_particle_and_weights(orc):
    L = 7.3
    x = np.array([[1.1], [2.9], [6.0]])
    s = orc.ssf(x, np.array([1.0]), L, 30)
    nonempty = [m for m in range(1, 31) if any(a * a + b * b + c * c == m
                                               for a in range(-6, 7) for b in range(-6, 7) for c in range(-6, 7))]
    assert np.allclose(s[nonempty], 1.0, rtol=0, atol=1e-13)
    assert s[0] == 0.0
    s3 = orc.ssf(x, np.array([3.0]), L, 30)
    assert np.allclose(s3[nonempty], 9.0, rtol=0, atol=1e-12)


def test_ssf_ideal_gas(orc):
    """Uniform random positions: |rho(k)|^2 / N is exponential with mean 1 for
    every k != 0, so the mean of S over all modes is 1 within its error."""
    N = 500
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=5)
    mmax = 60
    S = orc.ssf(st.x, np.ones(N), L, mmax) / N
    R = int(math.isqrt(mmax)) + 1
    cnt = np.zeros(mmax + 1)
    for n in itertools.product(range(-R, R + 1), repeat=3):
        m = sum(c * c for c in n)
        if 1 <= m <= mmax:
            cnt[m] += 1
    K = cnt.sum()
    mean = (S * cnt).sum() / K
    assert abs(mean - 1.0) <= 5.0 / math.sqrt(K), mean


def _rdf_numpy(x, L, r_max, nbins):
    d = x[:, :, None] - x[:, None, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(0))
    np.fill_diagonal(r, np.inf)
    r = r[r < r_max]
    return np.bincount(np.minimum((r / (r_max / nbins)).astype(np.int64), nbins - 1), minlength=nbins)


def test_rdf_against_numpy_pair_search(orc):
    N = 700
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=9)
    r_max, nbins = 0.45 * L, 90
    c, amb = orc.rdf(st.x, L, r_max, nbins)
    ref = _rdf_numpy(st.x, L, r_max, nbins)
    assert np.all(np.abs(c - ref) <= amb)
    assert c.sum() == ref.sum()


def test_rdf_crystal_shells(orc):
    M, L = 5, 10.0   # spacing 2
    x = _crystal(M, L)
    N = M ** 3
    c, amb = orc.rdf(x, L, 3.6, 36)   # shells at 2, 2 sqrt 2, 2 sqrt 3: 6, 12 and 8 neighbours
    assert c.sum() == N * (6 + 12 + 8)
    assert c[int(2 * math.sqrt(2) / 0.1)] == 12 * N and c[int(2 * math.sqrt(3) / 0.1)] == 8 * N
    assert c[19] + c[20] == 6 * N and amb[19] + amb[20] == 2 * 6 * N   # r = 2 lies on the edge of bin 20


def test_rdf_ideal_gas_normalisation(orc):
    """Uniform positions: the number of ordered pairs within r_max is
    N (N - 1) (4/3 pi r_max^3) / V within a few standard deviations."""
    N = 2000
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=13)
    r_max = 3.0
    c, _ = orc.rdf(st.x, L, r_max, 30)
    expect = N * (N - 1) * (4.0 / 3.0 * math.pi * r_max ** 3) / L ** 3
    assert abs(c.sum() - expect) <= 5 * math.sqrt(2 * expect), (c.sum(), expect)

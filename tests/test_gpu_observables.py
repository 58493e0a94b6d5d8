"""Observables through the library against the oracle: the static structure
factor by lattice shell (rbsog_ssf, the structure-factor kernels over every
mode of the shells) within 1e-12 relative per shell, and the pair-distance
histogram (rbsog_rdf) bit-exact except for pairs the oracle marks as lying
on a bin edge.  Inputs: seeded uniform and crystal positions, and a
configuration from the oracle's own dynamics."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2501_10946_amd")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return torch.device("cuda:0")


def gpu_ssf(dev, x, w, L, m_s):
    N = w.shape[0]
    nbytes = R.rbsog_ssf_scratch_size(N, m_s)
    scratch = torch.empty(nbytes // 8 + 64, dtype=torch.float64, device=dev)
    s = torch.full((m_s + 1,), -1.0, dtype=torch.float64, device=dev)
    R.rbsog_ssf(torch.tensor(x, device=dev), torch.tensor(w, device=dev), L, m_s, scratch, s)
    return s.cpu().numpy()


def _crystal(M, L):
    g = (np.arange(M) + 0.5) * L / M
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


@pytest.mark.parametrize("N,m_s,weights", [(1000, 60, "unit"), (777, 5, "charge"), (20000, 150, "unit"),
                                           (1, 30, "unit")])
def test_ssf_matches_oracle(dev, N, m_s, weights):
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=N + m_s, neutral=weights == "charge")
    w = np.ones(N) if weights == "unit" else st.q
    print(f"\n[case] ssf N={N} m_s={m_s} weights={weights}", flush=True)
    s = gpu_ssf(dev, st.x, w, L, m_s)
    so = oracle.ssf(st.x, w, L, m_s)
    nz = so > 0
    assert np.all(s[~nz] == 0.0)
    scale = np.abs(so[nz]).max()
    assert np.abs(s[nz] - so[nz]).max() <= 1e-12 * scale
    assert np.abs(s[nz] - so[nz]).max() / scale <= 1e-12


def test_ssf_crystal_bragg_peaks(dev):
    M, L, m_s = 6, 12.0, 100
    x = _crystal(M, L)
    N = M ** 3
    S = gpu_ssf(dev, x, np.ones(N), L, m_s) / N
    So = oracle.ssf(x, np.ones(N), L, m_s) / N
    assert np.abs(S - So).max() <= 1e-10 * N
    # Bragg peaks: each shell's reciprocal-lattice modes (n a multiple of M) give N, the others 0
    R_ = int(math.isqrt(m_s)) + 1
    rng = range(-R_, R_ + 1)
    for m in (36, 72, 100):
        shell = [(a, b, c) for a in rng for b in rng for c in rng if a * a + b * b + c * c == m]
        frac = sum(a % M == 0 and b % M == 0 and c % M == 0 for a, b, c in shell) / len(shell)
        assert abs(S[m] - N * frac) <= 1e-9 * N, (m, S[m], N * frac)


def test_ssf_refuses_small_scratch(dev):
    N, m_s = 100, 20
    x = torch.zeros((3, N), dtype=torch.float64, device=dev)
    w = torch.ones(N, dtype=torch.float64, device=dev)
    s = torch.zeros(m_s + 1, dtype=torch.float64, device=dev)
    scratch = torch.empty(16, dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError):
        R.rbsog_ssf(x, w, 10.0, m_s, scratch, s)


def _system(dev, w, st):
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    return R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, device=dev), o


def _assert_hist(h, c, amb):
    assert np.all(np.abs(h - c) <= amb), np.nonzero(np.abs(h - c) > amb)
    assert abs(int(h.sum()) - int(c.sum())) <= int(amb.sum())


@pytest.mark.parametrize("N,r_frac,nbins", [(2000, 1.0, 100), (3000, 0.5, 7), (5000, 1.0, 4096)])
def test_rdf_matches_oracle(dev, N, r_frac, nbins):
    w = workloads.Workload(f"rdf_n{N}", N=N, kappa=1.0, gamma=1.0, r_c=3.0, P=16, seed=N)
    st = workloads.make_state(w)
    s, _ = _system(dev, w, st)
    r_max = r_frac * w.r_c
    print(f"\n[case] rdf N={N} r_max={r_max} nbins={nbins}", flush=True)
    hist = torch.zeros(nbins, dtype=torch.int64, device=dev)
    R.rbsog_rdf(s.h, torch.tensor(st.x, device=dev), r_max, nbins, hist)
    torch.cuda.synchronize()
    c, amb = oracle.rdf(st.x, w.L, r_max, nbins)
    _assert_hist(hist.cpu().numpy(), c, amb)


def test_rdf_accumulates_and_leaves_forces_intact(dev):
    """Two snapshots add up; a force evaluation after the histogram (whose cell
    build reorders the workspace rows) matches the oracle."""
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s, o = _system(dev, w, st)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    x1 = st.x.copy()
    v = st.v.copy()
    f, _, _ = ref.force(x1, 0)
    x2 = x1.copy()
    ref.run(x2, v, f, 0, 50, w.dt)   # a second configuration from the oracle's dynamics
    hist = torch.zeros(60, dtype=torch.int64, device=dev)
    for x in (x1, x2):
        R.rbsog_rdf(s.h, torch.tensor(x, device=dev), w.r_c, 60, hist)
    c1, a1 = oracle.rdf(x1, w.L, w.r_c, 60)
    c2, a2 = oracle.rdf(x2, w.L, w.r_c, 60)
    torch.cuda.synchronize()
    _assert_hist(hist.cpu().numpy(), c1 + c2, a1 + a2)
    xt = torch.tensor(x2, device=dev)
    ft = torch.empty_like(xt)
    R.rbsog_compute_forces(s.h, 3, xt, ft)
    fo, _, _ = ref.force(x2, 3)
    d = ft.cpu().numpy() - fo
    assert np.linalg.norm(d) <= 1e-12 * np.linalg.norm(fo)


def test_rdf_refuses_bad_arguments(dev):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s, _ = _system(dev, w, st)
    x = torch.tensor(st.x, device=dev)
    hist = torch.zeros(10, dtype=torch.int64, device=dev)
    for r_max, nbins in ((w.r_c * 1.01, 10), (0.0, 10), (1.0, 0), (1.0, 5000)):
        with pytest.raises(R.RbsogError):
            R.rbsog_rdf(s.h, x, r_max, nbins, hist if nbins <= 10 else torch.zeros(nbins, dtype=torch.int64,
                                                                                    device=dev))

"""The Metropolis-Hastings draws of the Fourier modes (sampler
RBSOG_SAMPLER_MH) through the library against the oracle's chain: the draws
of consecutive steps bit for bit (the chain's integer states and the
coefficients), for the adaptive and the DH-4pi densities and a ragged batch;
a 30-step FP64 trajectory whose modes the library draws ahead in batches, to
1e-10; and the served ensemble refusing the sampler."""
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


def _pair(dev, w, density=0):
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    st = workloads.make_state(w)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, density=density, sampler=R.RBSOG_SAMPLER_MH,
                 device=dev)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed, density=density, sampler=1)
    return st, s, ref


W = workloads.Workload
CASES = [workloads.OCP_1K,
         W("ragged_n777_p300", N=777, kappa=1.0, gamma=1.0, r_c=3.0, P=300, seed=5),
         W("cold_n2000_p37", N=2000, kappa=0.5, gamma=50.0, r_c=4.0, P=37, seed=13)]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
@pytest.mark.parametrize("density", [0, 3])
def test_chain_draws_bit_exact(dev, w, density):
    print(f"\n[case] MH draws {w.name} density={density}", flush=True)
    st, s, ref = _pair(dev, w, density)
    n = torch.zeros((w.P, 3), dtype=torch.int32, device=dev)
    coef = torch.zeros(w.P, dtype=torch.float64, device=dev)
    moved = 0
    for step in range(12):
        R.rbsog_sample_k(s.h, step, n, coef)
        torch.cuda.synchronize()
        no, co = ref.draw(step)
        assert np.array_equal(n.cpu().numpy(), no), f"step {step}"
        assert np.array_equal(coef.cpu().numpy().view(np.uint64), co.view(np.uint64)), f"step {step}"
        moved += int(np.any(no[1:] != no[:-1], axis=1).sum())
    assert moved > 0


def test_chain_trajectory(dev):
    w = CASES[0]
    st, s, ref = _pair(dev, w)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    R.rbsog_step(s.h, x, v, f, 0, 30, w.dt)
    torch.cuda.synchronize()
    R.rbsog_check(s.h)
    xo, vo = st.x.copy(), st.v.copy()
    fo, _, _ = ref.force(xo, 0)
    ref.run(xo, vo, fo, 0, 30, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= 1e-10
    assert np.abs(v.cpu().numpy() - vo).max() <= 1e-9


def test_ensemble_refuses_the_chain(dev):
    w = CASES[0]
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    st = workloads.make_state(w)
    p = R.make_params(w.N, w.L, w.kT, w.P, 1, 0, 0, R.RBSOG_FP64, sampler=R.RBSOG_SAMPLER_MH)
    ens = R.rbsog_ens_create(1 << 28, 2)
    try:
        with pytest.raises(R.RbsogError) as e:
            R.rbsog_ens_admit(ens, p, sog, np.ascontiguousarray(st.x), np.ascontiguousarray(st.v),
                              np.ascontiguousarray(st.q), np.ascontiguousarray(st.m), 5, 0.01)
        assert e.value.code == R.RBSOG_EINVAL
    finally:
        R.rbsog_ens_destroy(ens)

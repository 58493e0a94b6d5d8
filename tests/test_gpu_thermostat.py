"""The Langevin thermostat of rbsog_step (the BAOAB splitting with Philox
normals) through the library against the oracle's: the trajectory to 1e-9 in
FP64 (split over two calls, so that the first-drift kernel and the drift fused
into the far kernel both run it), zero friction equal bit for bit to the NVE
run, and the kinetic temperature held at the bath's."""
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


def _pair(dev, w, st, precision=0, skin=-1.0):
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, precision=precision, skin=skin, device=dev)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    return s, ref


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("skin", [-1.0, 0.0], ids=["skin", "noskin"])
def test_langevin_trajectory_matches_oracle(dev, precision, skin):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s, ref = _pair(dev, w, st, precision, skin)
    friction, bath = 0.8, 2.5 * w.kT
    R.rbsog_set_thermostat(s.h, friction, bath)
    ref.set_langevin(friction, bath)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    R.rbsog_step(s.h, x, v, f, 0, 10, w.dt)
    R.rbsog_step(s.h, x, v, f, 10, 20, w.dt)
    torch.cuda.synchronize()
    R.rbsog_check(s.h)
    xo, vo = st.x.copy(), st.v.copy()
    fo, _, _ = ref.force(xo, 0)
    ref.run(xo, vo, fo, 0, 30, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    tol = 1e-9 if precision == 0 else 1e-4
    assert np.abs(d).max() <= tol, np.abs(d).max()
    assert np.abs(v.cpu().numpy() - vo).max() <= tol * 10 * max(1.0, np.abs(vo).max())
    # the bath acts: the run at friction 0 ends elsewhere
    nve = oracle.System(st.q, st.m, w.L, ref.sog, w.kT, w.P, seed=w.seed)
    xn, vn = st.x.copy(), st.v.copy()
    fn, _, _ = nve.force(xn, 0)
    nve.run(xn, vn, fn, 0, 30, w.dt)
    assert np.abs(vn - vo).max() > 1e-3


def test_zero_friction_is_nve_bit_for_bit(dev):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    outs = []
    for fr in (None, 0.0):
        s, _ = _pair(dev, w, st)
        if fr is not None:
            R.rbsog_set_thermostat(s.h, 0.5, 1.0)
            R.rbsog_set_thermostat(s.h, fr, 1.0)
        x = torch.tensor(st.x, device=dev)
        v = torch.tensor(st.v, device=dev)
        f = torch.empty_like(x)
        R.rbsog_compute_forces(s.h, 0, x, f)
        R.rbsog_step(s.h, x, v, f, 0, 15, w.dt)
        torch.cuda.synchronize()
        outs.append((x.cpu().numpy(), v.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_bath_sets_the_kinetic_temperature(dev):
    """A plasma started at k_B T and coupled to a bath at three times that
    (friction 2): after 1500 steps the mean kinetic energy over the last 500 is
    (3N/2) k_B T_bath within 3 %."""
    w = workloads.Workload("bath_n4000", N=4000, kappa=1.0, gamma=1.0, r_c=3.0, P=50, seed=61)
    st = workloads.make_state(w)
    s, _ = _pair(dev, w, st)
    bath = 3.0 * w.kT
    R.rbsog_set_thermostat(s.h, 2.0, bath)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    R.rbsog_step(s.h, x, v, f, 0, 1000, w.dt)
    eh = torch.zeros((500, R.ENERGY_COLS), dtype=torch.float64, device=dev)
    R.rbsog_step(s.h, x, v, f, 1000, 500, w.dt, eh)
    torch.cuda.synchronize()
    R.rbsog_check(s.h)
    ke = eh[:, 5].cpu().numpy().mean()
    assert abs(ke / (1.5 * w.N * bath) - 1) <= 0.03, ke / (1.5 * w.N * bath)


def test_thermostat_refuses_bad_arguments(dev):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s, _ = _pair(dev, w, st)
    for fr, kT in ((-1.0, 1.0), (float("nan"), 1.0), (1.0, 0.0), (1.0, float("inf"))):
        with pytest.raises(R.RbsogError):
            R.rbsog_set_thermostat(s.h, fr, kT)

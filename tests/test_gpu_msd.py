"""Displacement tracking and the MSD/VACF reduction through the library
(rbsog_track, rbsog_msd_vacf) against the oracle's: unwrapped displacements
within 1e-12 of the box length over a trajectory of seeded wrapped snapshots
(fma contraction of the minimum-image step may move the last bit), the two
averages within 1e-13 relative (the sums run in another order), the library's
averages bitwise repeatable, and a run of rbsog_step tracked call by call
against the oracle's tracker fed the same positions."""
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


def _msd(dev, disp, v0, v):
    scratch = torch.empty(R.rbsog_msd_scratch_size() // 8, dtype=torch.float64, device=dev)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
    R.rbsog_msd_vacf(disp, v0, v, scratch, out)
    return out.cpu().numpy()


# 262145 = one particle past a full sweep of the fixed 1024 x 256 grid (ragged second pass)
@pytest.mark.parametrize("N", [1, 333, 262145])
def test_track_and_averages_match_oracle(dev, N):
    print(f"\n[case] track N={N}", flush=True)
    rng = np.random.default_rng(N)
    L = 9.0
    x0 = rng.random((3, N)) * L
    v = rng.normal(0, 2.0, (3, N))
    x_last = np.ascontiguousarray(x0.copy())
    disp = np.zeros((3, N))
    xl_d = torch.tensor(x0, device=dev)
    dp_d = torch.zeros((3, N), dtype=torch.float64, device=dev)
    x = x0
    for n in range(25):
        x = np.mod(x + v * 0.1 + rng.normal(0, 0.5, (3, N)), L)
        x = np.ascontiguousarray(x)
        oracle.track(x, L, x_last, disp)
        R.rbsog_track(torch.tensor(x, device=dev), L, xl_d, dp_d)
    torch.cuda.synchronize()
    assert np.array_equal(xl_d.cpu().numpy(), x_last)
    assert np.abs(dp_d.cpu().numpy() - disp).max() <= 1e-12 * L
    v0 = rng.normal(0, 1.0, (3, N))
    v0_d, v_d = torch.tensor(v0, device=dev), torch.tensor(v, device=dev)
    got = _msd(dev, dp_d, v0_d, v_d)
    ref = oracle.msd_vacf(dp_d.cpu().numpy(), v0, v)
    assert abs(got[0] - ref[0]) <= 1e-13 * abs(ref[0])
    assert abs(got[1] - ref[1]) <= 1e-13 * np.abs(v0 * v).sum() / N
    assert np.array_equal(_msd(dev, dp_d, v0_d, v_d), got)


# N = 777: the axis boundaries 777 and 1554 of the [3][N] rows fall inside workgroups
@pytest.mark.parametrize("N", [1, 777, 262145])
def test_track_cuboid_matches_oracle(dev, N):
    """rbsog_track with three edges: each component folds by its own edge."""
    print(f"\n[case] track cuboid N={N}", flush=True)
    rng = np.random.default_rng(100 + N)
    Lb = (6.0, 11.0, 8.5)
    Lc = np.array(Lb)[:, None]
    x0 = rng.random((3, N)) * Lc
    v = rng.normal(0, 2.0, (3, N))
    x_last = np.ascontiguousarray(x0.copy())
    disp = np.zeros((3, N))
    xl_d = torch.tensor(x0, device=dev)
    dp_d = torch.zeros((3, N), dtype=torch.float64, device=dev)
    x = x0
    for n in range(25):
        x = np.ascontiguousarray(np.mod(x + v * 0.1 + rng.normal(0, 0.5, (3, N)), Lc))
        oracle.track(x, Lb, x_last, disp)
        R.rbsog_track(torch.tensor(x, device=dev), Lb, xl_d, dp_d)
    torch.cuda.synchronize()
    assert np.array_equal(xl_d.cpu().numpy(), x_last)
    assert np.abs(dp_d.cpu().numpy() - disp).max() <= 1e-12 * max(Lb)
    with pytest.raises(R.RbsogError):
        R.rbsog_track(xl_d, (6.0, 0.0, 8.5), xl_d.clone(), dp_d)


def test_tracks_a_library_run(dev):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, device=dev)
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    v0 = v.clone()
    xl_d = x.clone()
    dp_d = torch.zeros_like(x)
    x_last = np.ascontiguousarray(st.x.copy())
    disp = np.zeros_like(st.x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    for c in range(8):
        R.rbsog_step(s.h, x, v, f, 5 * c, 5 * c + 5, w.dt)
        R.rbsog_track(x, w.L, xl_d, dp_d)
        oracle.track(np.ascontiguousarray(x.cpu().numpy()), w.L, x_last, disp)
    torch.cuda.synchronize()
    R.rbsog_check(s.h)
    assert np.abs(dp_d.cpu().numpy() - disp).max() <= 1e-12 * w.L
    got = _msd(dev, dp_d, v0, v)
    ref = oracle.msd_vacf(dp_d.cpu().numpy(), v0.cpu().numpy(), v.cpu().numpy())
    assert abs(got[0] - ref[0]) <= 1e-13 * ref[0]
    assert abs(got[1] - ref[1]) <= 1e-13 * (v0 * v).abs().sum().item() / st.x.shape[1]
    assert got[0] > 0.0


def test_rejects_bad_arguments(dev):
    x = torch.zeros((3, 4), dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError):
        R.rbsog_track(x, -1.0, x.clone(), x.clone())
    scratch = torch.empty(4, dtype=torch.float64, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError):
        R.rbsog_msd_vacf(x, x, x, scratch, out)

"""Systems in a cuboid box (edges L_x, L_y, L_z) through the library against
the oracle: the point-by-point sampling tables and draws bit for bit, the
cell list bit for bit, forces, energies and virials within 1e-12 (FP64) /
1e-5 (mixed), the full-lattice far field, a 30-step trajectory to 1e-10, and
the pair histogram; cuboids the ensemble and the Metropolis-Hastings chain
refuse."""
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


def _case(w, stretch):
    """The workload at its density in a box stretched by `stretch` per axis
    (volume kept), positions scaled to it."""
    st = workloads.make_state(w)
    f = np.asarray(stretch, dtype=float)
    f = f / np.prod(f) ** (1 / 3)
    Lb = tuple(float(v) for v in w.L * f)
    st.x = np.ascontiguousarray(st.x * f[:, None])
    return st, Lb


def _pair(dev, w, stretch, precision=0, full_k=False):
    st, Lb = _case(w, stretch)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    s = R.System(st.q, st.m, Lb, sog, w.kT, w.P, seed=w.seed, precision=precision, full_k=full_k, device=dev)
    ref = oracle.System(st.q, st.m, Lb, o, w.kT, w.P, seed=w.seed, full_k=full_k)
    return st, Lb, s, ref


W = workloads.Workload
CASES = [(workloads.OCP_1K, (1.0, 1.3, 0.85)),
         (W("ragged_n777_p300", N=777, kappa=1.0, gamma=1.0, r_c=3.0, P=300, seed=5), (0.8, 1.0, 1.35)),
         (W("mix_n5000", N=5000, kappa=0.5, gamma=5.0, r_c=4.0, P=64, seed=12, frac_b=0.1, q_b=5.0, m_b=20.0),
          (1.5, 1.0, 0.9))]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("w,stretch", CASES, ids=lambda c: getattr(c, "name", "box"))
def test_tables_draws_and_cells_bit_exact(dev, w, stretch):
    st, Lb, s, ref = _pair(dev, w, stretch)
    print(f"\n[case] cuboid {w.name} L={Lb}", flush=True)
    info = R.rbsog_get_info(s.h)
    n3, _ = oracle.box_lattice(Lb, ref.sog)
    assert info.nlat == len(n3) and info.nshell == len(n3)
    _, cdf, _ = ref.tables()
    assert info.S == cdf[-1]
    n = torch.zeros((w.P, 3), dtype=torch.int32, device=dev)
    coef = torch.zeros(w.P, dtype=torch.float64, device=dev)
    for step in (0, 1, 17, 2 ** 40 + 3):
        R.rbsog_sample_k(s.h, step, n, coef)
        torch.cuda.synchronize()
        no, co = ref.draw(step)
        assert np.array_equal(n.cpu().numpy(), no)
        assert np.array_equal(coef.cpu().numpy().view(np.uint64), co.view(np.uint64))
    cs_o, ord_o, nc_o = oracle.cells_box(st.x, Lb, w.r_c)
    assert (info.nc, info.nc_y, info.nc_z) == tuple(int(v) for v in nc_o)
    cs = torch.zeros(len(cs_o), dtype=torch.int32, device=dev)
    order = torch.zeros(w.N, dtype=torch.int32, device=dev)
    R.rbsog_build_cells(s.h, torch.tensor(st.x, device=dev), cs, order)
    torch.cuda.synchronize()
    assert np.array_equal(cs.cpu().numpy(), cs_o) and np.array_equal(order.cpu().numpy(), ord_o)


@pytest.mark.parametrize("w,stretch", CASES, ids=lambda c: getattr(c, "name", "box"))
@pytest.mark.parametrize("precision", [0, 1])
def test_forces_energies(dev, w, stretch, precision):
    st, Lb, s, ref = _pair(dev, w, stretch, precision)
    x = torch.tensor(st.x, device=dev)
    f = torch.empty_like(x)
    fn = torch.empty_like(x)
    e = torch.zeros(R.ENERGY_COLS, dtype=torch.float64, device=dev)
    R.rbsog_compute_forces(s.h, 5, x, f, fn, e)
    torch.cuda.synchronize()
    fo, fno, eo = ref.force(st.x, 5)
    tol = 1e-12 if precision == 0 else 1e-5
    f, fn, e = f.cpu().numpy(), fn.cpu().numpy(), e.cpu().numpy()
    assert _rel(f, fo) <= tol and _rel(fn, fno) <= tol and _rel(f - fn, fo - fno) <= tol
    for k in (0, 1):
        assert abs(e[k] - eo[k]) <= tol * abs(eo[k])
    for k in (2, 3, 4):
        assert abs(e[k] - eo[k]) <= 1e-13 * max(1.0, abs(eo[k]))
    assert abs(e[6] - eo[6]) <= tol * (abs(eo[6]) + abs(eo[0]))
    assert abs(e[7] - eo[7]) <= max(tol, 1e-11) * (abs(eo[7]) + 3 * abs(eo[1]))


def test_full_lattice(dev):
    w, stretch = CASES[0]
    st, Lb, s, ref = _pair(dev, w, stretch, full_k=True)
    x = torch.tensor(st.x, device=dev)
    f = torch.empty_like(x)
    e = torch.zeros(R.ENERGY_COLS, dtype=torch.float64, device=dev)
    R.rbsog_compute_forces(s.h, 0, x, f, None, e)
    torch.cuda.synchronize()
    fo, _, eo = ref.force(st.x, 0)
    assert _rel(f.cpu().numpy(), fo) <= 1e-12
    assert abs(e.cpu().numpy()[1] - eo[1]) <= 1e-12 * abs(eo[1])


def test_trajectory(dev):
    w, stretch = CASES[0]
    st, Lb, s, ref = _pair(dev, w, stretch)
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
    Lv = np.asarray(Lb)[:, None]
    d = x.cpu().numpy() - xo
    d -= Lv * np.round(d / Lv)
    assert np.abs(d).max() <= 1e-10
    assert np.all(x.cpu().numpy() < Lv) and np.all(x.cpu().numpy() >= 0)


def test_refusals(dev):
    w, stretch = CASES[0]
    st, Lb = _case(w, stretch)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    for kw in ({"sampler": R.RBSOG_SAMPLER_MH}, {"mmax": 40}):
        with pytest.raises(R.RbsogError):
            R.rbsog_workspace_size(R.make_params(w.N, Lb, w.kT, w.P, 1, **kw), sog)
    ens = R.rbsog_ens_create(1 << 28, 2)
    try:
        with pytest.raises(R.RbsogError):
            R.rbsog_ens_admit(ens, R.make_params(w.N, Lb, w.kT, w.P, 1), sog, np.ascontiguousarray(st.x),
                              np.ascontiguousarray(st.v), np.ascontiguousarray(st.q), np.ascontiguousarray(st.m), 5,
                              0.01)
    finally:
        R.rbsog_ens_destroy(ens)


@pytest.mark.parametrize("w,stretch", CASES[:2], ids=lambda c: getattr(c, "name", "box"))
def test_rdf(dev, w, stretch):
    """The pair histogram of a cuboid system: equal to the oracle's except for
    pairs the oracle marks as lying on a bin edge."""
    st, Lb, s, ref = _pair(dev, w, stretch)
    hist = torch.zeros(50, dtype=torch.int64, device=dev)
    R.rbsog_rdf(s.h, torch.tensor(st.x, device=dev), w.r_c, 50, hist)
    torch.cuda.synchronize()
    c, amb = oracle.rdf(st.x, Lb, w.r_c, 50)
    h = hist.cpu().numpy()
    assert np.all(np.abs(h - c) <= amb)
    assert abs(int(h.sum()) - int(c.sum())) <= int(amb.sum())

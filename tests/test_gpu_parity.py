"""Parity of the gfx950 library (through its C-ABI) with the FP64 CPU oracle on
identical seeded inputs: sampled modes and cell lists bit-exact, structure
factors and forces within 1e-12 relative RMS in FP64 and 1e-5 in mixed
precision, energies, and the velocity-Verlet trajectory."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2501_10946_amd")

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


PER_ITEM = 10.0   # no single particle (or mode) may be off by more than 10x the RMS tolerance


def assert_close(a, b, tol, what="", per=PER_ITEM):
    """Relative RMS of a - b over all components within tol, and the largest
    per-item error (a particle of a [3, N] force array, a mode of a [P, 2]
    structure-factor array) within per * tol of the RMS item magnitude of b.
    Comparisons after a run of steps take a larger `per`: the two states then
    differ by the trajectory's rounding, which the steep pair force of a close
    pair magnifies for that particle alone."""
    a, b = np.asarray(a), np.asarray(b)
    r = rel(a, b)
    assert r <= tol, f"{what}: relative RMS {r:.3e} > {tol:.1e}"
    axis = 0 if (a.ndim == 2 and a.shape[0] == 3) else -1
    d = np.linalg.norm(a - b, axis=axis)
    scale = float(np.sqrt(np.mean(np.linalg.norm(b, axis=axis) ** 2)))
    worst = float(d.max()) / scale
    assert worst <= per * tol, f"{what}: largest item error {worst:.3e} of the RMS magnitude"


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return torch.device("cuda:0")


class Case:
    """One system on both sides: the oracle's SOG parameters expanded by the
    library (so both use the same coefficients bit for bit)."""

    def __init__(self, dev, w: workloads.Workload, precision=0, density=0, state=None, mmax=0, skin=-1.0):
        print(f"\n[case] {w.name} N={w.N} P={w.P} prec={precision} dens={density} skin={skin}", flush=True)
        self.w = w
        self.st = state or workloads.make_state(w)
        self.o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        self.sog = R.sog_from_parameters(self.o.lam, self.o.rc, self.o.h, self.o.t0, self.o.w, self.o.M1, self.o.M2)
        self.sys = R.System(self.st.q, self.st.m, w.L, self.sog, w.kT, w.P, seed=w.seed, precision=precision,
                            density=density, mmax=mmax, skin=skin, device=dev)
        self.ref = oracle.System(self.st.q, self.st.m, w.L, self.o, w.kT, w.P, seed=w.seed, density=density,
                                 mmax=mmax)
        self.dev = dev
        self.x = torch.tensor(self.st.x, device=dev)

    def forces(self, step, x=None):
        x = self.x if x is None else x
        f = torch.empty_like(x)
        fn = torch.empty_like(x)
        e = torch.zeros(R.ENERGY_COLS, dtype=torch.float64, device=self.dev)
        R.rbsog_compute_forces(self.sys.h, step, x, f, fn, e)
        torch.cuda.synchronize()
        return f.cpu().numpy(), fn.cpu().numpy(), e.cpu().numpy()


SMALL = [
    workloads.OCP_1K,
    workloads.Workload("ragged_n777_p300", N=777, kappa=1.0, gamma=1.0, r_c=3.0, P=300, seed=5),
    workloads.Workload("n1_single", N=1, kappa=1.0, gamma=1.0, r_c=0.5, P=7, seed=3),
    workloads.Workload("nc3_exact_k2", N=150, kappa=2.0, gamma=3.0, r_c=2.5, P=1, seed=8),
    workloads.Workload("mix_n5000", N=5000, kappa=0.5, gamma=5.0, r_c=4.0, P=64, seed=12, frac_b=0.1, q_b=5.0,
                       m_b=20.0),
    # many modes: six far-kernel sample tiles, partial-sum groups split over workgroups
    workloads.Workload("manymodes_n3000_p1500", N=3000, kappa=0.8, gamma=2.0, r_c=3.5, P=1500, seed=31),
]


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
@pytest.mark.parametrize("density", [0, 1, 2, 3])
def test_samples_bit_exact(dev, w, density):
    c = Case(dev, w, density=density)
    info = R.rbsog_get_info(c.sys.h)
    assert info.mmax == c.ref.mmax and info.nshell == c.ref.nshell
    n = torch.zeros((w.P, 3), dtype=torch.int32, device=dev)
    coef = torch.zeros(w.P, dtype=torch.float64, device=dev)
    for step in (0, 1, 17, 2 ** 40 + 3):
        R.rbsog_sample_k(c.sys.h, step, n, coef)
        torch.cuda.synchronize()
        no, co = c.ref.draw(step)
        assert np.array_equal(n.cpu().numpy(), no)
        assert np.array_equal(coef.cpu().numpy().view(np.uint64), co.view(np.uint64))


@pytest.mark.parametrize("w", SMALL + [workloads.OCP_100K], ids=lambda w: w.name)
def test_cells_bit_exact(dev, w):
    c = Case(dev, w)
    nc = int(math.floor(w.L / w.r_c))
    cs = torch.zeros(nc ** 3 + 1, dtype=torch.int32, device=dev)
    order = torch.zeros(w.N, dtype=torch.int32, device=dev)
    x = c.st.x.copy()
    x[0, : min(3, w.N)] = 0.0                       # edges: x = 0 and the largest x < L
    x[1, : min(3, w.N)] = np.nextafter(w.L, 0)
    xt = torch.tensor(x, device=dev)
    for _ in range(2):                               # rebuilding gives the same list
        R.rbsog_build_cells(c.sys.h, xt, cs, order)
        torch.cuda.synchronize()
        cso, oo = oracle.cells(x, w.L, w.r_c)
        assert np.array_equal(cs.cpu().numpy(), cso)
        assert np.array_equal(order.cpu().numpy(), oo)


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
@pytest.mark.parametrize("precision", [0, 1])
def test_rho(dev, w, precision):
    c = Case(dev, w, precision=precision)
    rho = torch.zeros((w.P, 2), dtype=torch.float64, device=dev)
    for step in (0, 5):
        R.rbsog_compute_rho(c.sys.h, step, c.x, rho)
        torch.cuda.synchronize()
        n3, coef = c.ref.draw(step)
        ro = oracle.rho(c.st.x, c.st.q, w.L, n3)
        tol = FP64_TOL if precision == 0 else MIXED_TOL
        assert_close(rho.cpu().numpy(), ro, tol, "rho")


# the default skin, and no skin (lists of r_c, rebuilt at every step: how hot systems run)
SKINS = [-1.0, 0.0]


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("skin", SKINS, ids=["skin", "noskin"])
def test_forces_and_energy(dev, w, precision, skin):
    c = Case(dev, w, precision=precision, skin=skin)
    tol = FP64_TOL if precision == 0 else MIXED_TOL
    for step in (0, 3):
        f, fn, e = c.forces(step)
        fo, fno, eo = c.ref.force(c.st.x, step)
        if w.N > 1:
            assert_close(f, fo, tol, "total")
            if np.linalg.norm(fno) > 0:
                assert_close(fn, fno, tol, "near")
            assert_close(f - fn, fo - fno, tol, "far")
        else:
            assert np.abs(f - fo).max() <= 1e-12 and np.abs(fn).max() == 0.0
        for k in (0, 1):
            assert abs(e[k] - eo[k]) <= tol * max(abs(eo[k]), 1e-300) + (1e-300 if eo[k] == 0 else 0)
        assert np.allclose(e[2:5], eo[2:5], rtol=1e-13, atol=0)
        assert_virials(e, eo, tol)


def assert_virials(e, eo, tol):
    """Near and far virials of an energy row against the oracle's, relative to
    the size of their terms (the far virial's mode terms change sign)."""
    assert abs(e[6] - eo[6]) <= tol * (abs(eo[6]) + abs(eo[0])), f"W_N {e[6]} vs {eo[6]}"
    assert abs(e[7] - eo[7]) <= tol * (abs(eo[7]) + 3 * abs(eo[1])), f"W_F {e[7]} vs {eo[7]}"


def test_forces_repeatable(dev):
    """Two evaluations of the same input give the same bits (fixed-order reductions)."""
    c = Case(dev, workloads.OCP_1K)
    a = c.forces(9)
    b = c.forces(9)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("precision", [0, 1])
def test_trajectory_small_ocp(dev, precision):
    """The small one-component plasma for 100 velocity-Verlet steps: positions
    agree with the oracle's trajectory to 1e-10 in FP64 (1e-4 mixed), and so do
    the per-step energies."""
    w = workloads.OCP_1K
    c = Case(dev, w, precision=precision)
    x = c.x.clone()
    v = torch.tensor(c.st.v, device=dev)
    f, _, _ = c.forces(0)
    ft = torch.tensor(f, device=dev)
    eh = torch.zeros((w.steps, R.ENERGY_COLS), dtype=torch.float64, device=dev)
    R.rbsog_step(c.sys.h, x, v, ft, 0, w.steps, w.dt, eh)
    R.rbsog_check(c.sys.h)
    xo, vo = c.st.x.copy(), c.st.v.copy()
    fo, _, _ = c.ref.force(xo, 0)
    eho = c.ref.run(xo, vo, fo, 0, w.steps, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    tol = 1e-10 if precision == 0 else 1e-4
    assert np.abs(d).max() <= tol
    ehn = eh.cpu().numpy()
    E, Eo = ehn[:, :6].sum(1), eho[:, :6].sum(1)
    assert np.abs(E - Eo).max() <= (1e-9 if precision == 0 else 1e-3) * np.abs(Eo).max()
    Wv, Wo = ehn[:, 6:].sum(1), eho[:, 6:].sum(1)
    assert np.abs(Wv - Wo).max() <= (1e-9 if precision == 0 else 1e-3) * np.abs(Wo).max()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("skin", SKINS, ids=["skin", "noskin"])
def test_clustered_cells(dev, precision, skin):
    """A third of the particles packed into a cube of edge 2.5 around the box
    corner: cells there hold ~100 particles (several 64-particle home chunks
    per cell pair in the list build), the cluster wraps around every face, and
    lists are long.  Forces and energies as for the uniform cases."""
    w = workloads.Workload("cluster_n3000", N=3000, kappa=1.0, gamma=1.0, r_c=3.0, P=64, seed=77)
    st = workloads.clustered_state(w, frac=1.0 / 3.0, side=2.5)
    c = Case(dev, w, precision=precision, state=st, skin=skin)
    f, fn, e = c.forces(3)
    fo, fno, eo = c.ref.force(st.x, 3)
    tol = FP64_TOL if precision == 0 else MIXED_TOL
    assert_close(f, fo, tol, "total")
    assert_close(fn, fno, tol, "near")
    assert_close(f - fn, fo - fno, tol, "far")
    assert abs(e[0] - eo[0]) <= tol * abs(eo[0])


@pytest.mark.parametrize("precision", [0, 1])
def test_split_calls_bit_exact(dev, precision):
    """A run of 30 steps in one rbsog_step call and the same run in calls of
    7, 1, 0 and 22 steps end in the same bits (x, v, f and the energy history):
    moving the state into cell order and back at each call, and the first
    step of a call drifting in its own kernel rather than in the far kernel
    of the step before, change no arithmetic."""
    w = workloads.OCP_1K
    runs = []
    for split in ([30], [7, 1, 0, 22]):
        c = Case(dev, w, precision=precision)
        x = c.x.clone()
        v = torch.tensor(c.st.v, device=dev)
        f, _, _ = c.forces(0)
        ft = torch.tensor(f, device=dev)
        eh = torch.zeros((30, R.ENERGY_COLS), dtype=torch.float64, device=dev)
        s0 = 0
        for n in split:
            R.rbsog_step(c.sys.h, x, v, ft, s0, n, w.dt, eh[s0:])
            s0 += n
        R.rbsog_check(c.sys.h)
        torch.cuda.synchronize()
        runs.append([t.cpu().numpy() for t in (x, v, ft, eh)])
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def _sampled_reference(c, step, idx):
    """Oracle forces on the particles idx only: near field by the subset pair sum,
    far field from the full structure factors of the same sampled modes."""
    w, st = c.w, c.st
    n3, coef = c.ref.draw(step)
    rho = oracle.rho(st.x, st.q, w.L, n3)
    fn = oracle.near_subset(st.x, st.q, w.L, c.o, idx)
    ff = oracle.far_rb(st.x[:, idx], st.q[idx], w.L, n3, coef, rho)
    return fn + ff, fn, rho


@pytest.mark.parametrize("w,skin", [(workloads.OCP_100K, -1.0), (workloads.MIXTURE_200K, -1.0),
                                    (workloads.OCP_1M_WEAK, 0.0), (workloads.OCP_1M_WEAK, -1.0),
                                    (workloads.OCP_1M_STRONG, 0.0), (workloads.OCP_1M_STRONG, -1.0)],
                         ids=lambda v: v.name if hasattr(v, "name") else ("noskin" if v == 0 else "skin"))
@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_sampled(dev, w, skin, precision):
    """At the full workload sizes, in the launch configurations the benchmark
    times (the N = 1e6 plasmas step with no skin, on the finer grid of lists
    of r_c): forces on 256 sampled particles (and all structure factors)
    against the oracle computed for those particles alone."""
    c = Case(dev, w, precision=precision, skin=skin)
    step = 11
    f, fn, e = c.forces(step)
    rng = np.random.default_rng(w.seed)
    idx = np.sort(rng.choice(w.N, 256, replace=False))
    fo, fno, rho_o = _sampled_reference(c, step, idx)
    tol = FP64_TOL if precision == 0 else MIXED_TOL
    assert_close(f[:, idx], fo, tol, "total")
    assert_close(fn[:, idx], fno, tol, "near")
    assert_close(f[:, idx] - fn[:, idx], fo - fno, tol, "far")
    rho = torch.zeros((w.P, 2), dtype=torch.float64, device=dev)
    R.rbsog_compute_rho(c.sys.h, step, c.x, rho)
    torch.cuda.synchronize()
    assert_close(rho.cpu().numpy(), rho_o, tol, "rho")


def test_full_size_steps_hot(dev):
    """The N = 1e6 weak-coupling plasma (k_B T = 10, fast particles: the default
    skin drops to 0 at the first step and lists of r_c are rebuilt every step
    on the finer grid) for two velocity-Verlet steps in FP64: all positions
    agree with the oracle's steps to 1e-10, and so do the velocities (1e-9)."""
    w = workloads.OCP_1M_WEAK
    c = Case(dev, w)
    assert R.rbsog_get_info(c.sys.h).skin > 0
    x = c.x.clone()
    v = torch.tensor(c.st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(c.sys.h, 0, x, f)
    nsteps = 2
    R.rbsog_step(c.sys.h, x, v, f, 0, nsteps, w.dt)
    R.rbsog_check(c.sys.h)
    info = R.rbsog_get_info(c.sys.h)
    assert info.skin == 0.0 and info.nf == int(math.floor(2 * w.L / w.r_c))
    print("[case] oracle steps at N = 1e6", flush=True)
    xo, vo = c.st.x.copy(), c.st.v.copy()
    fo, _, _ = c.ref.force(xo, 0)
    c.ref.run(xo, vo, fo, 0, nsteps, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= 1e-10
    assert np.abs(v.cpu().numpy() - vo).max() <= 1e-9
    assert_close(f.cpu().numpy(), fo, FP64_TOL, "force after the steps", per=1000.0)


def test_invalid_arguments(dev):
    """Errors are reported, not crashed on: a box below 3 cells, a null pointer,
    a workspace that is too small."""
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    sog = R.rbsog_sog_init(w.lam, w.r_c, 1e-4)
    q = torch.tensor(st.q, device=dev)
    m = torch.tensor(st.m, device=dev)
    bad = R.make_params(w.N, 2.5 * w.r_c, w.kT, w.P, 1)
    with pytest.raises(R.RbsogError) as ei:
        R.rbsog_workspace_size(bad, sog)
    assert ei.value.code == R.RBSOG_EINVAL
    p = R.make_params(w.N, w.L, w.kT, w.P, 1)
    need = R.rbsog_workspace_size(p, sog)
    small = torch.empty(need // 16, dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError) as ei:
        R.rbsog_create(p, sog, q, m, small)
    assert ei.value.code == R.RBSOG_EWORKSPACE


def test_nonfinite_flag(dev):
    """A NaN position yields a non-finite force, reported by rbsog_check."""
    c = Case(dev, workloads.OCP_1K)
    x = c.x.clone()
    x[0, 5] = float("nan")
    f = torch.empty_like(x)
    R.rbsog_compute_forces(c.sys.h, 0, x, f)
    with pytest.raises(R.RbsogError) as ei:
        R.rbsog_check(c.sys.h)
    assert ei.value.code == R.RBSOG_ENONFINITE
    R.rbsog_check(c.sys.h)  # the flag was cleared


@pytest.mark.parametrize("cap", [1, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_neighbour_list_overflow(dev, cap, precision, monkeypatch):
    """With the neighbour-list capacity forced tiny, every lane overflows and
    finishes its pairs by walking the cells: forces and energies unchanged,
    right after a build (rbsog_compute_forces) and after particles have
    drifted since the last build (steps with a skin, lists kept between
    rebuilds)."""
    monkeypatch.setenv("RBSOG_NEAR_CAPACITY", str(cap))
    w = workloads.Workload("ragged_n2000_cap", N=2000, kappa=0.5, gamma=2.0, r_c=4.0, P=50, seed=21)
    c = Case(dev, w, precision=precision)
    tol = FP64_TOL if precision == 0 else MIXED_TOL
    f, fn, e = c.forces(4)
    fo, fno, eo = c.ref.force(c.st.x, 4)
    assert_close(fn, fno, tol, "near")
    assert_close(f, fo, tol, "total")
    assert abs(e[0] - eo[0]) <= tol * abs(eo[0])
    # steps: the default skin stays (a cold plasma), so lists outlive the steps between rebuilds
    assert R.rbsog_get_info(c.sys.h).near_capacity == cap
    x = c.x.clone()
    v = torch.tensor(c.st.v, device=dev)
    ft = torch.tensor(fo, device=dev)
    nsteps = 12
    R.rbsog_step(c.sys.h, x, v, ft, 0, nsteps, w.dt)
    R.rbsog_check(c.sys.h)
    assert R.rbsog_get_info(c.sys.h).skin > 0
    xo, vo, ffo = c.st.x.copy(), c.st.v.copy(), fo.copy()
    c.ref.run(xo, vo, ffo, 0, nsteps, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= (1e-10 if precision == 0 else 1e-5)
    assert_close(ft.cpu().numpy(), ffo, tol if precision == 0 else 1e-4, "force after the steps", per=1000.0)


@pytest.mark.parametrize("skin", [0.0, 0.3, 1.5])
def test_trajectory_independent_of_skin(dev, skin):
    """The neighbour-list skin changes only when lists are rebuilt: 60 steps of
    the small plasma give the oracle's trajectory (1e-10) for any skin,
    including rebuilding every step (0) and rarely (1.5)."""
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, skin=skin, device=dev)
    assert abs(s.info.skin - skin) <= 1e-12
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    R.rbsog_step(s.h, x, v, f, 0, 60, w.dt)
    R.rbsog_check(s.h)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    xo, vo = st.x.copy(), st.v.copy()
    fo, _, _ = ref.force(xo, 0)
    ref.run(xo, vo, fo, 0, 60, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= 1e-10


@pytest.mark.parametrize("gamma,hot", [(1.0, False), (0.01, True)])
def test_default_skin_adapts(dev, gamma, hot):
    """The default skin (0.125 r_c) stays for a cold plasma and drops to 0 at
    the first step of a hot one, whose fastest thermal velocity component
    would cross skin/2 within two steps; the trajectory is the oracle's either
    way (1e-10)."""
    w = workloads.Workload(f"skin_default_g{gamma}", N=1000, kappa=1.0, gamma=gamma, r_c=3.0, P=100, seed=41)
    st = workloads.make_state(w)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, device=dev)
    skin0 = R.rbsog_get_info(s.h).skin
    assert abs(skin0 - 0.125 * w.r_c) <= 1e-12
    x = torch.tensor(st.x, device=dev)
    v = torch.tensor(st.v, device=dev)
    f = torch.empty_like(x)
    R.rbsog_compute_forces(s.h, 0, x, f)
    nsteps = 30
    R.rbsog_step(s.h, x, v, f, 0, nsteps, w.dt)
    R.rbsog_check(s.h)
    skin1 = R.rbsog_get_info(s.h).skin
    assert skin1 == (0.0 if hot else skin0)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed)
    xo, vo = st.x.copy(), st.v.copy()
    fo, _, _ = ref.force(xo, 0)
    ref.run(xo, vo, fo, 0, nsteps, w.dt)
    d = x.cpu().numpy() - xo
    d -= w.L * np.round(d / w.L)
    assert np.abs(d).max() <= 1e-10


FULLK = [
    workloads.OCP_1K,
    workloads.Workload("fullk_ragged_n777", N=777, kappa=1.0, gamma=1.0, r_c=3.0, P=300, seed=5),
    workloads.Workload("fullk_mix_n2000", N=2000, kappa=0.5, gamma=5.0, r_c=4.0, P=64, seed=12, frac_b=0.1, q_b=5.0,
                       m_b=20.0),
]


@pytest.mark.parametrize("w", FULLK, ids=lambda w: w.name)
@pytest.mark.parametrize("precision", [0, 1])
def test_full_k_forces_and_energy(dev, w, precision):
    """The deterministic full-lattice far field (full_k = 1) against the
    oracle's full-lattice sum (eqs. 3.5 and UF without sampling): forces,
    their far part, and the far energy; the result is the same at any
    evaluation index (nothing is sampled)."""
    st = workloads.make_state(w)
    o = oracle.sog_auto(w.lam, w.r_c, w.eps)
    sog = R.sog_from_parameters(o.lam, o.rc, o.h, o.t0, o.w, o.M1, o.M2)
    print(f"\n[case] full_k {w.name} N={w.N} prec={precision}", flush=True)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=w.seed, precision=precision, full_k=True, device=dev)
    ref = oracle.System(st.q, st.m, w.L, o, w.kT, w.P, seed=w.seed, full_k=True)
    x = torch.tensor(st.x, device=dev)
    outs = []
    for step in (3, 11):
        f = torch.empty_like(x)
        fn = torch.empty_like(x)
        e = torch.zeros(R.ENERGY_COLS, dtype=torch.float64, device=dev)
        R.rbsog_compute_forces(s.h, step, x, f, fn, e)
        torch.cuda.synchronize()
        outs.append((f.cpu().numpy(), fn.cpu().numpy(), e.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][2], outs[1][2])
    f, fn, e = outs[0]
    fo, fno, eo = ref.force(st.x, 3)
    tol = FP64_TOL if precision == 0 else MIXED_TOL
    assert_close(f, fo, tol, "total")
    assert_close(f - fn, fo - fno, tol, "far")
    assert abs(e[1] - eo[1]) <= tol * abs(eo[1])
    assert np.allclose(e[[0, 2, 3, 4]], eo[[0, 2, 3, 4]], rtol=tol, atol=0)
    assert_virials(e, eo, tol)


def test_full_k_refuses_sampling_calls(dev):
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    sog = R.rbsog_sog_init(w.lam, w.r_c, 1e-4)
    s = R.System(st.q, st.m, w.L, sog, w.kT, w.P, seed=1, full_k=True, device=dev)
    n = torch.zeros((w.P, 3), dtype=torch.int32, device=dev)
    coef = torch.zeros(w.P, dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError) as ei:
        R.rbsog_sample_k(s.h, 0, n, coef)
    assert ei.value.code == R.RBSOG_EINVAL
    rho = torch.zeros((w.P, 2), dtype=torch.float64, device=dev)
    with pytest.raises(R.RbsogError) as ei:
        R.rbsog_compute_rho(s.h, 0, torch.tensor(st.x, device=dev), rho)
    assert ei.value.code == R.RBSOG_EINVAL

"""The served ensemble (rbsog_ens_* through the C-ABI): a replica advanced
together with others of different sizes, screening lengths, mode counts,
Gaussian counts and precisions, admitted at different ensemble steps, ends in
exactly (bit for bit) the state and energy history of the same system stepped
alone; an FP64 replica follows the oracle's trajectory; admission control,
polling, retirement and the step timeline behave as declared."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2501_10946_amd")

DT = 0.01


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.lib()
    return torch.device("cuda:0")


class Req:
    """One replica's inputs: workload, state, SOG, parameters."""

    def __init__(self, w: workloads.Workload, replica: int, precision: int, nsteps: int):
        self.w = w
        self.st = workloads.make_state(w)
        self.o = oracle.sog_auto(w.lam, w.r_c, w.eps)
        self.sog = R.sog_from_parameters(self.o.lam, self.o.rc, self.o.h, self.o.t0, self.o.w, self.o.M1, self.o.M2)
        self.params = R.make_params(w.N, w.L, w.kT, w.P, 104, replica, 0, precision)
        self.precision = precision
        self.replica = replica
        self.nsteps = nsteps

    def admit(self, ens):
        return R.rbsog_ens_admit(ens, self.params, self.sog, np.ascontiguousarray(self.st.x),
                                 np.ascontiguousarray(self.st.v), np.ascontiguousarray(self.st.q),
                                 np.ascontiguousarray(self.st.m), self.nsteps, DT)

    def alone(self, dev):
        """The same system stepped alone: force index 0, then nsteps steps."""
        s = R.System(self.st.q, self.st.m, self.w.L, self.sog, self.w.kT, self.w.P, seed=104, replica=self.replica,
                     precision=self.precision, device=dev)
        x = torch.tensor(self.st.x, device=dev)
        v = torch.tensor(self.st.v, device=dev)
        f = torch.empty_like(x)
        e = torch.zeros((self.nsteps, R.ENERGY_COLS), dtype=torch.float64, device=dev)
        R.rbsog_compute_forces(s.h, 0, x, f)
        R.rbsog_step(s.h, x, v, f, 0, self.nsteps, DT, e)
        torch.cuda.synchronize()
        R.rbsog_check(s.h)
        return x.cpu().numpy(), v.cpu().numpy(), e.cpu().numpy()


def mixed_set():
    W = workloads.Workload
    return [
        Req(W("e_a", N=700, kappa=1.0, gamma=1.0, r_c=3.0, P=100, seed=31), 0, R.RBSOG_FP64, 12),
        Req(W("e_b", N=2600, kappa=0.5, gamma=10.0, r_c=4.0, P=200, seed=32), 1, R.RBSOG_MIXED, 20),
        Req(W("e_c", N=1500, kappa=2.0, gamma=0.5, r_c=4.0, P=37, seed=33), 2, R.RBSOG_FP64, 7),
        Req(W("e_d", N=900, kappa=0.2, gamma=3.0, r_c=4.0, P=300, seed=34), 3, R.RBSOG_MIXED, 15),
        # hot (k_B T = 20): the default skin drops to 0 at admission, as at the
        # first step of the system stepped alone
        Req(W("e_hot", N=1500, kappa=1.0, gamma=0.05, r_c=4.0, P=200, seed=35), 4, R.RBSOG_MIXED, 10),
        # long screening length: seven Gaussians, mixed precision
        Req(W("e_k01", N=4000, kappa=0.1, gamma=1.0, r_c=4.0, P=200, seed=36), 5, R.RBSOG_MIXED, 8),
        # the largest request size of the served workload
        Req(W("e_big", N=40000, kappa=0.5, gamma=10.0, r_c=4.0, P=200, seed=37), 6, R.RBSOG_FP64, 6),
    ]


def run_ensemble(reqs, late, budget=1 << 30, max_slots=8):
    """Admits reqs (those in `late` after three ensemble steps), steps until all
    are done, retires them; returns {index: (x, v, energy_hist)}."""
    ens = R.rbsog_ens_create(budget, max_slots)
    try:
        slot_of = {}
        for i, r in enumerate(reqs):
            if i not in late:
                slot_of[i] = r.admit(ens)
        for _ in range(3):
            R.rbsog_ens_step(ens)
        for i in late:
            slot_of[i] = reqs[i].admit(ens)
        out = {}
        inv = {s: i for i, s in slot_of.items()}
        for _ in range(200):
            R.rbsog_ens_step(ens)
            torch.cuda.synchronize()
            for s in R.rbsog_ens_poll(ens, max_slots):
                r = reqs[inv[s]]
                x = np.empty(3 * r.w.N)
                v = np.empty(3 * r.w.N)
                e = np.empty(R.ENERGY_COLS * r.nsteps)
                R.rbsog_ens_retire(ens, s, x, v, e)
                out[inv[s]] = (x.reshape(3, -1), v.reshape(3, -1), e.reshape(-1, R.ENERGY_COLS))
            if len(out) == len(reqs):
                break
        assert R.rbsog_ens_status(ens)["resident"] == 0
        return out
    finally:
        R.rbsog_ens_destroy(ens)


def test_ensemble_equals_alone(dev):
    reqs = mixed_set()
    assert reqs[5].sog.n == 7
    print(f"\n[ensemble] {len(reqs)} replicas, two admitted late", flush=True)
    out = run_ensemble(reqs, late={2, 4})
    assert sorted(out) == list(range(len(reqs)))
    for i, r in enumerate(reqs):
        x, v, e = out[i]
        xa, va, ea = r.alone(dev)
        assert np.array_equal(x, xa), f"replica {i}: positions differ from the system stepped alone"
        assert np.array_equal(v, va), f"replica {i}: velocities differ"
        assert np.array_equal(e, ea), f"replica {i}: energy history differs"
        assert np.all(np.isfinite(e))


def test_ensemble_replica_follows_oracle(dev):
    """An FP64 replica's positions after 5 steps agree with the oracle's
    velocity-Verlet run of the same system (force indices 0..5)."""
    r = Req(workloads.Workload("e_o", N=600, kappa=1.0, gamma=1.0, r_c=3.0, P=80, seed=41), 5, R.RBSOG_FP64, 5)
    out = run_ensemble([r, mixed_set()[1]], late=set())
    x, v, e = out[0]
    ref = oracle.System(r.st.q, r.st.m, r.w.L, r.o, r.w.kT, r.w.P, seed=104, replica=5)
    xo = r.st.x.copy()
    vo = r.st.v.copy()
    fo, _, _ = ref.force(xo, 0)
    ref.run(xo, vo, fo, 0, r.nsteps, DT)
    d = x - xo
    d -= r.w.L * np.rint(d / r.w.L)
    assert np.max(np.abs(d)) < 1e-10
    assert np.max(np.abs(v - vo)) < 1e-9


def test_ensemble_admission_and_timeline(dev):
    W = workloads.Workload
    big = Req(W("e_big", N=3000, kappa=0.5, gamma=10.0, r_c=4.0, P=200, seed=51), 0, R.RBSOG_MIXED, 4)
    small = Req(W("e_small", N=800, kappa=1.0, gamma=1.0, r_c=3.0, P=50, seed=52), 1, R.RBSOG_FP64, 3)
    need = R.rbsog_ens_bytes(big.params, big.sog, big.nsteps)
    assert need < R.rbsog_workspace_size(big.params, big.sog) + 11 * 8 * 3000 + R.ENERGY_COLS * 8 * 4 + 4096
    ens = R.rbsog_ens_create(need, 4)
    try:
        slot = big.admit(ens)
        with pytest.raises(R.RbsogError) as ei:
            small.admit(ens)           # the pool holds one replica of this size
        assert ei.value.code == R.RBSOG_EAGAIN
        st = R.rbsog_ens_status(ens)
        assert st["resident"] == 1 and st["active"] == 1
        for _ in range(4):
            assert R.rbsog_ens_poll(ens, 4) == []
            R.rbsog_ens_step(ens)
        R.rbsog_ens_step(ens)          # no active replica left: nothing to do
        torch.cuda.synchronize()
        assert R.rbsog_ens_poll(ens, 4) == [slot]
        assert R.rbsog_ens_poll(ens, 4) == []          # reported once
        times = [R.rbsog_ens_step_time(ens, k) for k in range(1, 5)]
        assert all(t > 0 for t in times) and times == sorted(times)
        with pytest.raises(R.RbsogError):
            R.rbsog_ens_step_time(ens, 0)
        R.rbsog_ens_retire(ens, slot)
        with pytest.raises(R.RbsogError):
            R.rbsog_ens_retire(ens, slot)               # already retired
        slot2 = small.admit(ens)                        # fits once the first is gone
        st = R.rbsog_ens_status(ens)
        assert st["resident"] == 1 and st["ens_steps"] == 4
        with pytest.raises(R.RbsogError):
            R.rbsog_ens_retire(ens, slot2)              # steps left
    finally:
        R.rbsog_ens_destroy(ens)


def test_ensemble_slot_limit(dev):
    W = workloads.Workload
    reqs = [Req(W(f"e_s{i}", N=500, kappa=1.0, gamma=1.0, r_c=3.0, P=20, seed=60 + i), i, R.RBSOG_MIXED, 2)
            for i in range(3)]
    ens = R.rbsog_ens_create(1 << 28, 2)
    try:
        reqs[0].admit(ens)
        reqs[1].admit(ens)
        with pytest.raises(R.RbsogError) as ei:
            reqs[2].admit(ens)
        assert ei.value.code == R.RBSOG_EAGAIN
    finally:
        R.rbsog_ens_destroy(ens)

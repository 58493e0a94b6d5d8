"""Seeded synthetic inputs for Yukawa one-component plasmas and mixtures.

This module holds only input generation: system sizes, box lengths and the
random positions, velocities, charges and masses of the workloads.  It does none
of the method's arithmetic, and both the GPU library's tests and the CPU oracle
draw their inputs from it.

Units are reduced: Wigner-Seitz radius a = 1, so the number density is
n = 3/(4 pi), the volume is V = 4 pi N / 3 and the box length L = V^(1/3);
lambda = 1/kappa; k_B T = 1/Gamma (Gamma = q^2/(a k_B T) with q = 1).

The five workloads follow the systems of the paper's numerical section
(Section 5): Yukawa one-component plasmas over a range of coupling and
screening, and a two-species mixture standing in for its deuterium-alpha
application.  All are synthetic; no dataset is involved.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One system: sizes, physics parameters and the seeds of its inputs."""

    name: str
    N: int
    kappa: float          # a / lambda
    gamma: float          # coupling; k_B T = 1/gamma
    r_c: float            # near-field cutoff
    P: int                # random-batch size
    eps: float = 1e-4     # SOG tolerance (Table 1, second row, is what the paper runs)
    dt: float = 0.01
    steps: int = 100
    seed: int = 1
    # second species (mixture): fraction of particles, charge and mass
    frac_b: float = 0.0
    q_b: float = 1.0
    m_b: float = 1.0

    @property
    def lam(self) -> float:
        return 1.0 / self.kappa

    @property
    def kT(self) -> float:
        return 1.0 / self.gamma

    @property
    def V(self) -> float:
        return 4.0 * math.pi * self.N / 3.0

    @property
    def L(self) -> float:
        return self.V ** (1.0 / 3.0)

    @property
    def n_b(self) -> int:
        return int(round(self.frac_b * self.N))


# The workloads.  The first is small enough for the oracle to finish in
# seconds; the second is the configuration throughput is quoted on.
OCP_1K = Workload("ocp_n1000_k1_g1", N=1000, kappa=1.0, gamma=1.0, r_c=3.0, P=100, steps=100, seed=101)
OCP_100K = Workload("ocp_n100000_k0.5_g10", N=100_000, kappa=0.5, gamma=10.0, r_c=4.0, P=200, steps=500,
                    seed=102)
OCP_1M_WEAK = Workload("ocp_n1000000_k0.1_g0.1", N=1_000_000, kappa=0.1, gamma=0.1, r_c=5.0, P=500, steps=200,
                       seed=103)
OCP_1M_STRONG = Workload("ocp_n1000000_k0.1_g100", N=1_000_000, kappa=0.1, gamma=100.0, r_c=5.0, P=500,
                         steps=200, seed=113)
MIXTURE_200K = Workload("mix_n200000_k0.5_g5", N=200_000, kappa=0.5, gamma=5.0, r_c=4.0, P=300, steps=500,
                        seed=105, frac_b=0.1, q_b=5.0, m_b=20.0)

ALL = [OCP_1K, OCP_100K, OCP_1M_WEAK, OCP_1M_STRONG, MIXTURE_200K]

# The fluctuation comparison of the sampling densities (Section 5.3, Fig. 8):
# a one-component plasma of 1000 particles with P = 20 modes per step over
# effective couplings Gamma* = Gamma (1 + kappa + kappa^2) exp(-kappa) from
# 1e-3 to 100.  The paper gives lambda and r_c in Angstrom (r_c = 5 lambda) but
# not the density of this run; r_c = 5 lambda is kept, and kappa = 1 (lambda =
# a) so that the box of 1000 particles at the reduced density holds three cells
# of width r_c.
VARIANCE_GAMMA_STAR = (1e-3, 1e-2, 1e-1, 1.0, 10.0, 100.0)
VARIANCE_KAPPA = 1.0


def gamma_from_effective(gamma_star: float, kappa: float) -> float:
    """The coupling Gamma whose effective coupling (Section 5.1) is gamma_star."""
    return gamma_star / ((1.0 + kappa + kappa * kappa) * math.exp(-kappa))


def variance_workload(gamma_star: float, seed: int = 301) -> Workload:
    kappa = VARIANCE_KAPPA
    return Workload(f"ocp_n1000_k1_gstar{gamma_star:g}", N=1000, kappa=kappa,
                    gamma=gamma_from_effective(gamma_star, kappa), r_c=5.0 / kappa, P=20, steps=0, seed=seed,
                    dt=0.01 * min(1.0, math.sqrt(gamma_from_effective(gamma_star, kappa))))


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """numpy Generator on a Philox bit stream keyed by (seed, stream)."""
    return np.random.Generator(np.random.Philox(key=np.array([seed, stream], dtype=np.uint64)))


def positions(N: int, L: float, seed: int) -> np.ndarray:
    """i.i.d. uniform positions in [0, L)^3, SoA float64 array of shape (3, N)."""
    x = rng(seed, 0).random((3, N)) * L
    x[x >= L] = 0.0
    return np.ascontiguousarray(x)


def charges_masses(w: Workload) -> tuple[np.ndarray, np.ndarray]:
    """Charges and masses: species A (q = 1, m = 1) first, then species B."""
    q = np.ones(w.N)
    m = np.ones(w.N)
    nb = w.n_b
    if nb:
        q[w.N - nb:] = w.q_b
        m[w.N - nb:] = w.m_b
    return q, m


def velocities(m: np.ndarray, kT: float, seed: int) -> np.ndarray:
    """Maxwell velocities N(0, kT/m) per component, centre-of-mass motion
    removed, rescaled so that the kinetic energy is (3N - 3) kT / 2."""
    N = m.shape[0]
    v = rng(seed, 1).standard_normal((3, N)) * np.sqrt(kT / m)[None, :]
    vcm = (v * m[None, :]).sum(axis=1) / m.sum()
    v -= vcm[:, None]
    ke = 0.5 * float((m[None, :] * v * v).sum())
    target = 0.5 * (3 * N - 3) * kT
    if ke > 0:
        v *= math.sqrt(target / ke)
    return np.ascontiguousarray(v)


@dataclasses.dataclass
class State:
    x: np.ndarray
    v: np.ndarray
    q: np.ndarray
    m: np.ndarray


def make_state(w: Workload, seed: Optional[int] = None) -> State:
    s = w.seed if seed is None else seed
    q, m = charges_masses(w)
    return State(x=positions(w.N, w.L, s), v=velocities(m, w.kT, s), q=q, m=m)


def clustered_state(w: Workload, frac: float, side: float, seed: Optional[int] = None) -> State:
    """The workload's state with a fraction `frac` of the particles moved into
    a cube of edge `side` centred on the box corner (so the cluster wraps
    around every face): cells there hold far more particles than the mean."""
    st = make_state(w, seed)
    g = rng(w.seed if seed is None else seed, 11)
    n = int(round(frac * w.N))
    idx = g.choice(w.N, size=n, replace=False)
    x = st.x.copy()
    x[:, idx] = np.mod(g.uniform(-0.5 * side, 0.5 * side, (3, n)), w.L)
    x[x >= w.L] = 0.0
    return State(x=np.ascontiguousarray(x), v=st.v, q=st.q, m=st.m)


def small_system(N: int, L: float, seed: int, neutral: bool = False, qmax: float = 1.0) -> State:
    """A tiny test system in an arbitrary box: uniform positions, charges
    uniform in [-qmax, qmax] shifted to sum to zero when neutral, else all
    positive in [0.5, 1.5] qmax; unit masses; unit-variance velocities."""
    g = rng(seed, 7)
    x = g.random((3, N)) * L
    x[x >= L] = 0.0
    if neutral:
        q = g.uniform(-qmax, qmax, N)
        q -= q.mean()
    else:
        q = g.uniform(0.5 * qmax, 1.5 * qmax, N)
    m = np.ones(N)
    v = g.standard_normal((3, N))
    return State(x=np.ascontiguousarray(x), v=np.ascontiguousarray(v), q=q, m=m)


def served_requests(n_req: int = 256, seed: int = 104, arrival_seed: int = 204, rate: float = 1.0):
    """The served-ensemble request stream: N log-uniform in [500, 5e4], Gamma
    log-uniform in [0.1, 100], kappa uniform in [0.1, 2], r_c = 4, P = 200,
    100 steps each, Poisson arrivals at `rate` requests per unit time.
    Returns a list of (arrival_time, Workload) in arrival order."""
    g = rng(seed, 3)
    ga = rng(arrival_seed, 4)
    out: List[tuple[float, Workload]] = []
    t = 0.0
    for i in range(n_req):
        N = int(round(math.exp(g.uniform(math.log(500), math.log(5e4)))))
        gamma = math.exp(g.uniform(math.log(0.1), math.log(100.0)))
        kappa = g.uniform(0.1, 2.0)
        t += ga.exponential(1.0 / rate)
        out.append((t, Workload(f"req{i}", N=N, kappa=kappa, gamma=gamma, r_c=4.0, P=200, steps=100,
                                seed=seed * 100000 + i)))
    return out

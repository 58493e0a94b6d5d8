"""Pins of the oracle's virials: W = -3V dU/dV with the configuration scaled
together with the box (r -> s r, L -> s L), checked against central finite
differences of the oracle's own energies, for the near field (both of its pair
searches), the full-lattice far field (with the lattice of modes held fixed)
and a whole system's energy row; and the unbiasedness of the random-batch
estimator of the far virial over many draws (the importance weights of eq.
UF).  The virial makes the pressure P = (2 KE + W) / (3V)."""
import math

import numpy as np
import pytest

import workloads


def _scaled(x, s):
    return np.ascontiguousarray(x * s)


def _fd(fun, h=1e-6):
    """-dU/ds at s = 1, which is -3V dU/dV for V proportional to s^3."""
    return -(fun(1.0 + h) - fun(1.0 - h)) / (2.0 * h)


@pytest.mark.parametrize("N,rc", [(300, 2.0), (3000, 3.0)])
def test_near_virial_is_volume_derivative(orc, N, rc):
    """Image loop (N = 300) and cell-list search (N = 3000): the near virial
    equals the finite-difference volume derivative of U_N.  U_N has no jump
    at r_c (N and N' vanish there), so pairs crossing r_c under the scaling
    do not spoil the difference."""
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=21)
    s = orc.sog_auto(1.0, rc, 1e-4)
    _, U, W = orc.near(st.x, st.q, L, s, virial=True)
    Wfd = _fd(lambda a: orc.near(_scaled(st.x, a), st.q, L * a, s)[1])
    assert abs(W - Wfd) <= 1e-8 * (abs(W) + abs(U)), (W, Wfd)


def test_far_full_virial_is_volume_derivative(orc):
    N, rc = 200, 2.0
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=22, neutral=True)
    s = orc.sog_auto(1.0, rc, 1e-4)
    mmax = orc.mmax_default(s, L)
    _, U, W = orc.far_full(st.x, st.q, L, s, mmax, virial=True)
    Wfd = _fd(lambda a: orc.far_full(_scaled(st.x, a), st.q, L * a, s, mmax)[1])
    assert abs(W - Wfd) <= 1e-7 * (abs(W) + abs(U)), (W, Wfd)
    assert abs(W - 3 * U) > 1e-3 * abs(U)   # the k-dependence of Fhat contributes


def test_system_virial_row(orc):
    """Full-lattice system: W_N + W_F + 3 (U_k0 + U_bg) is -3V dU/dV of the
    whole energy row's potential part (U_self does not depend on V), for a
    charged (non-neutral) system so that U_k0 and U_bg enter."""
    N, rc = 250, 2.0
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=23)
    s = orc.sog_auto(1.0, rc, 1e-4)
    mmax = orc.mmax_default(s, L)

    def potential(a):
        sysm = orc.System(st.q, st.m, L * a, s, 1.0, 10, seed=1, mmax=mmax, full_k=True)
        _, _, e = sysm.force(_scaled(st.x, a), 0)
        return e[:5].sum(), e

    U, e = potential(1.0)
    W = e[6] + e[7] + 3.0 * (e[2] + e[4])
    Wfd = _fd(lambda a: potential(a)[0])
    assert abs(W - Wfd) <= 1e-7 * (abs(e[:5]).sum() + abs(W)), (W, Wfd)


def test_random_batch_virial_unbiased(orc):
    """The mean of the far-field virial estimator over 4000 independent draws
    is the full-lattice virial (within five standard errors), for the adaptive
    and the flat densities."""
    N, rc, P = 100, 3.0, 20
    L = (4 * math.pi * N / 3) ** (1 / 3)
    st = workloads.small_system(N, L, seed=31)
    s = orc.sog_auto(1.0, rc, 1e-4)
    for density in (0, 1):
        sysm = orc.System(st.q, st.m, L, s, 1.0, P, seed=31, density=density)
        _, _, Wfull = orc.far_full(st.x, st.q, L, s, sysm.mmax, virial=True)
        Ws = []
        for b in range(4000):
            n3, coef = sysm.draw(b)
            rho = orc.rho(st.x, st.q, L, n3)
            Ws.append(orc.far_rb_virial(n3, coef, rho, L, s))
        Ws = np.array(Ws)
        z = (Ws.mean() - Wfull) / (Ws.std(ddof=1) / math.sqrt(Ws.size))
        assert abs(z) <= 5, (density, Ws.mean(), Wfull, z)


def test_energy_row_carries_virials(orc):
    """The random-batch system's row: W_N equals the near field's virial and
    W_F the estimator's for the drawn modes."""
    w = workloads.OCP_1K
    st = workloads.make_state(w)
    s = orc.sog_auto(w.lam, w.r_c, w.eps)
    sysm = orc.System(st.q, st.m, w.L, s, w.kT, w.P, seed=w.seed)
    _, _, e = sysm.force(st.x, 7)
    _, _, WN = orc.near(st.x, st.q, w.L, s, virial=True)
    n3, coef = sysm.draw(7)
    rho = orc.rho(st.x, st.q, w.L, n3)
    assert e[6] == WN
    assert e[7] == orc.far_rb_virial(n3, coef, rho, w.L, s)

"""Pins of the oracle's SOG decomposition (Section 3, Algorithm 1) against
what the paper prints and against the mathematics it rests on."""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE1 = np.loadtxt(os.path.join(HERE, "golden", "table1_c1_sog.txt"))
LAM = 0.5773
RC = 5 * LAM
U = 2.0 ** -53


def rows():
    for eps, h, t0, M1, M2, Mtot, w in TABLE1:
        yield float(eps), float(h), float(t0), int(M1), int(M2), int(Mtot), float(w)


@pytest.mark.parametrize("row", list(rows()), ids=lambda r: f"eps{r[0]:.0e}")
def test_table1_step_size(orc, row):
    """eq. (2.30) with delta = r_c reproduces every printed h to the printed
    precision (15 decimals, i.e. +-5e-16) plus a few ulp."""
    eps, h, *_ = row
    assert abs(orc.h_star(eps, RC) - h) <= 5e-16 + 4 * U * h


@pytest.mark.parametrize("row", list(rows()), ids=lambda r: f"eps{r[0]:.0e}")
def test_table1_printed_set_is_c0_c1(orc, row):
    """The printed (h, t0, w) make the decomposition continuous in value (eq. 2.38)
    and in force (eq. 1.25) at r_c, to FP64 rounding of the terms."""
    eps, h, t0, M1, M2, Mtot, w = row
    assert M1 + M2 + 1 == Mtot
    y = orc.lib().orc_yukawa(RC, LAM)
    yp = orc.lib().orc_yukawa_dr(RC, LAM)
    c0 = y - orc.sog_far(LAM, h, t0, w, M1, M2, RC)
    assert abs(c0) <= 64 * U * y
    # C1 residual with w eliminated through eq. (2.42), evaluated at the printed t0
    c1 = orc.sog_c1_residual(LAM, RC, h, t0, M1, M2)
    assert abs(c1) <= 64 * U * abs(yp)


@pytest.mark.parametrize("row", list(rows()), ids=lambda r: f"eps{r[0]:.0e}")
def test_table1_c1_root(orc, row):
    """Given the printed (h, M1, M2), the smallest C1 root in [0,h) with w > 0 is
    the printed t0, within 16x the FP64 conditioning of the root, which is
    |Y'(r_c)| u / |dR/dt0| for the C1 residual R (the residual is flat in t0 at
    high accuracy, so the last printed digits are not determined in FP64)."""
    eps, h, t0, M1, M2, Mtot, w = row
    s = orc.sog_c1(LAM, RC, h, M1, M2)
    d = 1e-6
    dR = (orc.sog_c1_residual(LAM, RC, h, t0 + d, M1, M2) - orc.sog_c1_residual(LAM, RC, h, t0 - d, M1, M2)) / (2 * d)
    cond = abs(orc.lib().orc_yukawa_dr(RC, LAM)) * 2 * U / abs(dR)
    assert abs(s.t0 - t0) <= 16 * cond + 2e-15
    # w follows from eq. (2.42); compare at the printed t0 within the
    # conditioning of that quotient, u Y(r_c) / (h f(t_M2, r_c)).
    fM2 = orc.lib().orc_f(t0 + M2 * h, RC, LAM)
    wcond = 2 * U * orc.lib().orc_yukawa(RC, LAM) / (h * fM2)
    assert abs(orc.sog_w(LAM, RC, h, t0, M1, M2) - w) <= 16 * wcond + 4 * U


@pytest.mark.parametrize("row", list(rows()), ids=lambda r: f"eps{r[0]:.0e}")
def test_theorem_1_1_bound(orc, row):
    """|Y(r) - F(r)| <= eps on [r_c, 33 lambda] for every Table 1 row (Theorem 1.1,
    with the range of Section 3.2), on a dense grid."""
    eps, h, t0, M1, M2, Mtot, w = row
    s = orc.sog_c1(LAM, RC, h, M1, M2)
    assert orc.sog_maxerr(s) <= eps
    r = np.linspace(RC, 33 * LAM, 20001)
    err = np.abs(np.exp(-r / LAM) / r - s.F(r))
    assert err.max() <= eps


def test_integral_representation(orc):
    """eq. (ftr): Y(r) = int f(t, r) dt, by adaptive quadrature in 30 digits."""
    mpmath.mp.dps = 30
    for lam in (0.5773, 2.0, 10.0):
        for r in (0.3, 1.0, 4.0):
            val = mpmath.quad(lambda t: orc.lib().orc_f(float(t), r, lam), [-40, -10, 0, 10, 40])
            assert abs(float(val) - math.exp(-r / lam) / r) <= 1e-12 * math.exp(-r / lam) / r


def test_expanded_form_matches_paper_form(orc):
    """The expanded coefficients c_j, s_j give the same F(r) as the paper's
    h [w f(t_M2, r) + sum f(t_m, r)] (eq. 2.41), and F(0) = sum c_j."""
    s = orc.sog_auto(2.0, 4.0, 1e-4)
    for r in np.linspace(0.0, 40.0, 81):
        a = orc.sog_far(s.lam, s.h, s.t0, s.w, s.M1, s.M2, float(r))
        b = float(s.F(r))
        assert abs(a - b) <= 1e-14 * max(abs(a), 1e-300)
    assert abs(s.F0 - float(s.F(0.0))) <= 1e-15 * s.F0


def test_fourier_transform_of_sog(orc):
    """Fhat(k) = sum A_j exp(-B_j k^2) is the 3-D Fourier transform of F(r):
    4 pi int_0^inf sin(kr)/k F(r) r dr (radial transform of Section 3.3), by quadrature."""
    s = orc.sog_auto(1.0, 3.0, 1e-6)
    for k in (0.05, 0.3, 1.0, 2.5):
        val, _ = integrate.quad(lambda r: 4 * math.pi * math.sin(k * r) / k * float(s.F(r)) * r, 0, 80, limit=400,
                                epsabs=1e-14, epsrel=1e-12)
        assert abs(val - float(s.Fhat(k * k))) <= 1e-9 * abs(val)
    # k = 0: 4 pi int F r^2 dr
    val, _ = integrate.quad(lambda r: 4 * math.pi * float(s.F(r)) * r * r, 0, 80, limit=400, epsrel=1e-12)
    assert abs(val - s.Fhat0) <= 1e-9 * val


@pytest.mark.parametrize("lam,rc", [(1.0, 3.0), (2.0, 4.0), (10.0, 5.0), (0.5, 4.0)])
def test_auto_rule(orc, lam, rc):
    """The automatic (M1, M2) choice meets the bound of Theorem 1.1, is C1, has
    a positive weight, and no set with fewer Gaussians passes (checked by trying
    every smaller M_tot with every split)."""
    eps = 1e-4
    s = orc.sog_auto(lam, rc, eps)
    assert s.err <= eps and s.w > 0 and 0 <= s.t0 < s.h
    yp = orc.lib().orc_yukawa_dr(rc, lam)
    assert abs(orc.sog_c1_residual(lam, rc, s.h, s.t0, s.M1, s.M2)) <= 1e-12 * abs(yp)
    h = orc.h_star(eps, rc)
    for mt in range(1, s.n):
        for M2 in range(-12, mt):
            M1 = mt - 1 - M2
            try:
                t = orc.sog_c1(lam, rc, h, M1, M2)
            except ValueError:
                continue
            assert orc.sog_maxerr(t) > eps

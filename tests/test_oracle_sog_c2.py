"""Pins of the oracle's C2-continuous SOG decomposition (Appendix C, eq. c2):
the potential, its first and its second derivative of Y - F vanish at r_c
(checked by finite differences of the expanded sum, independent of the
residual the root finder solves), the error bound holds on [r_c, 33 lambda],
the adjusted Gaussian stays the narrowest, no set with one Gaussian fewer
meets the tolerance, sigma = 1 reproduces the C1 expansion bit for bit, and
the closed form of Y'' matches finite differences.  Table 2's printed rows
are not a pin (they do not satisfy their own conditions); its h column is
eq. (2.30), pinned with Table 1."""
import math

import numpy as np
import pytest

LAM = 0.5773
RC = 5 * LAM


def _Y(r, lam=LAM):
    return math.exp(-r / lam) / r


def _D(s, r):
    return _Y(r, s.lam) - float(s.F(np.array([r]))[0])


@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-5, 1e-7, 1e-9, 1e-11])
def test_c2_conditions_and_error(orc, eps):
    s = orc.sog_auto2(LAM, RC, eps)
    assert s.smooth == 2 and s.w > 0 and s.sigma > math.exp(-s.h)
    y0, y1 = _Y(RC), abs(-_Y(RC) * (1 / LAM + 1 / RC))
    dr = 1e-3 * RC
    D = [_D(s, RC + k * dr) for k in (-2, -1, 0, 1, 2)]
    d1 = (D[0] - 8 * D[1] + 8 * D[3] - D[4]) / (12 * dr)
    d2 = (-D[0] + 16 * D[1] - 30 * D[2] + 16 * D[3] - D[4]) / (12 * dr * dr)
    assert abs(D[2]) <= 1e-12 * y0
    assert abs(d1) <= 1e-9 * y1
    assert abs(d2) <= 1e-6 * orc.lib().orc_yukawa_dr2(RC, LAM)
    # the bound on the grid, recomputed from the expanded coefficients
    R = 33 * LAM
    u = np.arange(1601) / 1600.0
    r = RC + (R - RC) * u * u
    err = np.abs(np.exp(-r / LAM) / r - s.F(r)).max()
    assert err <= eps and abs(err - s.err) <= 1e-3 * eps
    # the adjusted Gaussian is the narrowest
    assert s.s[-1] == s.s.max()


@pytest.mark.parametrize("eps", [1e-4, 1e-7])
def test_c2_auto_is_minimal(orc, eps):
    s = orc.sog_auto2(LAM, RC, eps)
    h = orc.h_star(eps, RC)
    fewer = s.n - 1
    for M2 in range(-12, fewer):
        M1 = fewer - 1 - M2
        if M1 < 0:
            continue
        try:
            t = orc.sog_c2(LAM, RC, h, M1, M2)
        except ValueError:
            continue
        assert orc.lib().orc_sog_maxerr2(LAM, RC, h, t.t0, t.w, t.sigma, M1, M2) > eps


def test_sigma_one_is_the_c1_expansion(orc):
    s1 = orc.sog_auto(LAM, RC, 1e-5)
    t = orc.SOG(s1.lam, s1.rc, s1.h, s1.t0, s1.w, s1.M1, s1.M2, sigma=1.0).expand()
    for a, b in ((s1.c, t.c), (s1.s, t.s), (s1.A, t.A), (s1.B, t.B)):
        assert np.array_equal(a, b)


def test_yukawa_second_derivative(orc):
    for r in (0.3, 1.7, 4.0):
        for lam in (0.5, 2.0):
            d = 1e-4 * r
            fd = (_Y(r - d, lam) - 2 * _Y(r, lam) + _Y(r + d, lam)) / (d * d)
            assert abs(orc.lib().orc_yukawa_dr2(r, lam) - fd) <= 1e-6 * abs(fd)


def test_table2_step_column(orc):
    """Table 2's h column (C2 sets) is the step of eq. (2.30) at each eps."""
    table2_h = {1e-3: 1.131155934143089, 1e-4: 0.894984933518395, 1e-5: 0.740391708745519,
                1e-7: 0.550285792019561, 1e-9: 0.437859267899280, 1e-11: 0.363578174148321,
                1e-13: 0.310844614243983}
    for eps, h in table2_h.items():
        assert abs(orc.h_star(eps, RC) - h) <= 5e-16 + 4 * 2.0 ** -53 * h   # printed to 15 decimals

"""Pins for the oracle's changeover functions W and K (eq. (cutfuncW) and the
integral relation between W and K, Section 2.1.1).

The oracle evaluates W as printed and K = W - y W'.  These tests pin it to
things other than itself:
  * the closed form K = 35x^4 - 84x^5 + 70x^6 - 20x^7, x = (y - g)/(1 - g),
    obtained by simplifying W - yW' symbolically (the y ln y terms cancel),
    evaluated here in 40-digit arithmetic; a single mistyped coefficient of
    f would break it;
  * the defining integral W(y)/y = int_y^inf K(s)/s^2 ds by quadrature;
  * continuity of W at y = gamma (ties the constant c to f) and at y = 1;
  * the stated limits: K = 0 below r_in = gamma r_out, K = 1 above r_out.
"""
import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

GAMMAS = [0.05, 0.1, 0.2, 0.5]


def _smooth(y, g):
    mp.mp.dps = 40
    y, g = mp.mpf(y), mp.mpf(g)
    x = (y - g) / (1 - g)
    x = min(max(x, mp.mpf(0)), mp.mpf(1))
    return 35 * x**4 - 84 * x**5 + 70 * x**6 - 20 * x**7


def _smooth_dy(y, g):
    mp.mp.dps = 40
    y, g = mp.mpf(y), mp.mpf(g)
    x = (y - g) / (1 - g)
    if x <= 0 or x >= 1:
        return mp.mpf(0)
    return 140 * x**3 * (1 - x) ** 3 / (1 - g)


@pytest.mark.parametrize("g", GAMMAS)
def test_K_equals_closed_form(orc, g):
    ys = np.concatenate([np.linspace(0.0 + 1e-6, 1.3, 257), [g, g + 1e-12, 1 - 1e-12, 1.0]])
    got = orc.K(ys, g)
    ref = np.array([float(_smooth(y, g)) for y in ys])
    # long-double evaluation of f - y f' loses ~ eps_ld * |coefficients| / |g-1|^7
    assert np.max(np.abs(got - ref)) < 3e-15 * max(1.0, (1 - g) ** -7 / 4)


@pytest.mark.parametrize("g", GAMMAS)
def test_dKdy_equals_closed_form(orc, g):
    ys = np.linspace(g + 1e-3, 1 - 1e-3, 199)
    got = orc.dKdy(ys, g)
    ref = np.array([float(_smooth_dy(y, g)) for y in ys])
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("g", GAMMAS)
def test_K_limits(orc, g):
    assert np.all(orc.K(np.linspace(0, g * (1 - 1e-12), 50), g) == 0.0)
    assert np.all(orc.K(np.linspace(1.0, 50.0, 50), g) == 1.0)
    assert abs(orc.K(g * (1 + 1e-9), g)) < 1e-12
    assert abs(orc.K(1 - 1e-9, g) - 1.0) < 1e-12


@pytest.mark.parametrize("g", GAMMAS)
def test_W_continuity(orc, g):
    eps = 1e-10
    assert abs(orc.W(g * (1 - eps), g) - orc.W(g * (1 + eps), g)) < 1e-8
    assert abs(orc.W(1 - eps, g) - 1.0) < 1e-8
    assert orc.W(1.0, g) == 1.0 and orc.W(7.0, g) == 1.0


@pytest.mark.parametrize("g", GAMMAS)
def test_integral_relation(orc, g):
    """W(y) / y = int_y^inf K(s) / s^2 ds (the definition of K)."""
    for y in [0.3 * g, g, 0.5 * (1 + g), 0.9, 1.0, 2.0]:
        lo = max(y, g)
        inner = 0.0
        if lo < 1.0:
            inner, _ = integrate.quad(lambda s: float(orc.K(s, g)) / s**2, lo, 1.0, epsabs=1e-14, epsrel=1e-13,
                                      limit=200)
        tail = 1.0 / max(y, 1.0)  # int_max(y,1)^inf 1/s^2 ds
        assert abs(orc.W(y, g) / y - (inner + tail)) < 1e-10 * (inner + tail)


@pytest.mark.parametrize("g", GAMMAS)
def test_dWdy_matches_finite_difference(orc, g):
    for y in np.linspace(g + 0.01, 0.99, 17):
        h = 1e-6
        fd = (orc.W(y + h, g) - orc.W(y - h, g)) / (2 * h)
        assert abs(fd - orc.dWdy(y, g)) < 1e-7


def test_K_monotone_in_range(orc):
    ys = np.linspace(0.1, 1.0, 500)
    k = orc.K(ys, 0.1)
    assert np.all(np.diff(k) >= -1e-15)

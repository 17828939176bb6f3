"""Pins for the oracle's prior covariance (Sec. 1 turbulence spectrum read as
Matern nu = 1/3; compact-support taper) and its quadrature rule."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import epo


def test_gk15_polynomial_exactness():
    xk, wk, wg = epo.gk15_rule()
    xs = np.concatenate([-xk[:7], [0.0], xk[6::-1]])
    ws = np.concatenate([wk[:7], [wk[7]], wk[6::-1]])
    gx = np.concatenate([-xk[1:7:2], [0.0], xk[5::-2]])
    gw = np.concatenate([wg[:3], [wg[3]], wg[2::-1]])
    for k in range(0, 23):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(ws, xs ** k) - exact) < 1e-14, k
        if k <= 13:
            assert abs(np.dot(gw, gx ** k) - exact) < 1e-14, k
    # G7 is not exact at degree 14: the embedded error estimate is live
    assert abs(np.dot(gw, gx ** 14) - 2.0 / 15) > 1e-6


@pytest.mark.parametrize("x", [0.01, 0.1, 0.5, 0.63, 1.0, 1.5, 2.36, 5.0])
def test_besselk_matches_independent_route(x):
    # scipy's kv (Amos/Temme) is a different route from the integral
    # representation the oracle integrates.
    assert epo.besselk(1.0 / 3.0, x) == pytest.approx(special.kv(1.0 / 3.0, x), rel=1e-13)


def test_besselk_half_integer_closed_form():
    # K_{1/2}(x) = sqrt(pi / 2x) e^{-x}
    for x in [0.2, 1.0, 3.0]:
        assert epo.besselk(0.5, x) == pytest.approx(math.sqrt(math.pi / (2 * x)) * math.exp(-x), rel=1e-13)


def test_matern_limits():
    assert epo.matern13(1.7, 100.0, 0.0) == 1.7
    # small-r behaviour: 1 - C(r)/var -> Gamma(1-nu)/Gamma(1+nu) (x/2)^{2 nu}
    nu = 1.0 / 3.0
    coef = math.gamma(1 - nu) / math.gamma(1 + nu)
    for r in [1e-3, 1e-2]:
        x = r / 100.0
        lhs = 1.0 - epo.matern13(1.0, 100.0, r)
        rhs = coef * (x / 2) ** (2 * nu)
        assert lhs == pytest.approx(rhs, rel=5 * x ** (2 - 2 * nu) / coef + 1e-9)
    # monotone decreasing, positive
    rs = np.linspace(1, 500, 60)
    c = np.array([epo.matern13(1.0, 100.0, r) for r in rs])
    assert np.all(np.diff(c) < 0) and np.all(c > 0)


def test_wendland_taper_shape():
    rs = 150.0
    assert epo.wendland(rs, 0.0) == 1.0
    assert epo.wendland(rs, rs) == 0.0 and epo.wendland(rs, 2 * rs) == 0.0
    h = 1e-4
    # C^2 smooth at the support edge and flat at the origin (one-sided)
    w = lambda r: epo.wendland(rs, r)
    assert abs((w(rs) - w(rs - h)) / h) < 1e-6
    assert abs((w(h) - w(0)) / h) < 1e-3


def test_tapered_covariance_positive_definite():
    rng = np.random.default_rng(0)
    pts = rng.random((300, 3)) * 600.0
    r = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    K = np.vectorize(lambda x: epo.cov(1.0, 100.0, 150.0, x))(r)
    assert np.linalg.eigvalsh(K).min() > 0.0
    # taper zero beyond the support, Matern inside
    assert epo.cov(1.0, 100.0, 150.0, 151.0) == 0.0
    x = 80.0
    assert epo.cov(1.0, 100.0, 150.0, x) == pytest.approx(epo.matern13(1.0, 100.0, x) * epo.wendland(150.0, x), rel=1e-15)

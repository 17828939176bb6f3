"""Pins for the oracle's tilted moments: cavity N(a; mu, v) times the
extinction likelihood N(A | e^a, s^2) (the per-star tilted distribution and
its first two moments, Sec. 4.1 and App. A.2)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import epo


def _brute(mu, v, A, s, lo, hi, m=1_000_001):
    a = np.linspace(lo, hi, m)
    ell = -(a - mu) ** 2 / (2 * v) - (A - np.exp(a)) ** 2 / (2 * s * s)
    mx = ell.max()
    w = np.exp(ell - mx)
    I0 = np.trapezoid(w, a)
    m1 = np.trapezoid(a * w, a) / I0
    m2 = np.trapezoid((a - m1) ** 2 * w, a) / I0
    lnZ = mx + math.log(I0) - 0.5 * math.log(2 * math.pi * v) - 0.5 * math.log(2 * math.pi * s * s)
    return lnZ, m1, m2


CASES = [
    (-0.5, 0.3, 0.6, 0.05),     # informative star
    (-2.0, 1.0, 0.1, 0.05),     # low extinction, broad cavity
    (0.5, 0.02, 1.7, 0.2),      # tight cavity
    (-6.0, 1.0, 0.2, 0.05),     # bimodal: cavity far below a 4-sigma detection
    (-1.0, 2.0, 0.15, 0.05),    # near-bimodal shoulder
    (-3.0, 0.5, -0.05, 0.05),   # negative observed extinction
    (1.0, 0.1, 2.5, 0.02),      # narrow likelihood, sigma/A ~ 0.01
]


@pytest.mark.parametrize("mu,v,A,s", CASES)
def test_matches_scipy_quad(mu, v, A, s):
    lnZ, mh, vh = (x[0] for x in epo.tilted(0, [mu], [v], [A], [s]))
    f = lambda a: math.exp(-(a - mu) ** 2 / (2 * v) - (A - math.exp(a)) ** 2 / (2 * s * s)) / (
        2 * math.pi * math.sqrt(v) * s)
    pts = [mh - 30 * math.sqrt(vh), mh + 30 * math.sqrt(vh)]
    lo, hi = mu - 40 * math.sqrt(v), max(mu + 40 * math.sqrt(v), math.log(abs(A) + 10 * s) + 1)
    Z = integrate.quad(f, lo, hi, points=pts, epsabs=0, epsrel=1e-13, limit=2000)[0]
    M1 = integrate.quad(lambda a: a * f(a), lo, hi, points=pts, epsabs=0, epsrel=1e-13, limit=2000)[0] / Z
    M2 = integrate.quad(lambda a: (a - M1) ** 2 * f(a), lo, hi, points=pts, epsabs=0, epsrel=1e-12,
                        limit=2000)[0] / Z
    assert lnZ == pytest.approx(math.log(Z), rel=1e-10, abs=1e-11)
    assert mh == pytest.approx(M1, rel=1e-10, abs=1e-11)
    assert vh == pytest.approx(M2, rel=1e-9)


@pytest.mark.parametrize("mu,v,A,s", CASES)
def test_matches_brute_force_trapezoid(mu, v, A, s):
    lnZ, mh, vh = (x[0] for x in epo.tilted(0, [mu], [v], [A], [s]))
    lo = min(mu - 40 * math.sqrt(v), mh - 40 * math.sqrt(vh))
    hi = max(mu + 40 * math.sqrt(v), math.log(abs(A) + 10 * s) + 1)
    hi = min(hi, mh + 40 * math.sqrt(vh) + 5)
    b = _brute(mu, v, A, s, lo, hi)
    assert lnZ == pytest.approx(b[0], abs=1e-7)
    assert mh == pytest.approx(b[1], abs=1e-7)
    assert vh == pytest.approx(b[2], rel=1e-6)


def test_bimodal_case_is_bimodal_and_mass_is_right():
    mu, v, A, s = -6.0, 1.0, 0.2, 0.05
    a = np.linspace(-15, 3, 400001)
    ell = -(a - mu) ** 2 / (2 * v) - (A - np.exp(a)) ** 2 / (2 * s * s)
    d = np.diff(ell)
    assert np.sum((d[:-1] > 0) & (d[1:] <= 0)) == 2   # two local maxima
    lnZ = epo.tilted(0, [mu], [v], [A], [s])[0][0]
    assert lnZ == pytest.approx(_brute(mu, v, A, s, -20, 3, m=2_000_001)[0], abs=1e-8)


def test_broad_likelihood_returns_cavity():
    # s -> infinity: the likelihood is flat in a, the tilted is the cavity
    _, mh, vh = epo.tilted(0, [-0.7], [0.4], [0.5], [1e6])
    assert mh[0] == pytest.approx(-0.7, abs=1e-9)
    assert vh[0] == pytest.approx(0.4, rel=1e-9)


def test_narrow_likelihood_pins_log_extinction():
    # s -> 0 with A > 0: the tilted concentrates at ln A with variance (s/A)^2
    A = 1.3
    for s in [1e-4, 1e-5]:
        _, mh, vh = epo.tilted(0, [-0.2], [0.5], [A], [s])
        assert mh[0] == pytest.approx(math.log(A), abs=5 * (s / A) ** 2 + 1e-12)
        assert vh[0] == pytest.approx((s / A) ** 2, rel=10 * s / A)


def test_gaussian_likelihood_closed_form():
    mu, v, a, s = -0.4, 0.7, 0.3, 0.2
    lnZ, mh, vh = (x[0] for x in epo.tilted(1, [mu], [v], [a], [s]))
    f = lambda t: math.exp(-(t - mu) ** 2 / (2 * v) - (a - t) ** 2 / (2 * s * s)) / (2 * math.pi * math.sqrt(v) * s)
    Z = integrate.quad(f, -20, 20, epsrel=1e-13, points=[a, mu])[0]
    M1 = integrate.quad(lambda t: t * f(t), -20, 20, epsrel=1e-13, points=[a, mu])[0] / Z
    M2 = integrate.quad(lambda t: (t - M1) ** 2 * f(t), -20, 20, epsrel=1e-13, points=[a, mu])[0] / Z
    assert lnZ == pytest.approx(math.log(Z), abs=1e-12)
    assert mh == pytest.approx(M1, abs=1e-12)
    assert vh == pytest.approx(M2, rel=1e-11)


def test_negative_observed_extinction_is_finite():
    lnZ, mh, vh = epo.tilted(0, [-2.0, -5.0], [1.0, 0.5], [-0.3, -0.01], [0.05, 0.02])
    assert np.all(np.isfinite(lnZ)) and np.all(np.isfinite(mh)) and np.all(vh > 0)
    # a negative observation pushes the extinction down
    assert mh[0] < -2.0

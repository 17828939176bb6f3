"""Pins for the FP64 reference of the tilted-moment surrogate network."""
import numpy as np

from oracle import epo, mlp


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    blob = rng.normal(0, 0.2, mlp.NPARAM)
    p = mlp.unpack(blob)
    X = rng.normal(size=(8, 4))
    Y = rng.normal(size=(8, 3))
    _, g = mlp.loss_grad(p, X, Y)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"):
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in p[name].shape)
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += eps
            lp, _ = mlp.loss_grad(q, X, Y)
            q[name][idx] -= 2 * eps
            lm, _ = mlp.loss_grad(q, X, Y)
            assert abs(g[name][idx] - (lp - lm) / (2 * eps)) < 1e-6 * max(1.0, abs(g[name][idx]))


def test_baseline_exact_for_gaussian_like_star():
    # a very precise observation: the tilted distribution is the likelihood's
    # log-space Gaussian times the cavity, which the baseline reproduces
    mu, v, A, s = np.array([-0.3]), np.array([0.2]), np.array([1.1]), np.array([1e-4])
    m0, v0, lnZ0 = mlp.baseline(mu, v, A, s)
    lnZ, mh, vh = epo.tilted(0, mu, v, A, s)
    assert abs(m0[0] - mh[0]) < 1e-6 and abs(v0[0] / vh[0] - 1) < 1e-3
    assert abs(lnZ0[0] - lnZ[0]) < 1e-3


def test_gauss_hermite_check_is_exact_for_gaussian_integrand():
    # with sigma -> infinity the tilted distribution is the cavity Gaussian;
    # an 8-node rule centred at its mean with its scale integrates it to
    # rounding (the integrand over the rule's weight is then a constant)
    mu, v = np.array([-1.2, 0.4]), np.array([0.3, 0.05])
    A, s = np.array([0.5, 2.0]), np.array([1e5, 1e5])
    lnZ, m, var = mlp.gauss_hermite_check(mu, v, A, s, mu, v)
    lz, mh, vh = epo.tilted(0, mu, v, A, s)
    assert np.allclose(m, mh, atol=1e-9) and np.allclose(var, vh, rtol=1e-8)
    assert np.allclose(lnZ, lz, atol=1e-9)

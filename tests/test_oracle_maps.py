"""Pins for the oracle's map predictions (lognormal density moments, the
posterior mean and sampled variance of the extinction to every node, the
two-point density predictive) against closed forms, quadrature, the
oracle's separately pinned sightline operator and Monte Carlo."""
import math

import numpy as np
import pytest

from oracle import epo, maps


def _cfg(n=6, L=500.0, step=2.0, obs=None):
    return dict(n=n, box_pc=L, observer_pc=obs if obs is not None else (L / 2, 0.0, L / 2), prior_mean=-7.0,
                prior_var=1.0, outer_scale_pc=100.0, support_pc=150.0, los_step_pc=step)


def _spd(N, scale, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((N, N)) / math.sqrt(N)
    Q = (B @ B.T + 0.5 * np.eye(N)) / scale
    S = np.linalg.inv(Q)
    return Q, 0.5 * (S + S.T)


@pytest.mark.parametrize("mu,v", [(-7.0, 0.01), (-5.0, 0.5), (0.3, 1.7)])
def test_density_moments_match_quadrature(mu, v):
    x, w = np.polynomial.hermite_e.hermegauss(120)
    w = w / math.sqrt(2 * math.pi)
    vals = np.exp(mu + math.sqrt(v) * x)
    e_q = float(np.sum(w * vals))
    var_q = float(np.sum(w * (vals - e_q) ** 2))
    e, var = maps.density_moments(np.array([mu]), np.array([v]))
    assert abs(e[0] - e_q) < 1e-12 * e_q
    assert abs(var[0] - var_q) < 1e-9 * var_q


def test_trilinear_weights_reproduce_linear_fields():
    cfg = _cfg(n=7, L=600.0)
    n, h = 7, 100.0
    rng = np.random.default_rng(1)
    p = rng.uniform(0, 600.0, (200, 3))
    p[:5] = [[600, 600, 600], [0, 0, 0], [600, 0, 300], [100, 200, 300], [599.999, 0.001, 600]]
    nodes, phi = maps.point_weights(cfg, p)
    assert np.allclose(phi.sum(1), 1.0, atol=1e-14) and phi.min() >= -1e-15
    pos = maps.node_positions(cfg)
    assert np.allclose(pos[:, 0], (np.arange(n ** 3) % n) * h)
    for coef in ([1.3, 0.0, 0.0], [0.0, -0.7, 0.0], [0.0, 0.0, 2.1], [0.3, -1.1, 0.4]):
        f = pos @ np.array(coef) + 0.25
        assert np.allclose(np.sum(phi * f[nodes], 1), p @ np.array(coef) + 0.25, rtol=0, atol=1e-10)


def test_sightlines_match_the_forward_model():
    cfg = _cfg(n=8, L=700.0)
    rng = np.random.default_rng(2)
    xyz = rng.uniform(0, 700.0, (25, 3))
    sl = epo.Sightlines(cfg, xyz)
    f = -6.0 + 0.8 * rng.standard_normal(sl.grid.N)
    _, lnA, _ = sl.linearise(f)
    for k in range(len(xyz)):
        w, nodes, phi = maps.sightline_points(cfg, xyz[k])
        A = float(np.sum(w * np.exp(np.sum(phi * f[nodes], 1))))
        assert abs(A - math.exp(lnA[k])) < 1e-12 * A


def test_extinction_mean_perfectly_correlated_constant_field():
    # f = c + xi with one xi ~ N(0, v) shared by every node: F(s) = c + xi on
    # the whole sightline, A = d e^{c + xi}, so E[A] = d e^{c + v/2}
    n, L = 5, 400.0
    cfg = _cfg(n=n, L=L, obs=(200.0, 0.0, 200.0))          # the observer sits on a node
    N = n ** 3
    c, v = -6.2, 0.37
    mean = maps.extinction_mean(cfg, np.full(N, c), np.full((N, N), v))
    d = np.linalg.norm(maps.node_positions(cfg) - np.array([200.0, 0.0, 200.0]), axis=1)
    assert np.allclose(mean, d * math.exp(c + v / 2), rtol=1e-13, atol=0)
    assert mean[2 + n * 0 + n * n * 2] == 0.0


def test_extinction_mean_matches_monte_carlo():
    n, L = 4, 300.0
    cfg = _cfg(n=n, L=L, step=5.0)
    N = n ** 3
    Q, S = _spd(N, 0.3, seed=4)
    mu = -6.0 + 0.3 * np.random.default_rng(5).standard_normal(N)
    targets = np.array([N - 1, 21, 47, 60])
    exact = maps.extinction_mean(cfg, mu, S, targets)
    K = 100000
    f = np.random.default_rng(6).multivariate_normal(mu, S, size=K)
    pos = maps.node_positions(cfg)
    for k, p in enumerate(targets):
        w, nodes, phi = maps.sightline_points(cfg, pos[p])
        A = np.exp(np.einsum("ta,kta->kt", phi, f[:, nodes])) @ w
        se = A.std() / math.sqrt(K)
        assert abs(A.mean() - exact[k]) < 5 * se, (k, A.mean(), exact[k], se)
        # dropping the variance term would be far outside the noise
        plug = float(np.sum(w * np.exp(np.sum(phi * mu[nodes], 1))))
        assert abs(plug - exact[k]) > 20 * se


def test_posterior_draws_have_covariance_q_inverse():
    # with z = the identity, the draws' deviations D satisfy D^T D = Q^{-1}
    N = 27
    Q, S = _spd(N, 1.0, seed=7)
    perm = np.random.default_rng(8).permutation(N).astype(np.int32)
    mu = np.linspace(-1, 1, N)
    D = maps.posterior_draws(mu, Q, perm, np.eye(N)) - mu[None, :]
    assert np.allclose(D.T @ D, S, rtol=0, atol=1e-12 * np.abs(S).max())
    # the first elimination-order component of z moves only through L^{-T}
    Lp = np.linalg.cholesky(Q[np.ix_(perm, perm)])
    x = np.linalg.solve(Lp.T, np.eye(N)[:, -1])
    assert np.allclose(D[-1][perm], x, atol=1e-13)


def test_sample_variance_converges_to_the_lognormal_variance():
    n, L = 4, 300.0
    cfg = _cfg(n=n, L=L, step=10.0)
    N = n ** 3
    Q, S = _spd(N, 0.15, seed=9)
    mu = np.full(N, -6.0)
    perm = np.arange(N, dtype=np.int32)[::-1].copy()
    targets = np.array([N - 1, 33])
    K = 6000
    z = np.random.default_rng(10).standard_normal((K, N))
    sv = maps.extinction_sample_var(cfg, mu, Q, perm, z, targets)
    pos = maps.node_positions(cfg)
    for k, p in enumerate(targets):
        w, nodes, phi = maps.sightline_points(cfg, pos[p])
        m = np.sum(phi * mu[nodes], 1)
        C = np.einsum("ta,tsab,sb->ts", phi, S[nodes[:, None, :, None], nodes[None, :, None, :]], phi)
        E = np.exp(m + 0.5 * np.diag(C))
        exact = float(w @ (np.expm1(C) * np.outer(E, E)) @ w)
        assert abs(sv[k] - exact) < 0.1 * exact, (sv[k], exact)


def test_point_predict_at_nodes_and_by_monte_carlo():
    n, L = 5, 400.0
    cfg = _cfg(n=n, L=L)
    N = n ** 3
    Q, S = _spd(N, 0.4, seed=11)
    mu = -5.5 + 0.4 * np.random.default_rng(12).standard_normal(N)
    pos = maps.node_positions(cfg)
    i, j = 31, 93
    out = maps.point_predict(cfg, mu, S, np.hstack([pos[i], pos[j]])[None, :])[0]
    e, v = maps.density_moments(mu[[i, j]], S[[i, j], [i, j]])
    assert np.allclose(out[:4], [e[0], e[1], v[0], v[1]], rtol=1e-12)
    assert abs(out[4] - math.expm1(S[i, j]) * e[0] * e[1]) < 1e-12 * abs(out[4])
    # generic points 10 pc apart in neighbouring cells
    rng = np.random.default_rng(13)
    pa = np.array([[151.0, 99.0, 207.0], [33.0, 250.0, 396.0]])
    pb = pa + np.array([[10.0, 0.0, 0.0], [0.0, 6.0, 8.0]])
    out = maps.point_predict(cfg, mu, S, np.hstack([pa, pb]))
    K = 400000
    f = rng.multivariate_normal(mu, S, size=K)
    for r in range(2):
        na, wa = maps.point_weights(cfg, pa[r])
        nb, wb = maps.point_weights(cfg, pb[r])
        ra = np.exp(f[:, na[0]] @ wa[0])
        rb = np.exp(f[:, nb[0]] @ wb[0])
        mc = [ra.mean(), rb.mean(), ra.var(), rb.var(), np.mean((ra - ra.mean()) * (rb - rb.mean()))]
        for k in range(5):
            assert abs(mc[k] - out[r, k]) < 0.02 * abs(out[r, k]), (r, k, mc[k], out[r, k])

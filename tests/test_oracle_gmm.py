"""Pins for the oracle's EP with unknown distances: the distance-marginalised
mixture tilted moments against brute-force 2-D quadrature of the
(ln s, a) integrand, the known-distance limit against the Gaussian tilted
moments, beta = d ln A / d ln s on fields with closed forms, and the EP
plumbing against the Gaussian-likelihood EP."""
import math

import numpy as np
import pytest

from oracle import epo, gmm
from synth import Workload, draw, gmm_catalogue


def _n2(l, b, m, C):
    det = C[0] * C[2] - C[1] ** 2
    dl, db = l - m[0], b - m[1]
    q = (C[2] * dl * dl - 2 * C[1] * dl * db + C[0] * db * db) / det
    return np.exp(-0.5 * q) / (2 * math.pi * math.sqrt(det))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tilted_matches_2d_quadrature(seed):
    rng = np.random.default_rng(seed)
    K = 3
    comps = np.zeros((1, K, 6))
    comps[0, :, 0] = rng.dirichlet(np.ones(K))
    comps[0, :, 1] = math.log(800.0) + rng.normal(0, 0.4, K)
    comps[0, :, 2] = rng.normal(-1.0, 0.5, K)
    sl_, sb_, rho = rng.uniform(0.05, 0.3, K), rng.uniform(0.05, 0.3, K), rng.uniform(-0.8, 0.8, K)
    comps[0, :, 3], comps[0, :, 4], comps[0, :, 5] = sl_ ** 2, rho * sl_ * sb_, sb_ ** 2
    mu_c, v_c = rng.normal(-1.0, 0.3), rng.uniform(0.02, 0.5)
    beta, lref = rng.uniform(0.2, 2.0), math.log(700.0)
    lnZ, mean, var = gmm.gmm_tilted([mu_c], [v_c], comps, [beta], [lref])
    # brute force over (a, l): N(a; mu_c, v_c) sum_z w_z N2((l, a + beta (l - lref)); m_z, C_z)
    a = np.linspace(mu_c - 12 * math.sqrt(v_c), mu_c + 12 * math.sqrt(v_c), 2401)
    lo, hi = comps[0, :, 1].min() - 3.0, comps[0, :, 1].max() + 3.0
    l = np.linspace(lo, hi, 3001)
    A, Lg = np.meshgrid(a, l, indexing="ij")
    f = np.exp(-0.5 * (A - mu_c) ** 2 / v_c) / math.sqrt(2 * math.pi * v_c)
    like = sum(comps[0, z, 0] * _n2(Lg, A + beta * (Lg - lref), comps[0, z, 1:3], comps[0, z, 3:6]) for z in range(K))
    g = f * like
    da, dl = a[1] - a[0], l[1] - l[0]
    Z = g.sum() * da * dl
    m1 = (g * A).sum() * da * dl / Z
    m2 = (g * (A - m1) ** 2).sum() * da * dl / Z
    assert abs(lnZ[0] - math.log(Z)) < 1e-9
    assert abs(mean[0] - m1) < 1e-9 * max(1.0, abs(m1))
    assert abs(var[0] - m2) < 1e-8 * m2


def test_known_distance_is_the_gaussian_likelihood():
    # one component with a vanishing distance spread: a Gaussian likelihood in
    # a with mean m_b - beta (m_l - lref) and variance C_bb
    rng = np.random.default_rng(5)
    S = 50
    comps = np.zeros((S, 1, 6))
    comps[:, 0, 0] = 1.0
    comps[:, 0, 1] = math.log(500.0) + rng.normal(0, 0.2, S)
    comps[:, 0, 2] = rng.normal(-1, 0.4, S)
    comps[:, 0, 3] = 1e-300
    comps[:, 0, 5] = rng.uniform(0.01, 0.2, S) ** 2
    beta, lref = rng.uniform(0.3, 1.5, S), np.full(S, math.log(450.0))
    mu_c, v_c = rng.normal(-1, 0.3, S), rng.uniform(0.01, 0.4, S)
    lz, m, v = gmm.gmm_tilted(mu_c, v_c, comps, beta, lref)
    a_obs = comps[:, 0, 2] - beta * (comps[:, 0, 1] - lref)
    lz2, m2, v2 = epo.tilted(1, mu_c, v_c, a_obs, np.sqrt(comps[:, 0, 5]))
    assert np.allclose(lz, lz2, rtol=0, atol=1e-12)
    assert np.allclose(m, m2, rtol=1e-13, atol=1e-13) and np.allclose(v, v2, rtol=1e-12)


def _cfg(n=8, L=700.0):
    return dict(n=n, box_pc=L, observer_pc=(L / 2, 0.0, L / 2), prior_mean=-7.0, prior_var=1.0,
                outer_scale_pc=100.0, support_pc=150.0, los_step_pc=2.0)


def test_beta_on_constant_and_linear_fields():
    cfg = _cfg()
    rng = np.random.default_rng(3)
    xyz = rng.uniform(50, 650, (30, 3))
    sl = epo.Sightlines(cfg, xyz)
    pos = sl.grid.xyz()
    # constant field: A = d e^c, so d ln A / d ln d = 1
    f = np.full(sl.grid.N, -6.3)
    _, lnA, _ = sl.linearise(f)
    assert np.allclose(gmm.beta_at(cfg, xyz, f, lnA), 1.0, rtol=0, atol=1e-12)
    # linear field F(s) = F0 + k s along each ray (trilinear reproduces it):
    # the continuous A = e^F0 (e^{k d} - 1)/k, beta = k d e^{k d}/(e^{k d} - 1);
    # the trapezoid at 2 pc agrees to O(step^2 k^2)
    kv = np.array([1.5e-3, -1.0e-3, 2.0e-3])
    f = -6.0 + pos @ kv
    _, lnA, _ = sl.linearise(f)
    o = np.asarray(cfg["observer_pc"])
    d = np.linalg.norm(xyz - o, axis=1)
    k = ((xyz - o) / d[:, None]) @ kv
    exact = k * d * np.exp(k * d) / np.expm1(k * d)
    assert np.allclose(gmm.beta_at(cfg, xyz, f, lnA), exact, rtol=1e-5)


def test_degenerate_mixture_ep_is_the_gaussian_ep():
    # every star: one component at the catalogue distance with no distance
    # spread, so beta drops out and the likelihood is N(a; m_b, C_bb): the
    # mixture EP must give the Gaussian-likelihood EP's sites (frozen
    # linearisation in both)
    w = Workload("t", n=7, box_pc=600.0, n_stars=60, sweeps=2, star_law="uniform", d_max_pc=600.0,
                 noise_law="const", noise_a=0.05, likelihood="gauss_linear", seed_id=4)
    cfg = dict(w.ep_fields(), relinearize=False)
    raw = draw(w)
    S = w.n_stars
    o = np.asarray(cfg["observer_pc"])
    comps = np.zeros((S, 1, 6))
    comps[:, 0, 0] = 1.0
    comps[:, 0, 1] = np.log(np.linalg.norm(raw["xyz"] - o, axis=1))
    comps[:, 0, 2] = -1.5 + 0.3 * raw["eps"]
    comps[:, 0, 3] = 1e-300
    comps[:, 0, 5] = raw["sigma"] ** 2
    a = gmm.DenseEPGMM(cfg, raw["xyz"], comps)
    b = epo.DenseEP(cfg, raw["xyz"], comps[:, 0, 2], raw["sigma"])
    for _ in range(2):
        a.sweep()
        b.sweep()
        assert np.allclose(a.tau, b.tau, rtol=1e-12) and np.allclose(a.nu, b.nu, rtol=1e-12, atol=1e-12)
    assert np.allclose(a.posterior_mean(), b.posterior_mean(), rtol=1e-12)


def test_synthetic_catalogue_is_consistent():
    w = Workload("t", n=7, box_pc=600.0, n_stars=400, sweeps=2, star_law="uniform", d_max_pc=600.0, seed_id=5)
    raw = draw(w)
    a_true = np.linspace(-2, 0, w.n_stars)
    cat = gmm_catalogue(w, raw["xyz"], a_true)
    c = cat["comps"]
    assert c.shape == (w.n_stars, 2, 6) and np.allclose(c[:, :, 0].sum(1), 1.0)
    assert np.all(c[:, :, 3] * c[:, :, 5] > c[:, :, 4] ** 2)
    # main component centred on a draw around the truth: standardised
    # residuals have unit spread; catalogue positions lie in the cube on the
    # true directions
    o = np.asarray(w.observer)
    d = np.linalg.norm(raw["xyz"] - o, axis=1)
    zl = (c[:, 0, 1] - np.log(d)) / math.sqrt(c[0, 0, 3])
    zb = (c[:, 0, 2] - a_true) / math.sqrt(c[0, 0, 5])
    assert 0.85 < zl.std() < 1.15 and 0.85 < zb.std() < 1.15 and abs(np.corrcoef(zl, zb)[0, 1] - 0.6) < 0.1
    assert np.all((cat["xyz"] >= 0) & (cat["xyz"] <= 600.0))
    u1 = (raw["xyz"] - o) / d[:, None]
    u2 = (cat["xyz"] - o) / np.linalg.norm(cat["xyz"] - o, axis=1)[:, None]
    assert np.allclose(u1, u2, atol=1e-12)


def test_degenerate_mixture_with_inferred_mean_is_the_gaussian_theta_ep():
    # the combined oracle (inferred disc + bump mean, mixture likelihood) with
    # degenerate mixtures must give the inferred-mean EP with the Gaussian
    # likelihood N(a; m_b, C_bb) (frozen linearisation in both)
    from oracle import meanfn
    w = Workload("t", n=7, box_pc=1200.0, n_stars=60, sweeps=2, star_law="uniform", d_max_pc=1200.0,
                 noise_law="const", noise_a=0.05, likelihood="gauss_linear", seed_id=6)
    cfg = dict(w.ep_fields(), relinearize=False, sun_radius_pc=8000.0, bump_width_pc=200.0,
               theta_prior=(1500.0, 150.0, 7.5e-4, 600.0, 0.1))
    raw = draw(w)
    S = w.n_stars
    o = np.asarray(cfg["observer_pc"])
    comps = np.zeros((S, 1, 6))
    comps[:, 0, 0] = 1.0
    comps[:, 0, 1] = np.log(np.linalg.norm(raw["xyz"] - o, axis=1))
    comps[:, 0, 2] = -1.0 + 0.3 * raw["eps"]
    comps[:, 0, 3] = 1e-300
    comps[:, 0, 5] = raw["sigma"] ** 2
    a = gmm.DenseEPThetaGMM(cfg, raw["xyz"], comps)
    b = meanfn.DenseEPTheta(cfg, raw["xyz"], comps[:, 0, 2], raw["sigma"])
    for _ in range(2):
        a.sweep()
        b.sweep()
        assert np.allclose(a.tau, b.tau, rtol=1e-12) and np.allclose(a.nu, b.nu, rtol=1e-12, atol=1e-12)
    assert np.allclose(a.theta_posterior()[0], b.theta_posterior()[0], rtol=1e-12)

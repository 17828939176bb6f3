"""Pins for the oracle's EP with an inferred parametric prior mean: the disc +
bump mean function, its Jacobian, the log-normal hyperprior, the joint
(delta, phi) EP against GP regression with explicit basis functions
(closed form in covariance form), the fixed-mean limit, and recovery of the
parameters on synthetic data."""
import math

import numpy as np
import pytest

from oracle import epo, meanfn
from synth import Workload, draw


def _cfg(n=6, L=4000.0, **kw):
    c = dict(n=n, box_pc=L, observer_pc=(L / 2, 0.0, L / 2), prior_mean=-7.0, prior_var=1.0,
             outer_scale_pc=100.0, support_pc=150.0, los_step_pc=2.0, sun_radius_pc=8000.0,
             bump_width_pc=400.0)
    c.update(kw)
    return c


def test_mean_function_at_worked_points():
    cfg = _cfg()
    theta = (3000.0, 150.0, 7.5e-4, 2000.0, 0.1)
    # at the observer: R = R0, h = 0, so the disc gives rk0; the bump is
    # 0.1 / (sqrt(2 pi) 400) * exp(-12.5)
    d, b = meanfn.components(cfg, np.array([[2000.0, 0.0, 2000.0]]), theta)
    assert abs(d[0] - 7.5e-4) < 1e-18
    assert abs(b[0] - 0.1 / (math.sqrt(2 * math.pi) * 400.0) * math.exp(-12.5)) < 1e-18
    # 2 kpc out along the line of sight, 300 pc above the plane: R = 10 kpc
    d, b = meanfn.components(cfg, np.array([[2000.0, 2000.0, 2300.0]]), theta)
    assert abs(d[0] - 7.5e-4 * math.exp(-2000.0 / 3000.0 - 2.0)) < 1e-18
    assert abs(b[0] - 0.1 / (math.sqrt(2 * math.pi) * 400.0) * math.exp(-2.0)) < 1e-18
    # 1.5 kpc sideways at y = y_o: R = sqrt(8000^2 + 1500^2)
    d, _ = meanfn.components(cfg, np.array([[3500.0, 0.0, 2000.0]]), theta)
    assert abs(d[0] - 7.5e-4 * math.exp(-(math.hypot(8000.0, 1500.0) - 8000.0) / 3000.0)) < 1e-18
    m, _ = meanfn.mean_and_jacobian(cfg, np.array([[2000.0, 2000.0, 2300.0]]), np.log(theta))
    assert abs(m[0] - math.log(7.5e-4 * math.exp(-2000.0 / 3000.0 - 2.0)
                               + 0.1 / (math.sqrt(2 * math.pi) * 400.0) * math.exp(-2.0))) < 1e-13


def test_jacobian_matches_central_differences():
    cfg = _cfg()
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 4000.0, (200, 3))
    phi = np.log([2500.0, 200.0, 1e-3, 1500.0, 0.3])
    _, J = meanfn.mean_and_jacobian(cfg, pos, phi)
    for j in range(5):
        e = np.zeros(5)
        e[j] = 1e-5
        mp, _ = meanfn.mean_and_jacobian(cfg, pos, phi + e)
        mm, _ = meanfn.mean_and_jacobian(cfg, pos, phi - e)
        fd = (mp - mm) / 2e-5
        assert np.allclose(J[:, j], fd, rtol=1e-6, atol=1e-8), j


def test_hyperprior_is_lognormal_with_mean_and_sd_equal():
    cfg = _cfg(theta_prior=(3000.0, 150.0, 7.5e-4, 2000.0, 0.1))
    mu0, s2 = meanfn.hyperprior(cfg)
    M = np.array(cfg["theta_prior"])
    assert np.allclose(np.exp(mu0 + s2 / 2), M, rtol=1e-14)               # log-normal mean
    assert np.allclose(np.sqrt(np.expm1(s2)) * np.exp(mu0 + s2 / 2), M, rtol=1e-14)   # its sd


def _small(n, L, stars, lik, seed=3):
    w = Workload("t", n=n, box_pc=L, n_stars=stars, sweeps=3, star_law="uniform", d_max_pc=L,
                 noise_law="const", noise_a=0.05, likelihood=lik, seed_id=seed)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=400.0)
    return cfg, draw(w)


def test_linear_mean_with_gaussian_likelihood_is_basis_function_regression():
    # f = Hb phi + delta, phi ~ N(mu0, B0), delta ~ N(0, K); y = c + G f + eps.
    # The joint EP is exact in one sweep and must equal GP regression with
    # the basis integrated out, in covariance form:
    #   C = K + Hb B0 Hb^T, Ky = G C G^T + R, r = y - c - G Hb mu0,
    #   E[f|y] = Hb mu0 + C G^T Ky^{-1} r,  E[phi|y] = mu0 + B0 Hb^T G^T Ky^{-1} r.
    cfg, raw = _small(6, 600.0, 80, "gauss_linear")
    vec = epo.Vecchia(cfg)
    pos = vec.grid.xyz()
    Hb = np.stack([np.ones(len(pos)), pos[:, 1] / 600.0, (pos[:, 2] - 300.0) / 600.0], axis=1)
    mu0, B0 = np.array([-6.5, 0.4, -0.3]), np.array([0.5, 0.2, 0.3])
    sl = epo.Sightlines(cfg, raw["xyz"])
    y = -0.5 + 0.3 * np.random.default_rng(1).standard_normal(len(raw["xyz"]))
    ep = meanfn.DenseEPTheta(cfg, raw["xyz"], y, raw["sigma"], sightlines=sl, vecchia=vec,
                             mean=lambda phi: (Hb @ phi, Hb), prior=(mu0, B0))
    ep.sweep()
    gval, _, c = sl.linearise(Hb @ mu0)
    G = sl.G_dense(gval)
    K = np.linalg.inv(vec.Q0_dense())
    C = K + Hb @ np.diag(B0) @ Hb.T
    Ky = G @ C @ G.T + np.diag(raw["sigma"] ** 2)
    r = y - c - G @ Hb @ mu0
    f_mean = Hb @ mu0 + C @ G.T @ np.linalg.solve(Ky, r)
    f_cov = C - C @ G.T @ np.linalg.solve(Ky, G @ C)
    phi_mean = mu0 + np.diag(B0) @ Hb.T @ G.T @ np.linalg.solve(Ky, r)
    phi_cov = np.diag(B0) - np.diag(B0) @ Hb.T @ G.T @ np.linalg.solve(Ky, G @ Hb @ np.diag(B0))
    assert np.allclose(ep.posterior_mean(), f_mean, rtol=1e-9, atol=1e-9)
    assert np.allclose(ep.marginal_var(), np.diag(f_cov), rtol=1e-8, atol=1e-12)
    pm, pc = ep.theta_posterior()
    assert np.allclose(pm, phi_mean, rtol=1e-9, atol=1e-10)
    assert np.allclose(pc, phi_cov, rtol=1e-8, atol=1e-12)


def test_vanishing_hyperprior_variance_gives_the_fixed_mean_ep():
    # one constant basis function with prior N(-7, s2): as s2 -> 0 the joint
    # EP must follow the fixed-mean EP with prior_mean -7 (extinction
    # likelihood, relinearised), with differences of order s2 (below ~1e-8
    # the augmented precision's conditioning takes over)
    cfg, raw = _small(6, 500.0, 60, "extinction")
    f_true, A, sl = epo.simulate(cfg, raw)
    N = cfg["n"] ** 3
    one = np.ones((N, 1))
    worst = {}
    for s2 in (1e-6, 1e-8):
        a = meanfn.DenseEPTheta(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl,
                                mean=lambda phi: (one[:, 0] * phi[0], one), prior=(np.array([-7.0]), np.array([s2])))
        b = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
        worst[s2] = 0.0
        for _ in range(3):
            a.sweep()
            b.sweep()
            worst[s2] = max(worst[s2], float(np.max(np.abs(a.tau - b.tau) / np.abs(b.tau))),
                            float(np.max(np.abs(a.nu - b.nu) / np.maximum(np.abs(b.nu), 1e-3))))
        if s2 == 1e-8:
            assert np.allclose(a.posterior_mean(), b.posterior_mean(), rtol=1e-7)
            assert np.allclose(a.marginal_var(), b.marginal_var(), rtol=1e-6)
    print("worst site differences", worst)
    assert worst[1e-8] < 5e-7
    assert 30 < worst[1e-6] / worst[1e-8] < 300


def test_partial_linearisation_step_keeps_the_fixed_point():
    """With the inferred mean and the extinction likelihood, moving the
    linearisation point (deltahat and phihat) only part of the way to the
    posterior means each sweep changes the path, not the EP fixed point."""
    cfg, raw = _small(6, 500.0, 60, "extinction")
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=200.0, theta_prior=meanfn.DEFAULT_PRIOR, damping=0.5)
    f_true, A, sl = meanfn.simulate(cfg, raw, np.array([2500.0, 200.0, 1.2e-3, 300.0, 0.1]))
    out = {}
    for r in (1.0, 0.5):
        ep = meanfn.DenseEPTheta(dict(cfg, relin_step=r), raw["xyz"], A, raw["sigma"], sightlines=sl)
        for it in range(400):
            f0, t0 = ep.fhat.copy(), ep.tau.copy()
            ep.sweep()
            if np.max(np.abs(ep.fhat - f0)) < 1e-11 and np.max(np.abs(ep.tau - t0)) < 1e-10:
                break
        assert it < 399, r
        m, _ = ep.mean(ep.phihat)
        mu = ep.posterior_mean()
        # at the fixed point the linearisation point is the posterior mean
        assert np.max(np.abs(mu - ep.fhat)) < 1e-9
        out[r] = (ep.fhat, ep.phihat, ep.tau, it)
    print("sweeps to converge: r = 1:", out[1.0][3], " r = 0.5:", out[0.5][3])
    assert np.allclose(out[1.0][0], out[0.5][0], rtol=0, atol=1e-8)
    assert np.allclose(out[1.0][1], out[0.5][1], rtol=0, atol=1e-8)
    assert np.allclose(out[1.0][2], out[0.5][2], rtol=1e-7, atol=1e-8)


def test_recovers_the_density_scale_on_synthetic_data():
    w = Workload("t", n=10, box_pc=4000.0, n_stars=500, sweeps=4, star_law="disc", d_max_pc=4000.0,
                 noise_law="const", noise_a=0.05, likelihood="extinction", seed_id=11)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=400.0, theta_prior=meanfn.DEFAULT_PRIOR)
    raw = draw(w)
    theta_true = np.array([2500.0, 200.0, 1.2e-3, 1800.0, 0.15])
    f_true, A, sl = meanfn.simulate(cfg, raw, theta_true)
    ep = meanfn.DenseEPTheta(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    mu0, s2 = meanfn.hyperprior(cfg)
    for _ in range(6):
        ep.sweep()
    pm, pc = ep.theta_posterior()
    sd = np.sqrt(np.diag(pc))
    z = (pm - np.log(theta_true)) / sd
    print("phi posterior", pm, "sd", sd, "z", z)
    assert np.all(np.abs(z) < 4)
    # the overall density scale is learned: its posterior is much narrower
    # than the hyperprior and moved from the prior mean towards the truth
    assert sd[2] < 0.3 * math.sqrt(s2[2])
    assert abs(pm[2] - math.log(theta_true[2])) < abs(mu0[2] - math.log(theta_true[2]))


@pytest.mark.parametrize("seed", [0, 1])
def test_theta_posterior_against_the_exact_posterior(seed):
    """Gaussian mode: the exact posterior of phi (importance sampling with the
    exact GP marginal) against the EP posterior with the mean linearised at
    the hyperprior mean only (the mean frozen with the sightlines) and with
    the mean re-linearised at phihat every sweep (damped).  The frozen form is
    overconfident (the disc's scale height comes out 2-3 times too narrow);
    re-linearising the mean brings the sds of the disc parameters and the
    bump's amplitude within 0.75-1.3 of the exact ones and every mean within
    0.75 exact sd.  The bump's distance keeps a skewed posterior that a
    Gaussian cannot match: its sd stays narrow (about 0.4-0.45 of the exact
    one) either way."""
    w = Workload("t", n=10, box_pc=4000.0, n_stars=500, sweeps=4, star_law="disc", d_max_pc=4000.0,
                 noise_law="const", noise_a=0.05, likelihood="gauss_linear", seed_id=seed)
    cfg = dict(w.ep_fields(), sun_radius_pc=8000.0, bump_width_pc=400.0, theta_prior=meanfn.DEFAULT_PRIOR)
    raw = draw(w)
    vec = epo.Vecchia(cfg)
    sl = epo.Sightlines(cfg, raw["xyz"])
    pos = vec.grid.xyz()
    theta_true = np.array([2500.0, 200.0, 1.2e-3, 1800.0, 0.15])
    mu0, _ = meanfn.hyperprior(cfg)
    m_true, _ = meanfn.mean_and_jacobian(cfg, pos, np.log(theta_true))
    f_true = m_true + vec.draw(0.0, raw["xi"])
    gval, _, c = sl.linearise(meanfn.mean_and_jacobian(cfg, pos, mu0)[0])
    a_obs = c + sl.G_dense(gval) @ f_true + raw["sigma"] * raw["eps"]
    out = {}
    for tag, relin in (("frozen", False), ("relinearised", True)):
        ep = meanfn.DenseEPTheta(dict(cfg, relinearize=relin, damping=0.5), raw["xyz"], a_obs, raw["sigma"],
                                 sightlines=sl, vecchia=vec)
        for _ in range(40):
            old = ep.phihat.copy()
            ep.sweep()
        if relin:
            assert np.max(np.abs(ep.phihat - old)) < 1e-6     # the damped linearisation point has settled
        out[tag] = ep.theta_posterior()
    em, ec, ess = meanfn.exact_theta_posterior_gaussian(cfg, sl, vec, a_obs, raw["sigma"], out["relinearised"][0],
                                                         4 * out["relinearised"][1], n_samples=20000, seed=seed)
    sd = np.sqrt(np.diag(ec))
    ratio = {k: np.sqrt(np.diag(v[1])) / sd for k, v in out.items()}
    shift = {k: np.abs(v[0] - em) / sd for k, v in out.items()}
    print(f"seed {seed}: ess {ess:.0f}; sd ratio frozen {np.round(ratio['frozen'], 2)}, relinearised "
          f"{np.round(ratio['relinearised'], 2)}; |mean shift| in exact sd frozen {np.round(shift['frozen'], 2)}, "
          f"relinearised {np.round(shift['relinearised'], 2)}")
    assert ess > 1500
    assert ratio["frozen"][1] < 0.5
    keep = np.array([0, 1, 2, 4])      # the bump's distance (3) keeps a skewed posterior: checked apart
    assert np.all(ratio["relinearised"][keep] > 0.75) and np.all(ratio["relinearised"][keep] < 1.3)
    assert 0.3 < ratio["relinearised"][3] < 1.3
    assert np.all(shift["relinearised"] < 0.75)

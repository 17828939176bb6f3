"""Pins for the oracle's parallel EP (Sec. 4.1 steps; App. A.2 parallel
procedure and moment matching)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import epo
from synth import Workload, draw


def _small(n=8, L=500.0, stars=60, lik="extinction", **kw):
    w = Workload("tiny", n=n, box_pc=L, n_stars=stars, sweeps=3, star_law="uniform",
                 noise_law="const", noise_a=0.05, likelihood=lik, seed_id=90)
    cfg = w.ep_fields()
    cfg.update(kw)
    return w, cfg


def test_gaussian_likelihood_exact_in_one_sweep():
    """Gaussian likelihood: one undamped sweep from zero sites gives the exact
    GP regression posterior (Sec. 2, conditioning on noisy observations)."""
    w, cfg = _small(lik="gauss_linear")
    raw = draw(w)
    f_true, a_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], a_obs, raw["sigma"], sightlines=sl)
    ep.sweep()
    # sites equal the likelihood exactly
    assert np.allclose(ep.tau, 1.0 / raw["sigma"] ** 2, rtol=1e-9)
    assert np.allclose(ep.nu, a_obs / raw["sigma"] ** 2, rtol=1e-8, atol=1e-8)
    # posterior = m + K H^T (H K H^T + S)^{-1} (y - c - H m), K = Q0^{-1}
    gval, _, c = sl.linearise(np.full(sl.grid.N, cfg["prior_mean"]))
    H = sl.G_dense(gval)
    K = np.linalg.inv(ep.Q0)
    m = np.full(sl.grid.N, cfg["prior_mean"])
    S = np.diag(raw["sigma"] ** 2)
    M = H @ K @ H.T + S
    mu = m + K @ H.T @ np.linalg.solve(M, a_obs - c - H @ m)
    Sig = K - K @ H.T @ np.linalg.solve(M, H @ K)
    assert np.allclose(ep.posterior_mean(), mu, rtol=1e-10, atol=1e-10)
    assert np.allclose(ep.marginal_var(), np.diag(Sig), rtol=1e-9, atol=1e-12)
    # a second sweep is a fixed point
    tau, nu = ep.tau.copy(), ep.nu.copy()
    ep.sweep()
    assert np.allclose(ep.tau, tau, rtol=1e-8) and np.allclose(ep.nu, nu, rtol=1e-7, atol=1e-7)


def test_one_star_frozen_projection_is_exact():
    """One star, projection frozen at the prior mean: after one sweep EP holds
    the exact posterior of f, by brute-force 1-D quadrature over s = g.f."""
    w, cfg = _small(stars=1, relinearize=False)
    raw = draw(w)
    raw["xyz"] = np.array([[300.0, 420.0, 180.0]])
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, raw["sigma"], sightlines=sl)
    ep.sweep()
    mu_ep, Sig_ep, G, c = ep.posterior()
    g = G[0]
    K = np.linalg.inv(ep.Q0)
    m = np.full(sl.grid.N, cfg["prior_mean"])
    ms = c[0] + g @ m
    vs = g @ K @ g
    A, s = A_obs[0], raw["sigma"][0]
    dens = lambda a: math.exp(-(a - ms) ** 2 / (2 * vs) - (A - math.exp(a)) ** 2 / (2 * s * s))
    lo, hi = ms - 12 * math.sqrt(vs), ms + 12 * math.sqrt(vs)
    Z = integrate.quad(dens, lo, hi, epsrel=1e-13, limit=500, points=[math.log(max(A, 1e-3))])[0]
    Es = integrate.quad(lambda a: a * dens(a), lo, hi, epsrel=1e-13, limit=500,
                        points=[math.log(max(A, 1e-3))])[0] / Z
    Vs = integrate.quad(lambda a: (a - Es) ** 2 * dens(a), lo, hi, epsrel=1e-12, limit=500,
                        points=[math.log(max(A, 1e-3))])[0] / Z
    Kg = K @ g
    mu_exact = m + Kg * (Es - ms) / vs
    Sig_exact = K - np.outer(Kg, Kg) * (vs - Vs) / vs ** 2
    assert np.allclose(mu_ep, mu_exact, rtol=1e-9, atol=1e-9)
    assert np.allclose(np.diag(Sig_ep), np.diag(Sig_exact), rtol=1e-9, atol=1e-12)


def test_moment_matching_invariant_at_convergence():
    """At an EP fixed point the q-marginal of every a_n equals the moments of
    its tilted distribution (App. A, moment matching)."""
    w, cfg = _small(stars=25, relinearize=False, damping=0.5)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, raw["sigma"], sightlines=sl)
    for _ in range(80):
        st = ep.sweep()
    assert st["max_dtau"] < 1e-9
    mu, Sig, G, c = ep.posterior()
    qm = c + G @ mu
    qv = np.einsum("ij,ij->i", G @ Sig, G)
    # tilted moments from the same q
    tau_c = 1 / qv - ep.tau
    nu_c = qm / qv - ep.nu
    _, mh, vh = epo.tilted(0, nu_c / tau_c, 1 / tau_c, A_obs, raw["sigma"])
    assert np.allclose(qm, mh, rtol=1e-8, atol=1e-8)
    assert np.allclose(qv, vh, rtol=1e-8)


def test_calibration_of_posterior_on_true_field():
    """z-scores of the true field under the EP posterior are roughly standard
    normal where the data constrain it (cf. the residual histograms of Sec. 5)."""
    w, cfg = _small(n=10, L=660.0, stars=400)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, raw["sigma"], sightlines=sl)
    for _ in range(6):
        ep.sweep()
    mu = ep.posterior_mean()
    var = ep.marginal_var()
    z = (f_true - mu) / np.sqrt(var)
    assert abs(np.mean(z)) < 0.3
    assert 0.6 < np.std(z) < 1.4
    assert np.all(var <= cfg["prior_var"] * 1.0001)   # data only shrink variance


def test_site_update_algebra():
    """Replacing a site by (tilted / cavity) gives back the tilted moments as the
    new marginal when the projection is a single coordinate."""
    tau_c, nu_c = 2.0, -1.2
    _, mh, vh = epo.tilted(0, [nu_c / tau_c], [1 / tau_c], [0.4], [0.05])
    tau_new = 1 / vh[0] - tau_c
    nu_new = mh[0] / vh[0] - nu_c
    assert 1 / (tau_c + tau_new) == pytest.approx(vh[0], rel=1e-14)
    assert (nu_c + nu_new) / (tau_c + tau_new) == pytest.approx(mh[0], rel=1e-13)


def _tilted_quad(mu_c, v_c, A, s):
    """Moments of N(a; mu_c, v_c) N(A; e^a, s^2) by plain adaptive quadrature
    (scipy), independent of the oracle's Gauss-Kronrod code."""
    dens = lambda a: math.exp(-(a - mu_c) ** 2 / (2 * v_c) - (A - math.exp(a)) ** 2 / (2 * s * s))
    sd = math.sqrt(v_c)
    lo, hi = mu_c - 14 * sd, mu_c + 14 * sd
    pts = [x for x in (mu_c, math.log(max(A, 1e-3))) if lo < x < hi]
    q = lambda f: integrate.quad(f, lo, hi, epsabs=0.0, epsrel=1e-13, limit=800, points=pts)[0]
    Z = q(dens)
    m = q(lambda a: a * dens(a)) / Z
    v = q(lambda a: (a - m) ** 2 * dens(a)) / Z
    return m, v


def test_multi_star_iterates_match_reduced_ep():
    """Several interacting stars, non-Gaussian likelihood, projection frozen at
    the prior mean: every site touches f only through a = c + G f, so parallel
    EP over f (Sec. 4.1, App. A.2) is parallel EP over the S-dimensional
    Gaussian prior of a, N(c + G m, G K G^T).  The sweeps are run in that
    reduced space with dense S x S algebra and scipy quadrature for the tilted
    moments, and every sweep's sites, cavities and q-marginals of a must agree
    with the oracle's, which assembles Q and b over the grid."""
    w, cfg = _small(stars=12, relinearize=False, damping=0.7)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    sig = raw["sigma"]
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, sig, sightlines=sl)
    gval, _, c = sl.linearise(np.full(sl.grid.N, cfg["prior_mean"]))
    H = sl.G_dense(gval)
    K = np.linalg.inv(ep.Q0)
    S = H @ K @ H.T
    ma = c + H @ np.full(sl.grid.N, cfg["prior_mean"])
    n = len(ma)
    t, nv = np.zeros(n), np.zeros(n)
    d = cfg["damping"]
    for sweep in range(8):
        # q(a): precision S^-1 + T, in the form that needs no S^-1
        r = np.sqrt(t)
        B = np.eye(n) + r[:, None] * S * r[None, :]
        Sa = S - (S * r[None, :]) @ np.linalg.solve(B, r[:, None] * S)
        mua = ma + Sa @ (nv - t * ma)
        va = np.diag(Sa)
        tc = 1.0 / va - t
        nc = mua / va - nv
        assert np.all(tc > 0)
        mh, vh = np.array([_tilted_quad(nc[i] / tc[i], 1.0 / tc[i], A_obs[i], sig[i]) for i in range(n)]).T
        t_new = 1.0 / vh - tc
        n_new = mh / vh - nc
        assert np.all(t_new >= 0)
        st = ep.sweep()
        assert np.allclose(st["cav_mu"], nc / tc, rtol=1e-10, atol=1e-10), sweep
        assert np.allclose(st["cav_var"], 1.0 / tc, rtol=1e-10), sweep
        t = (1 - d) * t + d * t_new
        nv = (1 - d) * nv + d * n_new
        assert np.allclose(ep.tau, t, rtol=1e-9, atol=1e-12), sweep
        assert np.allclose(ep.nu, nv, rtol=1e-9, atol=1e-10), sweep
    # the q-marginals of a after the last sweep
    mu, Sig, G, cc = ep.posterior()
    r = np.sqrt(t)
    B = np.eye(n) + r[:, None] * S * r[None, :]
    Sa = S - (S * r[None, :]) @ np.linalg.solve(B, r[:, None] * S)
    mua = ma + Sa @ (nv - t * ma)
    assert np.allclose(cc + G @ mu, mua, rtol=1e-10, atol=1e-10)
    assert np.allclose(G @ Sig @ G.T, Sa, rtol=1e-8, atol=1e-12)
    # the stars interact: the reduced prior is far from diagonal
    off = S - np.diag(np.diag(S))
    assert np.max(np.abs(off)) > 0.05 * np.max(np.diag(S))


def _lnA_plain(cfg, xyz, f):
    """ln A_n and its gradient by a plain numpy forward model written here:
    T = max(1, ceil(d / step)) equal steps from the observer, trapezoid
    weights, trilinear interpolation with cell clamp(floor(s / h), 0, n - 2)."""
    n, L = int(cfg["n"]), float(cfg["box_pc"])
    h = L / (n - 1)
    o = np.asarray(cfg["observer_pc"], dtype=np.float64)
    lnA = np.zeros(len(xyz))
    grad = np.zeros((len(xyz), n ** 3))
    for s, x in enumerate(xyz):
        d = float(np.linalg.norm(x - o))
        T = max(1, math.ceil(d / cfg["los_step_pc"]))
        t = np.arange(T + 1)
        w = np.full(T + 1, d / T)
        w[0] *= 0.5
        w[-1] *= 0.5
        pts = o[None, :] + (t[:, None] / T) * (x - o)[None, :]
        u = pts / h
        cell = np.clip(np.floor(u), 0, n - 2).astype(int)
        fr = u - cell
        F = np.zeros(T + 1)
        corners = []
        for di in (0, 1):
            for dj in (0, 1):
                for dk in (0, 1):
                    wt = ((fr[:, 0] if di else 1 - fr[:, 0]) * (fr[:, 1] if dj else 1 - fr[:, 1])
                          * (fr[:, 2] if dk else 1 - fr[:, 2]))
                    node = (cell[:, 0] + di) + n * ((cell[:, 1] + dj) + n * (cell[:, 2] + dk))
                    F += wt * f[node]
                    corners.append((node, wt))
        e = w * np.exp(F)
        A = e.sum()
        lnA[s] = math.log(A)
        for node, wt in corners:
            np.add.at(grad[s], node, e * wt / A)
    return lnA, grad


@pytest.mark.parametrize("relin_step", [1.0, 0.5])
def test_relinearised_fixed_point(relin_step):
    """With the sightlines re-linearised at the posterior mean every sweep
    (the linearisation of the log-extinction likelihood in a_n about the
    current field), iterate damped EP to its fixed point and check what the
    fixed point must satisfy:
      * the linearisation point equals the posterior mean it produces;
      * posterior() linearises at the current point: Q and b rebuilt from a
        plain numpy forward model and its gradient at fhat give the same mean
        and covariance;
      * the moment-matching invariant (App. A.2) holds at that point;
      * the fixed point is not the frozen-projection one (so a stale
        linearisation would fail the checks above)."""
    w, cfg = _small(n=7, L=420.0, stars=30, relinearize=True, damping=0.5)
    cfg = dict(cfg, relin_step=relin_step)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    sig = raw["sigma"]
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, sig, sightlines=sl)
    assert ep.relin
    m0b = ep.Q0 @ np.full(sl.grid.N, cfg["prior_mean"])
    # the iterates: each sweep moves the point to the mean of the posterior
    # built, with the sites it started from, at the point it started from
    # (the fraction relin_step of the way there)
    for _ in range(3):
        f0 = ep.fhat.copy()
        lnA, Gp = _lnA_plain(cfg, raw["xyz"], f0)
        Q = ep.Q0 + Gp.T @ (ep.tau[:, None] * Gp)
        mu_next = np.linalg.solve(Q, m0b + Gp.T @ (ep.nu - ep.tau * (lnA - Gp @ f0)))
        ep.sweep()
        assert np.allclose(ep.fhat, f0 + relin_step * (mu_next - f0), rtol=1e-11, atol=1e-11)
    for it in range(400):
        st = ep.sweep()
        if st["max_dtau"] < 1e-10 and st["max_dmu"] < 1e-10:
            break
    assert st["max_dtau"] < 1e-10 and st["max_dmu"] < 1e-10, (it, st["max_dtau"], st["max_dmu"])
    mu, Sig, G, c = ep.posterior()
    # (1) fhat = mu
    assert np.max(np.abs(mu - ep.fhat)) < 1e-10
    # (2) brute-force re-linearisation at the current fhat
    lnA, Gp = _lnA_plain(cfg, raw["xyz"], ep.fhat)
    cp = lnA - Gp @ ep.fhat
    assert np.allclose(G, Gp, rtol=0, atol=1e-12)
    Q = ep.Q0 + Gp.T @ (ep.tau[:, None] * Gp)
    b = ep.Q0 @ np.full(sl.grid.N, cfg["prior_mean"]) + Gp.T @ (ep.nu - ep.tau * cp)
    Sig_p = np.linalg.inv(Q)
    assert np.allclose(mu, np.linalg.solve(Q, b), rtol=1e-11, atol=1e-11)
    assert np.allclose(Sig, Sig_p, rtol=1e-10, atol=1e-13)
    # (3) moment matching at the fixed point
    qm = cp + Gp @ mu
    qv = np.einsum("ij,jk,ik->i", Gp, Sig_p, Gp)
    tau_c = 1 / qv - ep.tau
    nu_c = qm / qv - ep.nu
    assert np.all(tau_c > 0)
    _, mh, vh = epo.tilted(0, nu_c / tau_c, 1 / tau_c, A_obs, sig)
    assert np.allclose(qm, mh, rtol=1e-8, atol=1e-8)
    assert np.allclose(qv, vh, rtol=1e-8)
    # (4) the frozen projection converges elsewhere
    fz = epo.DenseEP(dict(cfg, relinearize=False), raw["xyz"], A_obs, sig, sightlines=sl)
    for _ in range(200):
        if fz.sweep()["max_dtau"] < 1e-10:
            break
    assert np.max(np.abs(fz.posterior_mean() - mu)) > 1e-3
    # (5) a partial linearisation step changes the path, not the fixed point
    if relin_step != 1.0:
        full = epo.DenseEP(dict(cfg, relin_step=1.0), raw["xyz"], A_obs, sig, sightlines=sl)
        for _ in range(400):
            st1 = full.sweep()
            if st1["max_dtau"] < 1e-10 and st1["max_dmu"] < 1e-10:
                break
        assert np.allclose(full.fhat, ep.fhat, rtol=0, atol=1e-8)
        assert np.allclose(full.tau, ep.tau, rtol=1e-8, atol=1e-8)


def test_posterior_uses_current_linearisation_point():
    """posterior() after a manual move of the linearisation point: its mean
    and covariance are those of Q and b rebuilt at the new point from the
    plain forward model (so no stale linearisation can be cached)."""
    w, cfg = _small(n=6, L=400.0, stars=15, relinearize=True)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, raw["sigma"], sightlines=sl)
    ep.sweep()
    ep.sweep()
    rng = np.random.default_rng(3)
    ep.fhat = ep.fhat + 0.3 * rng.standard_normal(sl.grid.N)
    mu, Sig, G, c = ep.posterior()
    lnA, Gp = _lnA_plain(cfg, raw["xyz"], ep.fhat)
    cp = lnA - Gp @ ep.fhat
    Q = ep.Q0 + Gp.T @ (ep.tau[:, None] * Gp)
    b = ep.Q0 @ np.full(sl.grid.N, cfg["prior_mean"]) + Gp.T @ (ep.nu - ep.tau * cp)
    assert np.allclose(mu, np.linalg.solve(Q, b), rtol=1e-11, atol=1e-11)
    assert np.allclose(Sig, np.linalg.inv(Q), rtol=1e-10, atol=1e-13)

"""Pins of the PITC / PIC block-EP oracle against what the mathematics fixes.

The oracle follows App. B in covariance form (conditionals through
(Sigma_k + S_k)^{-1}); every reference below is computed another way: the
information form K^{-1} + G^T S^{-1} G of the exact Gaussian posterior, the
determinant lemma, and the Snelson-Ghahramani closed form of the PITC
posterior (Woodbury in the other direction)."""
import math

import numpy as np
import pytest

from oracle import epo, pitc
from synth import Workload, draw
from synth.workloads import node_positions, sky_cells


def _case(n=6, L=500.0, stars=60, n_lon=3, n_lat=1, R=12, seed=5, law="uniform"):
    w = Workload("pitc", n=n, box_pc=L, n_stars=stars, sweeps=1, star_law=law, d_max_pc=L,
                 noise_law="uniform", noise_a=0.05, noise_b=0.15, likelihood="gauss_linear", seed_id=seed)
    cfg = w.ep_fields()
    raw = draw(w)
    f_true, a_obs, sl = epo.simulate(cfg, raw)
    blocks = sky_cells(w, raw["xyz"], n_lon, n_lat)
    node_block = sky_cells(w, node_positions(w), n_lon, n_lat)
    rng = np.random.default_rng(seed)
    u = np.sort(rng.choice(w.N, size=R, replace=False)) if R < w.N else np.arange(w.N)
    return w, cfg, raw, a_obs, sl, blocks, node_block, u


def _exact(o):
    """Exact GP posterior of f from all stars, information form."""
    S = o.s2
    Kinv = np.linalg.inv(o.K)
    P = Kinv + o.G.T @ (o.G / S[:, None])
    V = np.linalg.inv(P)
    m = np.full(o.grid.N, o.m0)
    mean = m + V @ (o.G.T @ ((o.a_obs - o.mu_a) / S))
    return mean, 0.5 * (V + V.T), P, Kinv


def _exact_lnZ(o, P):
    """ln N(a~; mu, G K G^T + S) by the determinant lemma and Woodbury."""
    S = o.s2
    r = o.a_obs - o.mu_a
    _, ldP = np.linalg.slogdet(P)
    _, ldK = np.linalg.slogdet(o.K)
    logdet = ldP + ldK + np.log(S).sum()
    t = o.G.T @ (r / S)
    quad = r @ (r / S) - t @ np.linalg.solve(P, t)
    return -0.5 * (len(r) * math.log(2 * math.pi) + logdet + quad)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def test_u_given_block_matches_information_form():
    w, cfg, raw, a, sl, blocks, nb, u = _case(R=15)
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    Kinv = np.linalg.inv(o.K)
    for k in range(o.nblk):
        idx = o.members[k]
        Gk = o.G[idx]
        P = Kinv + Gk.T @ (Gk / o.s2[idx][:, None])
        V = np.linalg.inv(P)
        mean = o.m0 + V @ (Gk.T @ ((a[idx] - o.mu_a[idx]) / o.s2[idx]))
        m1, C1 = o.u_given_block(k)
        assert _rel(m1, mean[u]) < 1e-9
        assert _rel(C1, V[np.ix_(u, u)]) < 1e-9
        # the conditional covariance shrinks: C - C'_k is positive semi-definite
        assert np.linalg.eigvalsh(o.C - C1).min() > -1e-12


def test_one_block_is_the_exact_gp():
    w, cfg, raw, a, sl, blocks, nb, u = _case(n_lon=1, R=10)
    assert blocks.max() == 0
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    mean, V, P, _ = _exact(o)
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, mean[u]) < 1e-9 and _rel(V_u, V[np.ix_(u, u)]) < 1e-9
    pm, pv = o.predict()
    assert _rel(pm, mean) < 1e-9 and _rel(pv, np.diag(V)) < 1e-8
    assert abs(o.log_evidence() - _exact_lnZ(o, P)) < 1e-8 * abs(_exact_lnZ(o, P))


def test_every_node_inducing_is_exact_for_any_blocking():
    w, cfg, raw, a, sl, blocks, nb, u = _case(n=5, stars=50, n_lon=4, n_lat=2, R=125)
    assert blocks.max() >= 3 and len(u) == w.N
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    mean, V, P, _ = _exact(o)
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, mean) < 1e-8 and _rel(V_u, V) < 1e-7
    pm, pv = o.predict()
    assert _rel(pm, mean) < 1e-8 and _rel(pv, np.diag(V)) < 1e-6
    assert abs(o.log_evidence() - _exact_lnZ(o, P)) < 1e-8 * abs(_exact_lnZ(o, P))


def test_sweep_gives_the_pitc_closed_form():
    """Snelson & Ghahramani: Sigma_u = C (C + rho^T Lam^{-1} rho)^{-1} C,
    mu_u = m + C (C + rho^T Lam^{-1} rho)^{-1} rho^T Lam^{-1} r with
    Lam = blockdiag(Sigma_k + S_k - rho_k C^{-1} rho_k^T)."""
    w, cfg, raw, a, sl, blocks, nb, u = _case(stars=80, n_lon=3, n_lat=2, R=20, seed=8)
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    S = len(a)
    rho = o.G @ o.K[:, u]
    Lam = np.zeros((S, S))
    for k in range(o.nblk):
        idx = o.members[k]
        Gk = o.G[idx]
        Lam[np.ix_(idx, idx)] = (Gk @ o.K @ Gk.T + np.diag(o.s2[idx])
                                 - rho[idx] @ np.linalg.solve(o.C, rho[idx].T))
    M = o.C + rho.T @ np.linalg.solve(Lam, rho)
    r = a - o.mu_a
    V_ref = o.C @ np.linalg.solve(M, o.C)
    m_ref = o.m_u + o.C @ np.linalg.solve(M, rho.T @ np.linalg.solve(Lam, r))
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, m_ref) < 1e-9 and _rel(V_u, V_ref) < 1e-8
    # evidence: |Lam + rho C^-1 rho^T| = |Lam| |M| / |C|, quadratic form by Woodbury
    _, l1 = np.linalg.slogdet(Lam)
    _, l2 = np.linalg.slogdet(M)
    _, l3 = np.linalg.slogdet(o.C)
    t = rho.T @ np.linalg.solve(Lam, r)
    quad = r @ np.linalg.solve(Lam, r) - t @ np.linalg.solve(M, t)
    ref = -0.5 * (S * math.log(2 * math.pi) + l1 + l2 - l3 + quad)
    assert abs(o.log_evidence() - ref) < 1e-9 * abs(ref)


def test_damped_sweeps_and_the_fixed_point():
    w, cfg, raw, a, sl, blocks, nb, u = _case(stars=50, n_lon=2, n_lat=2, R=10, seed=9)
    full = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    full.sweep(1.0)
    L1, e1 = full.Lam.copy(), full.eta.copy()
    full.sweep(1.0)                                    # already at the fixed point
    assert _rel(full.Lam, L1) < 1e-12 and _rel(full.eta, e1) < 1e-11
    half = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl, K=full.K)
    for t in range(1, 4):
        half.sweep(0.5)
        c = 1.0 - 0.5 ** t
        assert _rel(half.Lam, c * L1) < 1e-10 and _rel(half.eta, c * e1) < 1e-10


def test_no_inducing_points_is_the_local_gp():
    """R = 0: blocks independent (the local-GP special case, Sec. 4.1)."""
    w, cfg, raw, a, sl, blocks, nb, u = _case(stars=60, n_lon=3, n_lat=1, R=0, seed=4)
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u[:0], nb, sightlines=sl)
    o.sweep()
    Kinv = np.linalg.inv(o.K)
    pm, pv = o.predict()
    ref = 0.0
    for k in range(o.nblk):
        idx = o.members[k]
        Gk = o.G[idx]
        P = Kinv + Gk.T @ (Gk / o.s2[idx][:, None])
        V = np.linalg.inv(P)
        mean = o.m0 + V @ (Gk.T @ ((a[idx] - o.mu_a[idx]) / o.s2[idx]))
        nodes = nb == k
        assert _rel(pm[nodes], mean[nodes]) < 1e-9 and _rel(pv[nodes], np.diag(V)[nodes]) < 1e-8
        A = Gk @ o.K @ Gk.T + np.diag(o.s2[idx])
        r = a[idx] - o.mu_a[idx]
        ref += -0.5 * (len(idx) * math.log(2 * math.pi) + np.linalg.slogdet(A)[1] + r @ np.linalg.solve(A, r))
    assert abs(o.log_evidence() - ref) < 1e-9 * abs(ref)


def test_paper_sign_of_the_conditional_covariance_fails():
    """The printed '+' in C'_k would give a covariance larger than the prior's,
    contradicting the information-form conditional pinned above."""
    w, cfg, raw, a, sl, blocks, nb, u = _case(R=8)
    o = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    mu, A, rho = o.block_joint(0)
    plus = o.C + rho.T @ np.linalg.solve(A, rho)
    _, C1 = o.u_given_block(0)
    assert np.trace(plus) > np.trace(o.C) > np.trace(C1)


# --- the mean parameters in the sites (q(u, Theta)) --------------------------

THETA_PRIOR = (1500.0, 150.0, 7.5e-4, 600.0, 0.1)
THETA_TRUE = (1000.0, 200.0, 1.2e-3, 500.0, 0.2)


def _case_theta(n=5, L=400.0, stars=50, n_lon=2, n_lat=2, R=10, seed=6):
    from oracle import meanfn
    w = Workload("pitct", n=n, box_pc=L, n_stars=stars, sweeps=1, star_law="uniform", d_max_pc=L,
                 noise_law="uniform", noise_a=0.05, noise_b=0.15, likelihood="gauss_linear", seed_id=seed)
    cfg = w.ep_fields()
    # Vecchia conditioning over the whole box: Q0 = K^{-1} exactly (the
    # reference below uses the precision form)
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=200.0, theta_prior=THETA_PRIOR,
               vecchia_radius_pc=2.0 * L)
    raw = draw(w)
    sl = epo.Sightlines(cfg, raw["xyz"])
    vec = epo.Vecchia(cfg)
    pos = vec.grid.xyz()
    m_true, _ = meanfn.mean_and_jacobian(cfg, pos, np.log(THETA_TRUE))
    f_true = m_true + vec.draw(0.0, raw["xi"])
    mu0, _ = meanfn.hyperprior(cfg)
    mhat, _ = meanfn.mean_and_jacobian(cfg, pos, mu0)
    gval, _, c = sl.linearise(mhat)
    a = c + sl.G_dense(gval) @ f_true + raw["sigma"] * raw["eps"]
    blocks = sky_cells(w, raw["xyz"], n_lon, n_lat)
    _, blocks = np.unique(blocks, return_inverse=True)
    nb = np.minimum(sky_cells(w, node_positions(w), n_lon, n_lat), blocks.max())
    rng = np.random.default_rng(seed)
    u = np.sort(rng.choice(w.N, size=R, replace=False)) if R < w.N else np.arange(w.N)
    return w, cfg, raw, a, sl, vec, blocks, nb, u


def _exact_theta(cfg, raw, a, sl, vec):
    """The exact joint posterior of (f, phi) (dense EP with the linear mean in
    the Gaussian mode: one sweep is exact), as f's mean, covariance, phi's
    moments, and the evidence by the information form."""
    from oracle import meanfn
    ep = meanfn.DenseEPTheta(cfg, raw["xyz"], a, raw["sigma"], sightlines=sl, vecchia=vec)
    ep.sweep()
    mu, Sig, Gx, cp = ep.posterior_x()
    A, c0 = ep.f_operator()
    return c0 + A @ mu, A @ Sig @ A.T, ep.theta_posterior()


def test_theta_sites_every_node_inducing_is_exact():
    w, cfg, raw, a, sl, vec, blocks, nb, u = _case_theta(R=125)
    o = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    fm, fV, (pm_, pV_) = _exact_theta(cfg, raw, a, sl, vec)
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, fm) < 1e-8 and _rel(V_u, fV) < 1e-6
    tm, tV = o.theta_posterior()
    assert _rel(tm, pm_) < 1e-9 and _rel(tV, pV_) < 1e-7
    pm, pv = o.predict()
    assert _rel(pm, fm) < 1e-8 and _rel(pv, np.diag(fV)) < 1e-6


def test_theta_sites_one_block_is_exact():
    w, cfg, raw, a, sl, vec, blocks, nb, u = _case_theta(n_lon=1, n_lat=1, R=12)
    assert blocks.max() == 0
    o = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    fm, fV, (pm_, pV_) = _exact_theta(cfg, raw, a, sl, vec)
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, fm[u]) < 1e-9 and _rel(V_u, fV[np.ix_(u, u)]) < 1e-7
    tm, tV = o.theta_posterior()
    assert _rel(tm, pm_) < 1e-9 and _rel(tV, pV_) < 1e-7
    pm, pv = o.predict()
    assert _rel(pm, fm) < 1e-8 and _rel(pv, np.diag(fV)) < 1e-6
    # evidence: a~ ~ N(muhat, G K G^T + S + H S0 H^T), by the determinant lemma
    r = a - o.mu_a
    # marginalise delta first: cov_1 = S + G K G^T, then phi: + H S0 H^T
    C1 = np.diag(o.s2) + o.G @ o.K @ o.G.T
    C1inv = np.linalg.inv(C1)
    M = np.diag(1.0 / o.s0sq) + o.H.T @ C1inv @ o.H
    ld = (np.linalg.slogdet(C1)[1] + np.linalg.slogdet(M)[1] + np.log(o.s0sq).sum())
    t = o.H.T @ C1inv @ r
    quad = r @ C1inv @ r - t @ np.linalg.solve(M, t)
    ref = -0.5 * (len(r) * math.log(2 * math.pi) + ld + quad)
    assert abs(o.log_evidence() - ref) < 1e-9 * abs(ref)


def test_theta_sites_closed_form_with_blocks():
    """Several blocks: q(u, psi) equals the information form of
    p(a~ | u, psi) = N(muhat + Psi (u - mhat_u - J_u psi) + H psi, blockdiag B_k)
    under the prior N(0, C) x N(0, S0) of (u - m(phi), psi)."""
    w, cfg, raw, a, sl, vec, blocks, nb, u = _case_theta(stars=70, R=20, seed=7)
    assert blocks.max() >= 2
    o = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep()
    S = len(a)
    rho = o.G @ o.K[:, u]
    Psi = rho @ o.Cinv
    Lam = np.zeros((S, S))
    for k in range(o.nblk):
        idx = o.members[k]
        Lam[np.ix_(idx, idx)] = (o.G[idx] @ o.K @ o.G[idx].T + np.diag(o.s2[idx]) - rho[idx] @ o.Cinv @ rho[idx].T)
    Li = np.linalg.inv(Lam)
    X = np.hstack([Psi, o.H])                                  # coordinates (du, psi)
    R, M = len(u), o.M
    P = np.zeros((R + M, R + M))
    P[:R, :R] = o.Cinv
    P[R:, R:] = np.diag(1.0 / o.s0sq)
    P += X.T @ Li @ X
    V = np.linalg.inv(P)
    m = V @ (X.T @ Li @ (a - o.mu_a))                          # mean of (du, psi)
    T = np.hstack([np.eye(R), o.Ju])                           # u = mhat_u + du + J_u psi
    mu_ref, V_ref = o.m_u + T @ m, T @ V @ T.T
    mu_u, V_u = o.posterior_u()
    assert _rel(mu_u, mu_ref) < 1e-9 and _rel(V_u, V_ref) < 1e-8
    tm, tV = o.theta_posterior()
    assert _rel(tm, o.mu0 + m[R:]) < 1e-9 and _rel(tV, V[R:, R:]) < 1e-8


def test_theta_sites_damping():
    w, cfg, raw, a, sl, vec, blocks, nb, u = _case_theta(stars=50, R=10, seed=9)
    full = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    full.sweep(1.0)
    half = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl, K=full.K)
    for t in range(1, 3):
        half.sweep(0.5)
        assert _rel(half.Lam, (1 - 0.5 ** t) * full.Lam) < 1e-10


# ---------------------------------------------------------------------------
# the extinction likelihood: one Gaussian site per star under the PITC prior
# ---------------------------------------------------------------------------
def _ext_case(n=5, L=400.0, stars=40, n_lon=3, n_lat=1, R=10, seed=7, exact_prior=False):
    w = Workload("pitcx", n=n, box_pc=L, n_stars=stars, sweeps=1, star_law="uniform", d_max_pc=L,
                 noise_law="const", noise_a=0.05, likelihood="extinction", seed_id=seed)
    cfg = w.ep_fields()
    if exact_prior:
        # conditioning on every earlier node: the Vecchia factor is the exact
        # (tapered) prior, so the grid path's EP sees the same prior of a
        cfg["vecchia_radius_pc"] = cfg["support_pc"] = 4.0 * L
    raw = draw(w)
    f_true, A, sl = epo.simulate(cfg, raw)
    blocks = sky_cells(w, raw["xyz"], n_lon, n_lat)
    node_block = sky_cells(w, node_positions(w), n_lon, n_lat)
    rng = np.random.default_rng(seed)
    u = np.sort(rng.choice(w.N, size=R, replace=False))
    return w, cfg, raw, A, sl, blocks, node_block, u


def test_ext_one_block_with_the_exact_prior_is_the_grid_ep():
    """One sub-catalogue holding every star and an exact prior: PITC is then
    exact, so the star sites, the posterior of a and the predictive of f must
    be those of the grid path's EP with sightlines frozen at the prior mean
    (which works in f with the Vecchia precision)."""
    w, cfg, raw, A, sl, blocks, nb, u = _ext_case(exact_prior=True)
    one = np.zeros_like(blocks)
    o = pitc.DensePITCExt(cfg, raw["xyz"], A, raw["sigma"], one, u, np.zeros(w.N, dtype=int), sightlines=sl)
    g = epo.DenseEP(dict(cfg, relinearize=False), raw["xyz"], A, raw["sigma"], sightlines=sl)
    for d in (1.0, 0.7, 0.7, 1.0):
        so = o.sweep(d)
        g.damping = d
        sg = g.sweep()
        assert so["updated"] == sg["updated"]
        assert np.allclose(o.tau, g.tau, rtol=1e-8, atol=1e-10) and np.allclose(o.nu, g.nu, rtol=1e-8, atol=1e-8)
    pm, pv = o.predict()
    assert _rel(pm, g.posterior_mean()) < 1e-9
    assert np.allclose(pv, g.marginal_var(), rtol=1e-8)


def test_ext_scaled_forms_match_the_plain_gaussian_conditioning():
    """q(a) and q(u) from the scaled forms against the plain definition: the
    joint Gaussian of (u, a) under PITC times the sites, conditioned with
    explicit inverses (every site set after a sweep)."""
    w, cfg, raw, A, sl, blocks, nb, u = _ext_case()
    o = pitc.DensePITCExt(cfg, raw["xyz"], A, raw["sigma"], blocks, u, nb, sightlines=sl)
    o.sweep(1.0)
    o.sweep(0.8)
    assert np.all(o.tau > 0)
    R, S = len(u), len(A)
    Jc = np.block([[o.C, o.rho.T], [o.rho, o.Q]])
    P = np.linalg.inv(Jc)
    P[R:, R:] += np.diag(o.tau)
    V = np.linalg.inv(P)
    m0 = np.concatenate([o.m_u, o.mu_a])
    mean = V @ (np.linalg.solve(Jc, m0) + np.concatenate([np.zeros(R), o.nu]))
    ma, Pa = o.posterior_a()
    mu_, Vu = o.posterior_u()
    assert _rel(ma, mean[R:]) < 1e-9 and np.allclose(Pa, V[R:, R:], rtol=1e-7, atol=1e-12)
    assert _rel(mu_, mean[:R]) < 1e-9 and np.allclose(Vu, V[:R, :R], rtol=1e-7, atol=1e-12)


def test_ext_moment_matching_at_convergence():
    """At the fixed point the marginals of q(a) equal the tilted moments of
    the cavities they define (App. A.2), and the sub-catalogue structure
    matters: the sites differ from the one-block ones."""
    w, cfg, raw, A, sl, blocks, nb, u = _ext_case()
    o = pitc.DensePITCExt(cfg, raw["xyz"], A, raw["sigma"], blocks, u, nb, sightlines=sl)
    for it in range(200):
        st = o.sweep(0.7)
        if st["max_dtau"] < 1e-10:
            break
    assert st["max_dtau"] < 1e-10, it
    m, P = o.posterior_a()
    v = np.diag(P)
    tau_c, nu_c = 1 / v - o.tau, m / v - o.nu
    assert np.all(tau_c > 0)
    _, mh, vh = epo.tilted(epo.LIK_EXTINCTION, nu_c / tau_c, 1 / tau_c, A, raw["sigma"])
    assert np.allclose(m, mh, rtol=1e-8, atol=1e-9) and np.allclose(v, vh, rtol=1e-7)
    one = pitc.DensePITCExt(cfg, raw["xyz"], A, raw["sigma"], np.zeros_like(blocks), u, np.zeros(w.N, dtype=int),
                            sightlines=sl)
    for _ in range(60):
        one.sweep(0.7)
    assert np.max(np.abs(one.tau - o.tau) / o.tau) > 1e-3

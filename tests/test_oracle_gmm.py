"""Pins for the oracle's EP with unknown distances (Sec. 4.2 general case):
the extended sightline forward model on fields with closed forms, the
distance-marginalised tilted moments against brute-force 2-D quadrature of
the (a, ln s) integrand with the extinction at each distance from an
independent discretisation, the closed-form mixture where the extinction
curve is exactly linear in ln s, the far alias where a one-derivative
projection fails, the known-distance limits, and the EP plumbing against the
Gaussian-likelihood EP."""
import math

import numpy as np
import pytest

from oracle import epo, gmm
from synth import Workload, draw, gmm_catalogue


def _cfg(n=8, L=700.0):
    return dict(n=n, box_pc=L, observer_pc=(L / 2, 0.0, L / 2), prior_mean=-7.0, prior_var=1.0,
                outer_scale_pc=100.0, support_pc=150.0, los_step_pc=2.0)


def _n2(l, b, m, C):
    det = C[0] * C[2] - C[1] ** 2
    dl, db = l - m[0], b - m[1]
    q = (C[2] * dl * dl - 2 * C[1] * dl * db + C[0] * db * db) / det
    return np.exp(-0.5 * q) / (2 * math.pi * math.sqrt(det))


def _lnA_R8(cfg, o, u, s):
    """ln A to the points o + s u by the oracle's star forward model (its own
    step count T = ceil(s / step) at each distance): an independent
    discretisation of the same integral."""
    sl = epo.Sightlines(cfg, o[None, :] + np.asarray(s)[:, None] * u[None, :])
    return sl


def test_ray_extinction_on_constant_and_linear_fields():
    cfg = _cfg()
    rng = np.random.default_rng(3)
    o = np.asarray(cfg["observer_pc"])
    xyz = rng.uniform(50, 650, (12, 3))
    N = cfg["n"] ** 3
    # constant field: A(s) = s e^c at every distance (lattice points or not)
    for x in xyz:
        ray = gmm.Ray(cfg, x)
        s = np.concatenate([rng.uniform(0.1, ray.s_exit, 40), [ray.s_ref, ray.s_exit, 0.3 * ray.delta]])
        A, Aref = ray.extinction(np.full(N, -6.3), s)
        assert np.allclose(A, s * math.exp(-6.3), rtol=1e-13, atol=0)
        assert Aref == pytest.approx(ray.s_ref * math.exp(-6.3), rel=1e-13)
    # linear field F = F0 + k.x (trilinear reproduces it): along the ray
    # A(s) = e^{F(o)} (e^{beta s} - 1)/beta, trapezoid error O(step^2)
    kv = np.array([1.5e-3, -1.0e-3, 2.0e-3])
    pos = epo.Grid(cfg).xyz()
    f = -6.0 + pos @ kv
    for x in xyz:
        ray = gmm.Ray(cfg, x)
        u = (x - o) / ray.s_ref
        beta = u @ kv
        s = rng.uniform(1.0, ray.s_exit, 30)
        A, _ = ray.extinction(f, s)
        exact = math.exp(-6.0 + o @ kv) * np.expm1(beta * s) / beta
        assert np.allclose(A, exact, rtol=2e-6)
        # continuity across a lattice point
        t = (ray.T + 3) * ray.delta
        Al, _ = ray.extinction(f, np.array([t * (1 - 1e-12), t, t * (1 + 1e-12)]))
        assert np.ptp(Al) < 1e-10 * Al[1]
    # A(s~) is the star's own forward model (the sightline of the EP sites)
    f = -7.0 + 0.5 * np.sin(pos[:, 0] / 90.0) * np.cos(pos[:, 2] / 70.0)
    sl = epo.Sightlines(cfg, xyz)
    _, lnA, _ = sl.linearise(f)
    for n, x in enumerate(xyz):
        _, Aref = gmm.Ray(cfg, x).extinction(f, np.array([1.0]))
        assert math.log(Aref) == pytest.approx(lnA[n], abs=1e-13)


def _field(cfg, seed):
    w = Workload("f", n=cfg["n"], box_pc=cfg["box_pc"], n_stars=1, sweeps=1, seed_id=seed)
    vec = epo.Vecchia(dict(cfg, vecchia_radius_pc=cfg["support_pc"]))
    return vec.draw(cfg["prior_mean"], draw(w)["xi"])


def _brute(cfg, x, f, mu_c, v_c, comps, na=1601, nl=2401):
    """Moments of N(a; mu_c, v_c) sum_z w_z N2((l, a + delta(l)); m_z, C_z) on
    a dense (a, l) grid, delta(l) = ln A(e^l) - ln A(s~) with A from the
    oracle's star forward model placed at each distance."""
    o = np.asarray(cfg["observer_pc"], dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    d = float(np.linalg.norm(x - o))
    u = (x - o) / d
    ray = gmm.Ray(cfg, x)
    ln_exit = math.log(ray.s_exit)
    sds = np.sqrt(comps[:, 3])
    lo = float(np.min(comps[:, 1] - 9 * sds))
    hi = min(float(np.max(comps[:, 1] + 9 * sds)), ln_exit)
    l = np.linspace(lo, hi, nl)
    sl = epo.Sightlines(cfg, o[None, :] + np.exp(l)[:, None] * u[None, :])
    _, lnA_l, _ = sl.linearise(f)
    sl0 = epo.Sightlines(cfg, x[None, :])
    _, lnA0, _ = sl0.linearise(f)
    dl = lnA_l - lnA0[0]
    sv = math.sqrt(v_c)
    a = np.linspace(mu_c - 11 * sv, mu_c + 11 * sv, na)
    Aa, Ll = np.meshgrid(a, l, indexing="ij")
    Dl = np.broadcast_to(dl[None, :], Aa.shape)
    like = sum(c[0] * _n2(Ll, Aa + Dl, c[1:3], c[3:6]) for c in comps)
    g = np.exp(-0.5 * (Aa - mu_c) ** 2 / v_c) / math.sqrt(2 * math.pi * v_c) * like
    wa = np.full(na, a[1] - a[0])
    wa[[0, -1]] *= 0.5
    wl = np.full(nl, l[1] - l[0])
    wl[[0, -1]] *= 0.5
    W = wa[:, None] * wl[None, :]
    Z = float(np.sum(g * W))
    m1 = float(np.sum(g * W * Aa)) / Z
    m2 = float(np.sum(g * W * (Aa - m1) ** 2)) / Z
    return math.log(Z), m1, m2


def _comps_two(ml, mb, sd_l=0.15, sd_b=0.08, rho=0.6, alias_l=math.log(2.5), alias_b=0.25, w0=0.75):
    c = np.zeros((2, 6))
    c[0] = [w0, ml, mb, sd_l ** 2, rho * sd_l * sd_b, sd_b ** 2]
    c[1] = c[0]
    c[1, 0] = 1 - w0
    c[1, 1] += alias_l
    c[1, 2] += alias_b
    return c


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tilted_matches_2d_quadrature(seed):
    cfg = _cfg(n=9, L=900.0)
    f = _field(cfg, 40 + seed)
    rng = np.random.default_rng(seed)
    o = np.asarray(cfg["observer_pc"])
    x = o + np.array([rng.uniform(-80, 80), rng.uniform(120, 220), rng.uniform(-60, 60)])
    ray = gmm.Ray(cfg, x)
    _, A0 = ray.extinction(f, np.array([1.0]))
    comps = _comps_two(math.log(ray.s_ref) + rng.normal(0, 0.1), math.log(A0) + rng.normal(0, 0.1))
    mu_c, v_c = math.log(A0) + rng.normal(0, 0.2), rng.uniform(0.02, 0.3)
    lnZ, mean, var = gmm.tilted_one(ray, f, mu_c, v_c, comps)
    bz, bm, bv = _brute(cfg, x, f, mu_c, v_c, comps)
    print(f"seed {seed}: lnZ {lnZ:.8f}/{bz:.8f} mean {mean:.8f}/{bm:.8f} var {var:.8e}/{bv:.8e}")
    assert abs(lnZ - bz) < 2e-5
    assert abs(mean - bm) < 2e-5 * max(1.0, abs(bm))
    assert abs(var - bv) < 1e-4 * bv


def test_exactly_linear_extinction_curve_gives_the_closed_form_mixture():
    # constant field: delta(l) = l - l~ exactly, so each component's
    # likelihood in a_n is the density of b - (l - l~) under (l, b) ~ N(m, C):
    # N(a_n; m_b - (m_l - l~), C_bb - 2 C_lb + C_ll), a Gaussian mixture with
    # closed-form moments
    cfg = _cfg(n=8, L=1400.0)
    N = cfg["n"] ** 3
    f = np.full(N, -6.8)
    o = np.asarray(cfg["observer_pc"])
    rng = np.random.default_rng(8)
    for _ in range(6):
        x = o + np.array([rng.uniform(-30, 30), rng.uniform(40, 80), rng.uniform(-30, 30)])
        ray = gmm.Ray(cfg, x)
        lref = math.log(ray.s_ref)
        comps = _comps_two(lref + rng.normal(0, 0.1), rng.normal(-1, 0.3), sd_l=rng.uniform(0.05, 0.2),
                           sd_b=rng.uniform(0.03, 0.1), rho=rng.uniform(-0.7, 0.7))
        assert np.all(comps[:, 1] + 8 * np.sqrt(comps[:, 3]) < math.log(ray.s_exit))   # no clipping
        mu_c, v_c = rng.normal(-1, 0.3), rng.uniform(0.01, 0.4)
        lnZ, mean, var = gmm.tilted_one(ray, f, mu_c, v_c, comps)
        m = comps[:, 2] - (comps[:, 1] - lref)
        v = comps[:, 5] - 2 * comps[:, 4] + comps[:, 3]
        s = v_c + v
        lz = np.log(comps[:, 0]) - 0.5 * np.log(2 * math.pi * s) - 0.5 * (m - mu_c) ** 2 / s
        r = np.exp(lz - lz.max())
        mz = (v * mu_c + v_c * m) / s
        vz = v_c * v / s
        Z = r.sum()
        em = (r * mz).sum() / Z
        ev = (r * (vz + (mz - em) ** 2)).sum() / Z
        assert lnZ == pytest.approx(lz.max() + math.log(Z), abs=1e-11)
        assert mean == pytest.approx(em, abs=1e-11)
        assert var == pytest.approx(ev, rel=1e-10)


def test_far_alias_sees_the_extinction_a_derivative_misses():
    # a dense shell between 1.3 s~ and 2.0 s~ from the observer: the alias at
    # 2.5 s~ lies behind it.  The forward model puts that extinction into
    # delta(l); a one-derivative projection at s~ (slope 1 there: the field is
    # flat around the star) extrapolates a(2.5 s~) = a_n + ln 2.5 and misses it.
    cfg = _cfg(n=17, L=1600.0)
    pos = epo.Grid(cfg).xyz()
    o = np.asarray(cfg["observer_pc"])
    r = np.linalg.norm(pos - o, axis=1)
    s0 = 250.0
    f = np.where((r > 1.3 * s0) & (r < 2.0 * s0), -4.5, -7.0)
    x = o + s0 * np.array([0.1, 0.99, 0.1]) / np.linalg.norm([0.1, 0.99, 0.1])
    ray = gmm.Ray(cfg, x)
    _, A0 = ray.extinction(f, np.array([1.0]))
    a0 = math.log(A0)
    comps = _comps_two(math.log(ray.s_ref), a0, w0=0.5)
    # the observation favours the alias: the far component's b matches the
    # extinction behind the shell
    A_far, _ = ray.extinction(f, np.array([2.5 * ray.s_ref]))
    comps[1, 2] = math.log(A_far[0])
    mu_c, v_c = a0, 0.3
    lnZ, mean, var = gmm.tilted_one(ray, f, mu_c, v_c, comps)
    bz, bm, bv = _brute(cfg, x, f, mu_c, v_c, comps)
    # (the shell's sharp edges make the two discretisations of the extinction
    # integral differ by ~1e-4 here)
    assert abs(mean - bm) < 2e-4 and abs(var - bv) < 1e-3 * bv and abs(lnZ - bz) < 2e-4
    # the one-derivative projection (beta = 1 at the star) gives another answer
    m = comps[:, 2] - (comps[:, 1] - math.log(ray.s_ref))
    v = comps[:, 5] - 2 * comps[:, 4] + comps[:, 3]
    s = v_c + v
    lz = np.log(comps[:, 0]) - 0.5 * np.log(2 * math.pi * s) - 0.5 * (m - mu_c) ** 2 / s
    rr = np.exp(lz - lz.max())
    proj_mean = (rr * (v * mu_c + v_c * m) / s).sum() / rr.sum()
    print(f"forward model {mean:.4f}, brute force {bm:.4f}, one-derivative projection {proj_mean:.4f}")
    assert abs(proj_mean - mean) > 0.1


def test_known_distances_are_gaussian_likelihoods():
    cfg = _cfg(n=9, L=900.0)
    f = _field(cfg, 50)
    o = np.asarray(cfg["observer_pc"])
    rng = np.random.default_rng(5)
    for _ in range(8):
        x = o + np.array([rng.uniform(-100, 100), rng.uniform(100, 300), rng.uniform(-100, 100)])
        ray = gmm.Ray(cfg, x)
        mu_c, v_c = rng.normal(-2, 0.3), rng.uniform(0.01, 0.4)
        sb = rng.uniform(0.02, 0.2)
        # at the catalogue distance: N(a_n; m_b, C_bb)
        c = np.array([[1.0, math.log(ray.s_ref), -1.7, 0.0, 0.0, sb * sb]])
        lz, m, v = gmm.tilted_one(ray, f, mu_c, v_c, c)
        lz2, m2, v2 = epo.tilted(1, [mu_c], [v_c], [-1.7], [sb])
        assert lz == pytest.approx(lz2[0], abs=1e-12) and m == pytest.approx(m2[0], abs=1e-13)
        assert v == pytest.approx(v2[0], rel=1e-12)
        # at another known distance s: N(a_n + delta(s); m_b, C_bb), delta from
        # the star forward model placed at s (another discretisation)
        s = ray.s_ref * rng.uniform(0.5, 1.8)
        c[0, 1] = math.log(s)
        lz, m, v = gmm.tilted_one(ray, f, mu_c, v_c, c)
        u = (x - o) / ray.s_ref
        _, lnA, _ = epo.Sightlines(cfg, np.stack([o + s * u, x])).linearise(f)
        lz2, m2, v2 = epo.tilted(1, [mu_c], [v_c], [-1.7 - (lnA[0] - lnA[1])], [sb])
        assert lz == pytest.approx(lz2[0], abs=5e-5) and m == pytest.approx(m2[0], abs=5e-5)
        assert v == pytest.approx(v2[0], rel=1e-12)


def test_distances_outside_the_cube_carry_no_likelihood():
    cfg = _cfg(n=9, L=900.0)
    f = _field(cfg, 51)
    o = np.asarray(cfg["observer_pc"])
    x = o + np.array([30.0, 400.0, -20.0])
    ray = gmm.Ray(cfg, x)
    c = _comps_two(math.log(ray.s_ref), -1.0)
    far = c[1].copy()
    far[1] = math.log(ray.s_exit) + 9 * math.sqrt(far[3])      # wholly past the cube's face
    near_only = gmm.tilted_one(ray, f, -1.1, 0.1, c[:1])
    with_far = gmm.tilted_one(ray, f, -1.1, 0.1, np.stack([c[0], far]))
    assert with_far == near_only
    none = gmm.tilted_one(ray, f, -1.1, 0.1, far[None, :])
    assert none[0] == -math.inf and math.isnan(none[1]) and math.isnan(none[2])


def test_degenerate_mixture_ep_is_the_gaussian_ep():
    # every star: one component at the catalogue distance with no distance
    # spread, so the likelihood is N(a; m_b, C_bb): the mixture EP must give
    # the Gaussian-likelihood EP's sites (frozen linearisation in both)
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
    comps[:, 0, 5] = raw["sigma"] ** 2
    a = gmm.DenseEPGMM(cfg, raw["xyz"], comps)
    b = epo.DenseEP(cfg, raw["xyz"], comps[:, 0, 2], raw["sigma"])
    for _ in range(2):
        a.sweep()
        b.sweep()
        assert np.allclose(a.tau, b.tau, rtol=1e-12) and np.allclose(a.nu, b.nu, rtol=1e-12, atol=1e-12)
    assert np.allclose(a.posterior_mean(), b.posterior_mean(), rtol=1e-12)


def test_mixture_ep_uses_the_linearisation_point_of_its_sweep():
    # re-linearised mixture EP: each sweep's tilted moments come from the
    # cavity of that sweep's q and delta(s) at the point the sweep linearised
    # about (fhat before the sweep moves it)
    w = Workload("t", n=7, box_pc=700.0, n_stars=25, sweeps=2, star_law="uniform", d_max_pc=700.0,
                 noise_law="const", noise_a=0.05, seed_id=9)
    cfg = dict(w.ep_fields(), damping=0.7)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    o = np.asarray(cfg["observer_pc"])
    cat = gmm_catalogue(w, raw["xyz"], np.log(np.maximum(A_obs, 1e-3)))
    ep = gmm.DenseEPGMM(cfg, cat["xyz"], cat["comps"])
    for _ in range(3):
        fhat = ep.fhat.copy()
        mu, Sig, G, c = ep.posterior()
        st = ep.sweep()
        lz, m, v = gmm.gmm_tilted(cfg, cat["xyz"], fhat, st["cav_mu"], st["cav_var"], cat["comps"])
        assert np.array_equal(m, st["tilted_mean"]) and np.array_equal(v, st["tilted_var"])
        assert np.allclose(ep.fhat, mu, rtol=1e-12)
    assert np.max(np.abs(ep.fhat - cfg["prior_mean"])) > 0.01


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
    comps[:, 0, 5] = raw["sigma"] ** 2
    a = gmm.DenseEPThetaGMM(cfg, raw["xyz"], comps)
    b = meanfn.DenseEPTheta(cfg, raw["xyz"], comps[:, 0, 2], raw["sigma"])
    for _ in range(2):
        a.sweep()
        b.sweep()
        assert np.allclose(a.tau, b.tau, rtol=1e-12) and np.allclose(a.nu, b.nu, rtol=1e-12, atol=1e-12)
    assert np.allclose(a.theta_posterior()[0], b.theta_posterior()[0], rtol=1e-12)

"""GPU parity of EP with the inferred disc + bump prior mean (the field and
phi = ln theta jointly; the five parameters as a Schur-complement border of
the grid factorization) against the dense FP64 oracle, through the C ABI.
FP64 throughout: 1e-8 relative."""
import numpy as np
import pytest

from oracle import meanfn

from gpu_common import relerr
from synth import Workload, draw

pytestmark = pytest.mark.gpu

THETA_PRIOR = (1500.0, 150.0, 7.5e-4, 600.0, 0.1)
THETA_TRUE = (1000.0, 200.0, 1.2e-3, 500.0, 0.2)


def _case(n=9, L=1200.0, stars=200, lik="extinction", leaf=48, seed=21):
    w = Workload("t", n=n, box_pc=L, n_stars=stars, sweeps=3, star_law="uniform", d_max_pc=L,
                 noise_law="const", noise_a=0.05, likelihood=lik, seed_id=seed)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=200.0, theta_prior=THETA_PRIOR)
    raw = draw(w)
    f_true, A, sl = meanfn.simulate(cfg, raw, THETA_TRUE)
    gcfg = dict(cfg, leaf_size=leaf, mean_fn="disc_bump")
    gcfg.pop("sweeps", None)
    return cfg, gcfg, raw, A, sl


def _rel_phi(a, b):
    return float(np.max(np.abs(np.asarray(a) - b) / np.maximum(np.abs(b), 1.0)))


@pytest.mark.parametrize("n,L,stars,leaf,relin_step", [(8, 1000.0, 120, 32, 1.0), (9, 1200.0, 200, 48, 1.0),
                                                        (11, 1200.0, 300, 64, 1.0), (9, 1200.0, 200, 48, 0.5)])
def test_theta_ep_matches_oracle(n, L, stars, leaf, relin_step):
    from paper_1708_09705_amd import ep as E
    cfg, gcfg, raw, A, sl = _case(n=n, L=L, stars=stars, leaf=leaf)
    cfg["relin_step"] = gcfg["relin_step"] = relin_step
    print(f"case n={n} L={L} stars={stars} relin_step={relin_step}", flush=True)
    ora = meanfn.DenseEPTheta(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    for s in range(3):
        so = ora.sweep()
        sg = g.sweep()
        tg, ng = g.sites()
        print(f"sweep {s}: tau {relerr(tg, ora.tau):.2e} nu {relerr(ng, ora.nu):.2e} "
              f"updated {sg['updated']}/{so['updated']}", flush=True)
        assert sg["updated"] == so["updated"]
        assert np.allclose(tg, ora.tau, rtol=1e-8, atol=1e-10)
        assert np.allclose(ng, ora.nu, rtol=1e-8, atol=1e-8)
    mo, vo = ora.posterior_mean(), ora.marginal_var()
    mg, vg = g.posterior_mean(), g.marginal_var()
    pm_o, pc_o = ora.theta_posterior()
    pm_g, pc_g = g.theta()
    print(f"f mean {relerr(mg, mo):.2e} var {relerr(vg, vo):.2e}; phi mean {_rel_phi(pm_g, pm_o):.2e} "
          f"cov {relerr(pc_g, pc_o):.2e}; phi {pm_g}", flush=True)
    assert relerr(mg, mo) < 1e-8 and relerr(vg, vo) < 1e-8
    assert _rel_phi(pm_g, pm_o) < 1e-8
    assert np.allclose(pc_g, pc_o, rtol=1e-8, atol=1e-12 * np.abs(pc_o).max())
    # the linearisation point carries phihat
    lp = g.linpoint()
    assert lp.shape == (n ** 3 + 5,) and np.allclose(lp[-5:], ora.phihat, rtol=1e-8, atol=1e-10)
    assert relerr(lp[:-5], ora.fhat) < 1e-8
    # density moments of f
    dm, dv = g.density_moments()
    om, ov = np.exp(mo + vo / 2), np.expm1(vo) * np.exp(2 * mo + vo)
    assert relerr(dm, om) < 1e-8 and relerr(dv, ov) < 1e-8
    g.close()


def test_theta_gaussian_likelihood_one_sweep():
    from paper_1708_09705_amd import ep as E
    cfg, gcfg, raw, A, sl = _case(n=9, L=1200.0, stars=200, lik="gauss_linear")
    # observations of a_n in the Gaussian mode (any values do): the site
    # variable is linear, with g and c frozen at the prior mean m(x; mu0)
    y = np.log(np.maximum(A, 1e-3))
    ora = meanfn.DenseEPTheta(cfg, raw["xyz"], y, raw["sigma"], sightlines=sl)
    g = E.EP(gcfg, raw["xyz"], y, raw["sigma"])
    ora.sweep()
    g.sweep()
    tau, nu = g.sites()
    assert np.allclose(tau, 1 / raw["sigma"] ** 2, rtol=1e-9)
    assert np.allclose(nu, y / raw["sigma"] ** 2, rtol=1e-8, atol=1e-8)
    assert relerr(g.posterior_mean(), ora.posterior_mean()) < 1e-8
    assert relerr(g.marginal_var(), ora.marginal_var()) < 1e-8
    pm_o, pc_o = ora.theta_posterior()
    pm_g, pc_g = g.theta()
    assert _rel_phi(pm_g, pm_o) < 1e-8
    assert np.allclose(pc_g, pc_o, rtol=1e-8, atol=1e-12 * np.abs(pc_o).max())
    g.close()


def test_theta_checkpoint_resume():
    from paper_1708_09705_amd import ep as E
    cfg, gcfg, raw, A, sl = _case(n=8, L=1000.0, stars=120, leaf=32)
    a = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    for _ in range(2):
        a.sweep()
    tau, nu = a.sites()
    lp = a.linpoint()
    b = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    b.set_sites(tau, nu)
    b.set_linpoint(lp)
    a.sweep()
    b.sweep()
    ta, na = a.sites()
    tb, nb = b.sites()
    assert relerr(tb, ta) < 1e-10 and relerr(nb, na) < 1e-10
    assert _rel_phi(b.theta()[0], a.theta()[0]) < 1e-10
    a.close()
    b.close()


def test_theta_errors():
    from paper_1708_09705_amd import ep as E
    cfg, gcfg, raw, A, sl = _case(n=8, L=1000.0, stars=120, leaf=32)
    for bad in (dict(precision="mixed"), dict(theta_prior=(1500.0, 0.0, 7.5e-4, 600.0, 0.1)),
                dict(bump_width_pc=0.0), dict(mean_fn=7)):
        with pytest.raises(E.EPError) as ei:
            E.EP(dict(gcfg, **bad), raw["xyz"], A, raw["sigma"])
        assert ei.value.code == -1
    g = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    g.sweep()
    with pytest.raises(E.EPError) as ei:
        g.extinction_map()
    assert ei.value.code == -5
    with pytest.raises(E.EPError) as ei:
        g.point_predict(np.array([[100.0, 100.0, 100.0, 105.0, 100.0, 100.0]]))
    assert ei.value.code == -5
    bad_lp = g.linpoint()
    bad_lp[-1] = np.nan
    with pytest.raises(E.EPError) as ei:
        g.set_linpoint(bad_lp)
    assert ei.value.code == -1
    g.close()
    h = E.EP(dict(gcfg, mean_fn="constant"), raw["xyz"], A, raw["sigma"])
    with pytest.raises(E.EPError) as ei:
        h.theta()
    assert ei.value.code == -5
    assert h.linpoint().shape == (8 ** 3,)
    h.close()


# ---- the 64^3 / 100,000-star workload (the benchmark's launch configuration) ----
@pytest.fixture(scope="module")
def cfg2_theta():
    from oracle import epo
    from synth import preset
    w = preset(2)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=400.0, theta_prior=meanfn.DEFAULT_PRIOR)
    raw = draw(w)
    vec = epo.Vecchia(cfg)
    pos = vec.grid.xyz()
    mu0, s0sq = meanfn.hyperprior(cfg)
    m0, J0 = meanfn.mean_and_jacobian(cfg, pos, mu0)
    return w, cfg, raw, vec, mu0, s0sq, m0, J0


def test_config2_theta_first_sweep_sites_sampled(cfg2_theta):
    """Sweep 1 starts from zero sites, so every star's cavity is its prior
    marginal under the joint prior of (delta, phi): mean ln A_n(m(mu0)),
    variance g^T Q0^{-1} g + h^T diag(s0^2) h with h = J^T g.  Sampled stars,
    computed one by one by the oracle."""
    from oracle import epo
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, vec, mu0, s0sq, m0, J0 = cfg2_theta
    f_true, A, _ = meanfn.simulate(cfg, raw, (2500.0, 200.0, 1.2e-3, 1800.0, 0.15), vecchia=vec)
    g = E.EP(dict(cfg, leaf_size=512, mean_fn="disc_bump"), raw["xyz"], A, raw["sigma"])
    g.sweep()
    tau_g, nu_g = g.sites()
    g.close()
    idx = np.random.default_rng(6).choice(w.n_stars, 48, replace=False)
    sl = epo.Sightlines(cfg, raw["xyz"][idx])
    gval, lnA, c = sl.linearise(m0)
    rows = np.repeat(np.arange(len(idx)), np.diff(sl.ptr))
    h = np.stack([np.bincount(rows, weights=gval * J0[sl.nodes, j], minlength=len(idx)) for j in range(5)], axis=1)
    v = vec.prior_quadform(sl.ptr, sl.nodes, gval) + (h ** 2) @ s0sq
    _, mh, vh = epo.tilted(0, lnA, v, A[idx], raw["sigma"][idx])
    tau_o = 1 / vh - 1 / v
    nu_o = mh / vh - lnA / v
    print(f"config 2 theta sampled sites: tau {relerr(tau_g[idx], tau_o):.2e} nu {relerr(nu_g[idx], nu_o):.2e}",
          flush=True)
    assert np.allclose(tau_g[idx], tau_o, rtol=1e-8)
    assert np.allclose(nu_g[idx], nu_o, rtol=1e-8, atol=1e-8)


def test_config2_theta_gaussian_mode_residual(cfg2_theta):
    """Gaussian likelihood at full size: after one sweep the sites are the
    likelihood's, and (mu_delta, mu_phi) recovered from the outputs solve the
    bordered system with the oracle's own Q0, G, J and those sites."""
    from oracle import epo
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, vec, mu0, s0sq, m0, J0 = cfg2_theta
    cfg = dict(cfg, likelihood="gauss_linear")
    sl = epo.Sightlines(cfg, raw["xyz"])
    gval, _, c = sl.linearise(m0)
    rows = np.repeat(np.arange(sl.n_stars), np.diff(sl.ptr))
    Gx = lambda x: np.bincount(rows, weights=gval * x[sl.nodes], minlength=sl.n_stars)
    GT = lambda y: np.bincount(sl.nodes, weights=gval * y[rows], minlength=sl.grid.N)
    f_true = m0 + vec.draw(0.0, raw["xi"])
    a_obs = c + Gx(f_true) + raw["sigma"] * raw["eps"]
    # the mean's linearisation frozen at mu0 (relinearize = 0), so the
    # outputs are those of the system built at m0, J0
    g = E.EP(dict(cfg, leaf_size=512, mean_fn="disc_bump", relinearize=0), raw["xyz"], a_obs, raw["sigma"])
    g.sweep()
    tau, nu = g.sites()
    assert np.allclose(tau, 1 / raw["sigma"] ** 2, rtol=1e-9)
    fm = g.posterior_mean()
    mphi, _ = g.theta()
    g.close()
    tau_o, nu_o = 1 / raw["sigma"] ** 2, a_obs / raw["sigma"] ** 2
    H = np.stack([Gx(J0[:, j]) for j in range(5)], axis=1)
    cp = c + Gx(m0) - H @ mu0
    mdel = fm - m0 - J0 @ (mphi - mu0)
    r = nu_o - tau_o * cp
    row_d = vec.Q0_matvec(mdel) + GT(tau_o * (Gx(mdel) + H @ mphi)) - GT(r)
    row_p = mphi / s0sq + H.T @ (tau_o * (Gx(mdel) + H @ mphi)) - (mu0 / s0sq + H.T @ r)
    res_d = np.linalg.norm(row_d) / np.linalg.norm(GT(r))
    res_p = np.linalg.norm(row_p) / np.linalg.norm(mu0 / s0sq + H.T @ r)
    print(f"config 2 theta gaussian: residuals delta {res_d:.2e} phi {res_p:.2e}; phi {mphi}", flush=True)
    assert res_d < 1e-10 and res_p < 1e-10

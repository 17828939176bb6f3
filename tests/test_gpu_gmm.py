"""GPU parity of EP with unknown distances (per-star distance / extinction
mixtures, the distance marginalised in the tilted distribution) against the
dense FP64 oracle, through the C ABI.  FP64: 1e-8 relative."""
import numpy as np
import pytest

from oracle import epo, gmm

from gpu_common import relerr
from synth import Workload, draw, gmm_catalogue, preset

pytestmark = pytest.mark.gpu


def _case(n=9, L=700.0, stars=200, leaf=48, seed=31):
    w = Workload("t", n=n, box_pc=L, n_stars=stars, sweeps=3, star_law="uniform", d_max_pc=L,
                 noise_law="const", noise_a=0.05, seed_id=seed)
    cfg = w.ep_fields()
    raw = draw(w)
    vec = epo.Vecchia(cfg)
    f_true = vec.draw(cfg["prior_mean"], raw["xi"])
    _, lnA_true, _ = epo.Sightlines(cfg, raw["xyz"]).linearise(f_true)
    cat = gmm_catalogue(w, raw["xyz"], lnA_true)
    gcfg = dict(cfg, leaf_size=leaf, likelihood="gmm")
    return w, cfg, gcfg, cat, vec


@pytest.mark.parametrize("n,L,stars,leaf,relin_step", [(8, 500.0, 80, 32, 1.0), (10, 700.0, 200, 48, 1.0),
                                                        (12, 800.0, 300, 64, 1.0), (10, 700.0, 200, 48, 0.5)])
def test_gmm_ep_matches_oracle(n, L, stars, leaf, relin_step):
    from paper_1708_09705_amd import ep as E
    w, cfg, gcfg, cat, vec = _case(n=n, L=L, stars=stars, leaf=leaf)
    cfg["relin_step"] = gcfg["relin_step"] = relin_step
    print(f"case n={n} L={L} stars={stars} relin_step={relin_step}", flush=True)
    ora = gmm.DenseEPGMM(cfg, cat["xyz"], cat["comps"], vecchia=vec)
    g = E.EP(gcfg, cat["xyz"])
    g.set_gmm(cat["comps"])
    for s in range(3):
        so = ora.sweep()
        sg = g.sweep()
        tg, ng = g.sites()
        st = g.star_state()
        ok = st["tilted_var"] > 0
        print(f"sweep {s}: tau {relerr(tg, ora.tau):.2e} nu {relerr(ng, ora.nu):.2e} "
              f"lnZ {relerr(st['lnZ'][ok], so['lnZ'][ok]):.2e} updated {sg['updated']}/{so['updated']}", flush=True)
        assert sg["updated"] == so["updated"]
        assert np.allclose(tg, ora.tau, rtol=1e-8, atol=1e-10)
        assert np.allclose(ng, ora.nu, rtol=1e-8, atol=1e-8)
        assert np.allclose(st["tilted_mean"], so["tilted_mean"], rtol=1e-8, atol=1e-10)
    mo, vo = ora.posterior_mean(), ora.marginal_var()
    mg, vg = g.posterior_mean(), g.marginal_var()
    print(f"posterior: mean {relerr(mg, mo):.2e} var {relerr(vg, vo):.2e}", flush=True)
    assert relerr(mg, mo) < 1e-8 and relerr(vg, vo) < 1e-8
    g.close()


def test_gmm_errors():
    from paper_1708_09705_amd import ep as E
    w, cfg, gcfg, cat, vec = _case(n=8, L=500.0, stars=80, leaf=32)
    g = E.EP(gcfg, cat["xyz"])
    with pytest.raises(E.EPError) as ei:
        g.sweep()                                   # no mixtures yet
    assert ei.value.code == -5
    bad = cat["comps"].copy()
    bad[3, 0, 5] = -0.1
    for c in (bad, np.full_like(cat["comps"], np.nan), np.zeros((80, 9, 6))):
        with pytest.raises(E.EPError) as ei:
            g.set_gmm(c)
        assert ei.value.code == -1
    g.set_gmm(cat["comps"])
    g.sweep()
    g.set_gmm(cat["comps"][:, :1].copy())           # K changes: one component
    g.sweep()
    g.close()
    with pytest.raises(E.EPError) as ei:
        E.EP(dict(gcfg, moments="surrogate"), cat["xyz"])
    assert ei.value.code == -1
    h = E.EP(dict(gcfg, likelihood="extinction"), cat["xyz"], np.ones(80), np.full(80, 0.05))
    with pytest.raises(E.EPError) as ei:
        h.set_gmm(cat["comps"])
    assert ei.value.code == -5
    h.close()


def test_config2_gmm_first_sweep_sites_sampled():
    """64^3 / 100,000 stars (the bench launch configuration): sweep 1 starts
    from zero sites, so a star's cavity is its prior marginal (mean ln A at
    m0, variance g^T Q0^{-1} g) and the extinction curves are those of the
    constant prior mean; sampled stars' sites computed one by one by the
    oracle (its distance quadrature along each extended sightline)."""
    from paper_1708_09705_amd import ep as E
    w = preset(2)
    cfg = w.ep_fields()
    raw = draw(w)
    vec = epo.Vecchia(cfg)
    f_true = vec.draw(cfg["prior_mean"], raw["xi"])
    _, lnA_true, _ = epo.Sightlines(cfg, raw["xyz"]).linearise(f_true)
    cat = gmm_catalogue(w, raw["xyz"], lnA_true)
    g = E.EP(dict(cfg, leaf_size=512, likelihood="gmm"), cat["xyz"])
    g.set_gmm(cat["comps"])
    g.sweep()
    tau_g, nu_g = g.sites()
    g.close()
    idx = np.random.default_rng(7).choice(w.n_stars, 48, replace=False)
    sl = epo.Sightlines(cfg, cat["xyz"][idx])
    f0 = np.full(sl.grid.N, cfg["prior_mean"])
    gval, lnA, c = sl.linearise(f0)
    v = vec.prior_quadform(sl.ptr, sl.nodes, gval)
    _, mh, vh = gmm.gmm_tilted(cfg, cat["xyz"][idx], f0, lnA, v, cat["comps"][idx])
    tau_o = 1 / vh - 1 / v
    nu_o = mh / vh - lnA / v
    neg = ~(tau_o >= 0)                 # a negative site update is skipped: the site stays 0
    tau_o, nu_o = np.where(neg, 0.0, tau_o), np.where(neg, 0.0, nu_o)
    print(f"config 2 gmm sampled sites: tau {relerr(tau_g[idx], tau_o):.2e} nu {relerr(nu_g[idx], nu_o):.2e}; "
          f"{int(neg.sum())} of {len(idx)} skipped", flush=True)
    assert np.allclose(tau_g[idx], tau_o, rtol=1e-8)
    assert np.allclose(nu_g[idx], nu_o, rtol=1e-8, atol=1e-8)


def test_gmm_with_inferred_mean_matches_oracle():
    """Both widenings at once: the disc + bump mean inferred with the field,
    and per-star distance mixtures."""
    from paper_1708_09705_amd import ep as E
    from oracle import meanfn
    w = Workload("t", n=9, box_pc=1200.0, n_stars=200, sweeps=3, star_law="uniform", d_max_pc=1200.0,
                 noise_law="const", noise_a=0.05, seed_id=33)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=200.0, theta_prior=(1500.0, 150.0, 7.5e-4, 600.0, 0.1))
    raw = draw(w)
    f_true, _, sl = meanfn.simulate(cfg, raw, (1000.0, 200.0, 1.2e-3, 500.0, 0.2))
    _, lnA_true, _ = sl.linearise(f_true)
    cat = gmm_catalogue(w, raw["xyz"], lnA_true)
    ora = gmm.DenseEPThetaGMM(cfg, cat["xyz"], cat["comps"])
    g = E.EP(dict(cfg, leaf_size=48, likelihood="gmm", mean_fn="disc_bump"), cat["xyz"])
    g.set_gmm(cat["comps"])
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
    assert relerr(g.posterior_mean(), mo) < 1e-8 and relerr(g.marginal_var(), vo) < 1e-8
    pm_o, _ = ora.theta_posterior()
    pm_g, _ = g.theta()
    assert np.max(np.abs(pm_g - pm_o) / np.maximum(np.abs(pm_o), 1.0)) < 1e-8
    g.close()

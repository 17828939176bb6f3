"""GPU parity of the PITC sub-catalogue EP and the PIC predictive (Sec. 4.1,
App. A.1, App. B, App. C) against the dense FP64 oracle, through the C ABI:
q(u) (mean and covariance), the PITC log evidence, and the predictive mean
and variance of the field at every node.  FP64 throughout; the two sides
differ only in rounding order (covariance form with explicit inverses in the
oracle, whitened Cholesky form on the GPU): 1e-8 relative."""
import numpy as np
import pytest

from oracle import pitc

from gpu_common import relerr
from synth import Workload, draw, preset
from synth.workloads import boundary_inducing, node_positions, sky_cells

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def _case(n, L, stars, n_lon, n_lat, R, law="uniform", seed=31, inducing="random", lik="gauss_linear"):
    w = Workload("pitc", n=n, box_pc=L, n_stars=stars, sweeps=1, star_law=law, d_max_pc=L,
                 noise_law="uniform", noise_a=0.05, noise_b=0.15, likelihood=lik, seed_id=seed)
    cfg = w.ep_fields()
    raw = draw(w)
    from oracle import epo
    f_true, a_obs, sl = epo.simulate(cfg, raw)
    blocks = sky_cells(w, raw["xyz"], n_lon, n_lat)
    # relabel to drop empty cells: every sub-catalogue holds stars
    used, blocks = np.unique(blocks, return_inverse=True)
    node_cell = sky_cells(w, node_positions(w), n_lon, n_lat)
    lut = np.full(n_lon * n_lat, -1)
    lut[used] = np.arange(len(used))
    # nodes of an empty cell go to the nearest used cell by index
    for c in range(n_lon * n_lat):
        if lut[c] < 0:
            lut[c] = int(np.argmin(np.abs(used - c)))
    node_block = lut[node_cell].astype(np.int32)
    if inducing == "random":
        u = np.sort(np.random.default_rng(seed).choice(w.N, size=R, replace=False)).astype(np.int32)
    else:
        u = boundary_inducing(w, n_lon, n_lat, inducing)
    return w, cfg, raw, a_obs, sl, blocks.astype(np.int32), u, node_block


def _pair(case, damping=(1.0,)):
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, a, sl, blocks, u, nb = case
    ora = pitc.DensePITC(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    g = E.EP(dict(cfg, leaf_size=48), raw["xyz"], a, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    lz = None
    for d in damping:
        ora.sweep(d)
        lz = g.pitc_sweep(d)
    return ora, g, lz


# sub-catalogues of 1-3 row tiles with ragged tails, R of 1-3 tiles, prediction
# sets of several tiles; the last case has the paper's layout (disc stars,
# inducing points on the cell boundaries at fixed distances)
CASES = [
    dict(n=8, L=600.0, stars=150, n_lon=3, n_lat=2, R=40),
    dict(n=9, L=800.0, stars=400, n_lon=3, n_lat=1, R=150, seed=33),
    dict(n=10, L=1000.0, stars=500, n_lon=4, n_lat=2, R=0, law="disc", seed=35,
         inducing=(250.0, 500.0, 750.0, 1000.0)),
    # one sub-catalogue of 21 row tiles: its late column updates are cut in K
    dict(n=8, L=600.0, stars=1300, n_lon=1, n_lat=1, R=60, seed=39),
    # a taper of one spacing in a 12^3 grid: the covariance products skip
    # the K tiles the taper zeroes
    dict(n=12, L=2000.0, stars=400, n_lon=2, n_lat=1, R=90, seed=41),
]


@pytest.mark.parametrize("kw", CASES, ids=["n8-6blk", "n9-3blk-3tiles", "n10-disc-boundary", "n8-1blk-21tiles",
                                    "n12-narrow-taper"])
def test_pitc_matches_oracle(kw):
    case = _case(**kw)
    w, cfg, raw, a, sl, blocks, u, nb = case
    print(f"case n={kw['n']} stars={kw['stars']} blocks={blocks.max() + 1} R={len(u)} "
          f"block sizes {np.bincount(blocks).min()}-{np.bincount(blocks).max()}", flush=True)
    ora, g, lz = _pair(case)
    om, oV = ora.posterior_u()
    gm, gV = g.pitc_inducing()
    olz = ora.log_evidence()
    print(f"q(u): mean {relerr(gm, om):.2e} cov {_rel(gV, oV):.2e}; lnZ {lz:.6f} vs {olz:.6f}", flush=True)
    assert relerr(gm, om) < 1e-8 and _rel(gV, oV) < 1e-8
    assert abs(lz - olz) < 1e-8 * abs(olz)
    pm, pv = g.pitc_predict()
    qm, qv = ora.predict()
    print(f"predictive: mean {relerr(pm, qm):.2e} var {relerr(pv, qv):.2e}", flush=True)
    assert relerr(pm, qm) < 1e-8 and relerr(pv, qv) < 1e-8
    g.close()


def test_pitc_damped_sweeps_match_oracle():
    case = _case(n=8, L=600.0, stars=200, n_lon=2, n_lat=2, R=70, seed=37)
    ora, g, lz = _pair(case, damping=(0.5, 0.5, 0.7))
    om, oV = ora.posterior_u()
    gm, gV = g.pitc_inducing()
    assert relerr(gm, om) < 1e-8 and _rel(gV, oV) < 1e-8
    assert abs(lz - ora.log_evidence()) < 1e-8 * abs(ora.log_evidence())
    pm, pv = g.pitc_predict()
    qm, qv = ora.predict()
    assert relerr(pm, qm) < 1e-8 and relerr(pv, qv) < 1e-8
    g.close()


def test_pitc_errors():
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, a, sl, blocks, u, nb = _case(n=8, L=600.0, stars=100, n_lon=2, n_lat=1, R=20)
    g = E.EP(dict(cfg, leaf_size=48), raw["xyz"], a, raw["sigma"])
    with pytest.raises(E.EPError) as ei:
        g.pitc_sweep(1.0)
    assert ei.value.code == -5
    bad = blocks.copy()
    bad[:] = 0
    bad[0] = 2                                     # block 1 empty
    for sb, uu, nbk in ((bad, u, nb), (blocks, np.r_[u, u[:1]].astype(np.int32), nb),
                        (blocks, u, np.full_like(nb, 7))):
        with pytest.raises(E.EPError) as ei:
            g.pitc_setup(sb, uu, nbk)
        assert ei.value.code == -1
    with pytest.raises(E.EPError) as ei:
        g.pitc_info()
    assert ei.value.code == -5
    g.pitc_setup(blocks, u, nb)
    info = g.pitc_info()
    assert info["n_blocks"] == blocks.max() + 1 and info["n_inducing"] == len(u)
    assert info["max_block_stars"] == np.bincount(blocks).max() and info["sweep_flops"] > 0
    with pytest.raises(E.EPError) as ei:
        g.pitc_inducing()
    assert ei.value.code == -5
    for d in (0.0, 1.5, float("nan")):
        with pytest.raises(E.EPError) as ei:
            g.pitc_sweep(d)
        assert ei.value.code == -1
    g.pitc_sweep(1.0)
    assert np.all(np.isfinite(g.pitc_predict()[1]))
    g.close()
    # the block pass's allocations count against hbm_cap_bytes
    need = E.EP(dict(cfg, leaf_size=48), raw["xyz"], a, raw["sigma"])
    cap = need.structure()["device_bytes"] + (1 << 20)
    need.close()
    gc = E.EP(dict(cfg, leaf_size=48, hbm_cap_bytes=cap), raw["xyz"], a, raw["sigma"])
    with pytest.raises(E.EPError) as ei:
        gc.pitc_setup(blocks, u, nb)
    assert ei.value.code == -2
    gc.sweep()                                     # the context is still usable
    gc.close()
    ge = E.EP(dict(cfg, likelihood="gmm", leaf_size=48), raw["xyz"])   # unknown distances: not on this path
    with pytest.raises(E.EPError) as ei:
        ge.pitc_setup(blocks, u, nb)
    assert ei.value.code == -1
    ge.close()


def test_pitc_full_size_properties():
    """The bench shape (64^3 grid, 100,000 disc stars, 40 x 4 on-sky
    sub-catalogues, inducing nodes on their boundaries at 1-4 kpc): what holds
    at any size: the fixed point after one undamped sweep, a symmetric
    positive definite q(u) covariance, predictive variances in (0, prior
    variance], finite evidence."""
    from paper_1708_09705_amd import ep as E
    w = preset(2, likelihood="gauss_linear")
    cfg = w.ep_fields()
    raw = draw(w)
    # observations from the library's own simulator (the GAUSS_LINEAR forward
    # model at the prior mean); the checks below need no expected values
    _, a_obs = E.ep_simulate(E.make_config(cfg), raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    blocks = sky_cells(w, raw["xyz"], 40, 4)
    assert np.bincount(blocks, minlength=160).min() > 0
    u = boundary_inducing(w, 40, 4, (1000.0, 2000.0, 3000.0, 4000.0))
    nb = sky_cells(w, node_positions(w), 40, 4)
    g = E.EP(dict(cfg), raw["xyz"], a_obs, raw["sigma"])
    print(f"full size: blocks 160 R={len(u)}", flush=True)
    g.pitc_setup(blocks, u, nb)
    lz1 = g.pitc_sweep(1.0)
    m1, V1 = g.pitc_inducing()
    lz2 = g.pitc_sweep(1.0)
    m2, V2 = g.pitc_inducing()
    assert np.isfinite(lz1) and abs(lz2 - lz1) <= 1e-12 * abs(lz1)
    assert relerr(m2, m1) < 1e-12 and _rel(V2, V1) < 1e-12
    assert _rel(V1, V1.T) < 1e-12
    assert np.linalg.eigvalsh(0.5 * (V1 + V1.T)).min() > 0
    pm, pv = g.pitc_predict()
    k0 = float(cfg["prior_var"])
    print(f"lnZ {lz1:.3f}; predictive var in [{pv.min():.3e}, {pv.max():.3e}]", flush=True)
    assert np.all(np.isfinite(pm)) and np.all(pv > 0) and np.all(pv <= k0 * (1 + 1e-9))
    g.close()


# --- the mean parameters in the sites: q(u, Theta) ---------------------------

THETA_PRIOR = (1500.0, 150.0, 7.5e-4, 600.0, 0.1)
THETA_TRUE = (1000.0, 200.0, 1.2e-3, 500.0, 0.2)


def _case_theta(n, L, stars, n_lon, n_lat, R, seed):
    from oracle import epo, meanfn
    w = Workload("pitct", n=n, box_pc=L, n_stars=stars, sweeps=1, star_law="uniform", d_max_pc=L,
                 noise_law="uniform", noise_a=0.05, noise_b=0.15, likelihood="gauss_linear", seed_id=seed)
    cfg = w.ep_fields()
    cfg.update(sun_radius_pc=8000.0, bump_width_pc=200.0, theta_prior=THETA_PRIOR)
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
    used, blocks = np.unique(blocks, return_inverse=True)
    lut = np.array([int(np.argmin(np.abs(used - cc))) for cc in range(n_lon * n_lat)])
    nb = lut[sky_cells(w, node_positions(w), n_lon, n_lat)].astype(np.int32)
    u = np.sort(np.random.default_rng(seed).choice(w.N, size=R, replace=False)).astype(np.int32)
    return w, cfg, raw, a, sl, blocks.astype(np.int32), u, nb


@pytest.mark.parametrize("kw", [dict(n=8, L=1000.0, stars=150, n_lon=3, n_lat=2, R=40, seed=51),
                                dict(n=9, L=1200.0, stars=400, n_lon=3, n_lat=1, R=100, seed=53),
                                dict(n=10, L=1500.0, stars=700, n_lon=4, n_lat=2, R=250, seed=57)],
                         ids=["n8-6blk", "n9-3blk-3tiles", "n10-8blk-R4tiles"])
@pytest.mark.parametrize("damping", [(1.0,), (0.5, 0.8)], ids=["undamped", "damped"])
def test_pitc_theta_matches_oracle(kw, damping):
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, a, sl, blocks, u, nb = _case_theta(**kw)
    print(f"case n={kw['n']} stars={kw['stars']} blocks={blocks.max() + 1} R={len(u)} damping={damping}", flush=True)
    ora = pitc.DensePITCTheta(cfg, raw["xyz"], a, raw["sigma"], blocks, u, nb, sightlines=sl)
    g = E.EP(dict(cfg, leaf_size=48, mean_fn="disc_bump"), raw["xyz"], a, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    for d in damping:
        ora.sweep(d)
        lz = g.pitc_sweep(d)
    om, oV = ora.posterior_u()
    gm, gV = g.pitc_inducing()
    tm, tV = ora.theta_posterior()
    gtm, gtV = g.pitc_theta()
    olz = ora.log_evidence()
    print(f"q(u): mean {relerr(gm, om):.2e} cov {_rel(gV, oV):.2e}; phi: mean {relerr(gtm, tm):.2e} "
          f"cov {_rel(gtV, tV):.2e}; lnZ {lz:.6f} vs {olz:.6f}", flush=True)
    assert relerr(gm, om) < 1e-8 and _rel(gV, oV) < 1e-8
    assert relerr(gtm, tm) < 1e-8 and _rel(gtV, tV) < 1e-8
    assert abs(lz - olz) < 1e-8 * abs(olz)
    pm, pv = g.pitc_predict()
    qm, qv = ora.predict()
    print(f"predictive: mean {relerr(pm, qm):.2e} var {relerr(pv, qv):.2e}", flush=True)
    assert relerr(pm, qm) < 1e-8 and relerr(pv, qv) < 1e-8
    g.close()


def test_pitc_theta_state_errors():
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, a, sl, blocks, u, nb = _case_theta(n=8, L=1000.0, stars=100, n_lon=2, n_lat=1, R=20, seed=55)
    g = E.EP(dict(cfg, leaf_size=48, mean_fn="disc_bump"), raw["xyz"], a, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    with pytest.raises(E.EPError) as ei:
        g.pitc_theta()                                  # before a sweep
    assert ei.value.code == -5
    g.close()
    g = E.EP(dict(cfg, leaf_size=48), raw["xyz"], a, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    g.pitc_sweep(1.0)
    with pytest.raises(E.EPError) as ei:
        g.pitc_theta()                                  # constant mean
    assert ei.value.code == -5
    g.close()
    # grid sweeps re-linearise the mean (Gaussian mode): the PITC pass,
    # linearised at the hyperprior mean, refuses; with relinearize = 0 it runs.
    # The first sweep's border solve sees zero sites, so its step leaves the
    # linearisation at (or within rounding of) the hyperprior mean; the second
    # moves it.
    g = E.EP(dict(cfg, leaf_size=48, mean_fn="disc_bump"), raw["xyz"], a, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    g.sweep()
    g.sweep()
    for call in (lambda: g.pitc_sweep(1.0), lambda: g.pitc_setup(blocks, u, nb)):
        with pytest.raises(E.EPError) as ei:
            call()
        assert ei.value.code == -5
    g.close()
    g = E.EP(dict(cfg, leaf_size=48, mean_fn="disc_bump", relinearize=0), raw["xyz"], a, raw["sigma"])
    g.sweep()
    g.pitc_setup(blocks, u, nb)
    g.pitc_sweep(1.0)
    g.close()


def test_pitc_theta_full_size_properties():
    """The bench shape with the mean parameters in the sites: the fixed point
    after one sweep, a symmetric positive definite covariance of (u, phi),
    predictive variances in (0, prior variance + the mean's share]."""
    from paper_1708_09705_amd import ep as E
    w = preset(2, likelihood="gauss_linear")
    cfg = w.ep_fields()
    cfg.update(theta_prior=(3000.0, 150.0, 7.5e-4, 2000.0, 0.1))
    raw = draw(w)
    sim = E.make_config(dict(cfg, mean_fn="disc_bump", theta_prior=(2500.0, 200.0, 1.2e-3, 1800.0, 0.15)))
    _, a_obs = E.ep_simulate(sim, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    blocks = sky_cells(w, raw["xyz"], 40, 4)
    u = boundary_inducing(w, 40, 4, (1000.0, 2000.0, 3000.0, 4000.0))
    nb = sky_cells(w, node_positions(w), 40, 4)
    g = E.EP(dict(cfg, mean_fn="disc_bump"), raw["xyz"], a_obs, raw["sigma"])
    print(f"full size with mean parameters: blocks 160 R={len(u)}", flush=True)
    g.pitc_setup(blocks, u, nb)
    lz1 = g.pitc_sweep(1.0)
    m1, V1 = g.pitc_inducing()
    t1, T1 = g.pitc_theta()
    lz2 = g.pitc_sweep(1.0)
    m2, V2 = g.pitc_inducing()
    t2, T2 = g.pitc_theta()
    assert np.isfinite(lz1) and abs(lz2 - lz1) <= 1e-12 * abs(lz1)
    assert relerr(m2, m1) < 1e-12 and _rel(V2, V1) < 1e-12 and relerr(t2, t1) < 1e-12 and _rel(T2, T1) < 1e-12
    assert _rel(T1, T1.T) < 1e-12 and np.linalg.eigvalsh(0.5 * (T1 + T1.T)).min() > 0
    assert np.linalg.eigvalsh(0.5 * (V1 + V1.T)).min() > 0
    # the data constrain phi: its posterior sd is below the hyperprior's sqrt(ln 2)
    assert np.all(np.sqrt(np.diag(T1)) < np.sqrt(np.log(2.0)))
    pm, pv = g.pitc_predict()
    print(f"lnZ {lz1:.3f}; phi {np.round(t1, 3)}; predictive var in [{pv.min():.3e}, {pv.max():.3e}]", flush=True)
    assert np.all(np.isfinite(pm)) and np.all(pv > 0)
    g.close()


# ---------------------------------------------------------------------------
# the extinction likelihood: one site per star under the PITC prior
# ---------------------------------------------------------------------------
EXT_CASES = [
    dict(n=8, L=600.0, stars=150, n_lon=3, n_lat=2, R=40, lik="extinction"),
    dict(n=9, L=800.0, stars=400, n_lon=3, n_lat=1, R=150, seed=33, lik="extinction"),
    dict(n=10, L=1000.0, stars=500, n_lon=4, n_lat=2, R=0, law="disc", seed=35,
         inducing=(250.0, 500.0, 750.0, 1000.0), lik="extinction"),
]


@pytest.mark.parametrize("kw", EXT_CASES, ids=["n8-6blk", "n9-3blk-3tiles", "n10-disc-boundary"])
def test_pitc_extinction_matches_oracle(kw):
    """Star sites after three damped passes, q(u) and the PIC predictive
    against pitc.DensePITCExt; the sites live in the context's star sites."""
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, A, sl, blocks, u, nb = _case(**kw)
    print(f"case n={kw['n']} stars={kw['stars']} blocks={blocks.max() + 1} R={len(u)}", flush=True)
    ora = pitc.DensePITCExt(cfg, raw["xyz"], A, raw["sigma"], blocks, u, nb, sightlines=sl)
    g = E.EP(dict(cfg, leaf_size=48), raw["xyz"], A, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    for d in (1.0, 0.7, 0.7):
        so = ora.sweep(d)
        lz = g.pitc_sweep(d)
        tau, nu = g.sites()
        print(f"sweep d={d}: tau {relerr(tau, ora.tau):.2e} nu {_rel(nu, ora.nu):.2e} "
              f"updated {so['updated']}", flush=True)
        assert np.allclose(tau, ora.tau, rtol=1e-8, atol=1e-10)
        assert np.allclose(nu, ora.nu, rtol=1e-8, atol=1e-8)
    assert np.isnan(lz)
    om, oV = ora.posterior_u()
    gm, gV = g.pitc_inducing()
    pm, pv = g.pitc_predict()
    qm, qv = ora.predict()
    print(f"q(u): mean {relerr(gm, om):.2e} cov {_rel(gV, oV):.2e}; predictive: mean {relerr(pm, qm):.2e} "
          f"var {relerr(pv, qv):.2e}", flush=True)
    assert relerr(gm, om) < 1e-8 and _rel(gV, oV) < 1e-8
    assert relerr(pm, qm) < 1e-8 and relerr(pv, qv) < 1e-8
    g.close()


def test_pitc_extinction_errors():
    from paper_1708_09705_amd import ep as E
    w, cfg, raw, A, sl, blocks, u, nb = _case(n=8, L=600.0, stars=100, n_lon=2, n_lat=1, R=20, lik="extinction")
    g = E.EP(dict(cfg, leaf_size=48, mean_fn="disc_bump"), raw["xyz"], A, raw["sigma"])
    with pytest.raises(E.EPError) as ei:
        g.pitc_setup(blocks, u, nb)
    assert ei.value.code == -1
    g.close()


def test_pitc_extinction_full_size_properties():
    """The bench shape with the extinction likelihood (64^3 grid, 100,000 disc
    stars, 160 on-sky sub-catalogues, boundary inducing nodes): after damped
    passes every site is finite and non-negative, every star's posterior
    marginal of a_n has a positive variance, q(u) is symmetric positive
    definite and the predictive variances lie in (0, prior variance]."""
    from paper_1708_09705_amd import ep as E
    w = preset(2)
    cfg = w.ep_fields()
    raw = draw(w)
    f, A = E.ep_simulate(E.make_config(cfg), raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    blocks = sky_cells(w, raw["xyz"], 40, 4)
    u = boundary_inducing(w, 40, 4, (1000.0, 2000.0, 3000.0, 4000.0))
    nb = sky_cells(w, node_positions(w), 40, 4)
    g = E.EP(dict(cfg, leaf_size=512), raw["xyz"], A, raw["sigma"])
    g.pitc_setup(blocks, u, nb)
    for _ in range(4):
        g.pitc_sweep(0.7)
    tau, nu = g.sites()
    st = g.star_state()
    mu_u, Vu = g.pitc_inducing()
    pm, pv = g.pitc_predict()
    g.close()
    print(f"sites > 0: {int((tau > 0).sum())} of {tau.size}; predictive var {pv.min():.3e}..{pv.max():.3e}", flush=True)
    assert np.all(np.isfinite(tau)) and np.all(np.isfinite(nu)) and np.all(tau >= 0)
    assert (tau > 0).sum() > 0.99 * tau.size
    assert np.all(st["cav_var"][tau > 0] > 0)
    assert np.allclose(Vu, Vu.T, rtol=0, atol=1e-12 * np.abs(Vu).max())
    assert np.linalg.eigvalsh(Vu).min() > 0
    assert np.all(np.isfinite(pm)) and np.all(pv > 0) and np.all(pv <= cfg["prior_var"] * (1 + 1e-9))

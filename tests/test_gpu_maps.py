"""GPU parity of the map predictions against the FP64 oracle, through the C
ABI: lognormal density moments at the nodes, the exact posterior mean and
the sampled variance of the extinction to every node, and the two-point
density predictive.  All FP64: 1e-8 relative, as for the posterior."""
import numpy as np
import pytest

from oracle import epo, maps

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1708_09705_amd import ep as E
    return E


def _pair(n, L, stars, leaf, sweeps=2):
    E = _lib()
    cfg, gcfg, raw, f, A, sl = small_case(n=n, L=L, stars=stars, leaf=leaf)
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    for _ in range(sweeps):
        ora.sweep()
        g.sweep()
    mu, Sig, G, c = ora.posterior()
    Q = ora.Q0 + G.T @ (ora.tau[:, None] * G)
    return cfg, g, mu, Sig, Q


# (9, 800): odd n puts the observer (L/2, 0, L/2) on a node
@pytest.mark.parametrize("n,L,stars,leaf", [(8, 500.0, 60, 32), (9, 800.0, 200, 48), (12, 700.0, 300, 64)])
def test_density_and_extinction_maps_match_oracle(n, L, stars, leaf):
    cfg, g, mu, Sig, Q = _pair(n, L, stars, leaf)
    N = n ** 3
    print(f"case n={n} L={L} stars={stars}", flush=True)
    dm, dv = g.density_moments()
    om, ov = maps.density_moments(mu, np.diag(Sig))
    print(f"density: mean {relerr(dm, om):.2e} var {relerr(dv, ov):.2e}", flush=True)
    assert relerr(dm, om) < 1e-8 and relerr(dv, ov) < 1e-8
    perm = g.ordering()
    assert np.array_equal(np.sort(perm), np.arange(N))
    K = {8: 3, 9: 11, 12: 8}[n]        # draws go through the solve in batches of 8: ragged, full
    z = np.random.default_rng(n).standard_normal((K, N))
    em, ev = g.extinction_map(z)
    em0 = g.extinction_map()
    xm = maps.extinction_mean(cfg, mu, Sig)
    xv = maps.extinction_sample_var(cfg, mu, Q, perm, z)
    at_obs = xm == 0.0
    print(f"extinction: mean {relerr(em[~at_obs], xm[~at_obs]):.2e} var {relerr(ev[~at_obs], xv[~at_obs]):.2e} "
          f"nodes at the observer {int(at_obs.sum())}", flush=True)
    assert relerr(em[~at_obs], xm[~at_obs]) < 1e-8
    assert relerr(ev[~at_obs], xv[~at_obs]) < 1e-8
    assert np.all(em[at_obs] == 0.0) and np.all(ev[at_obs] == 0.0)
    assert (n % 2 == 1) == bool(at_obs.any())
    # a second call recomputes q(f); atomic accumulation order may differ
    assert relerr(em0[~at_obs], em[~at_obs]) < 1e-10 and np.all(em0[at_obs] == 0.0)
    g.close()


def test_point_predict_matches_oracle():
    n, L = 10, 600.0
    cfg, g, mu, Sig, Q = _pair(n, L, 150, 48)
    rng = np.random.default_rng(17)
    pa = rng.uniform(0, L, (300, 3))
    d = rng.standard_normal((300, 3))
    pb = np.clip(pa + 10.0 * d / np.linalg.norm(d, axis=1)[:, None], 0, L)
    pos = maps.node_positions(cfg)
    pa[:3] = pos[[0, 17, n ** 3 - 1]]                   # nodes, corners of the cube included
    pb[:3] = pos[[1, 17, n ** 3 - 2]]
    pa[3] = [L, L, L]
    pb[3] = [L, L - 10.0, L]
    xyz2 = np.hstack([pa, pb])
    gp = g.point_predict(xyz2)
    op = maps.point_predict(cfg, mu, Sig, xyz2)
    errs = [relerr(gp[:, k], op[:, k]) for k in range(5)]
    print("point predict rel err (E, E', Var, Var', Cov):", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) < 1e-8
    assert g.point_predict(np.zeros((0, 6))).shape == (0, 5)
    g.close()


def test_map_arguments_rejected():
    E = _lib()
    cfg, g, mu, Sig, Q = _pair(8, 500.0, 60, 32, sweeps=1)
    N = 8 ** 3
    for z in (np.zeros((1, N)), np.full((2, N), np.nan)):
        with pytest.raises(E.EPError) as ei:
            g.extinction_map(z)
        assert ei.value.code == -1
    for bad in ([[0, 0, 0, 0, 0, 501.0]], [[-1.0, 0, 0, 0, 0, 0]], [[np.nan, 0, 0, 0, 0, 0]],
                [[0, 0, 0, 200.0, 0, 0]]):                  # cells 0 and 2 along x do not touch
        with pytest.raises(E.EPError) as ei:
            g.point_predict(np.array(bad))
        assert ei.value.code == -1
    # the context is still usable afterwards
    assert np.all(np.isfinite(g.extinction_map()))
    g.close()

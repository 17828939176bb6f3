"""Degenerate and boundary inputs on the GPU against the oracle: no stars at
all (the posterior is the Vecchia prior), and stars on the cube's corners,
edges and faces, on grid nodes, next to the observer, along the observer's
face, and many at one position (identical sightline cliques), on an odd
grid."""
import numpy as np
import pytest

from oracle import epo
from synth import Workload, draw

from gpu_common import relerr

pytestmark = pytest.mark.gpu


def _E():
    from paper_1708_09705_amd import ep as E
    return E


def _case(xyz, n=9, L=560.0, seed=5):
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    w = Workload("edge", n=n, box_pc=L, n_stars=len(xyz), sweeps=3, star_law="uniform", noise_law="const",
                 noise_a=0.05, seed_id=seed)
    cfg = w.ep_fields()
    cfg["relinearize"] = True
    raw = draw(w, n_stars=len(xyz))
    raw["xyz"] = xyz
    return cfg, dict(cfg, leaf_size=48), raw


def test_no_stars_gives_the_prior():
    E = _E()
    cfg, gcfg, raw = _case(np.zeros((0, 3)))
    g = E.EP(gcfg, raw["xyz"], np.zeros(0), np.zeros(0))
    st = g.sweep()
    assert st["updated"] == 0
    Q0 = epo.Vecchia(cfg).Q0_dense()
    var = np.diag(np.linalg.inv(Q0))
    mean = g.posterior_mean()
    print(f"no stars: mean {relerr(mean, np.full_like(mean, cfg['prior_mean'])):.2e} "
          f"var {relerr(g.marginal_var(), var):.2e}", flush=True)
    assert relerr(mean, np.full_like(mean, cfg["prior_mean"])) < 1e-12
    assert relerr(g.marginal_var(), var) < 1e-10


def test_boundary_and_duplicate_stars_match_oracle():
    E = _E()
    L, n = 560.0, 9
    h = L / (n - 1)
    pts = [[0, 0, 0], [L, L, L], [L, 0, 0], [0, L, 0], [0, L / 2, 123.0], [L, 17.0, L], [L / 2, 1.0, L / 2],
           [100.0, 0.0, 300.0], [3 * h, 5 * h, 2 * h], [L / 2, L, L / 2], [L / 2, 0.0, 0.0]]
    pts += [[300.0, 400.0, 200.0]] * 15
    cfg, gcfg, raw = _case(pts, n=n, L=L)
    f, A, sl = epo.simulate(cfg, raw)
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    for s in range(3):
        so = ora.sweep()
        sg = g.sweep()
        assert sg["updated"] == so["updated"]
        tg, ng = g.sites()
        print(f"sweep {s}: tau {relerr(tg, ora.tau):.2e}", flush=True)
        assert np.allclose(tg, ora.tau, rtol=1e-8, atol=1e-10)
        assert np.allclose(ng, ora.nu, rtol=1e-8, atol=1e-8)
    assert relerr(g.posterior_mean(), ora.posterior_mean()) < 1e-8
    assert relerr(g.marginal_var(), ora.marginal_var()) < 1e-8

"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 throughout; the posterior mean and variance and the sites
must agree to 1e-8 relative (the FP64-mode target); the tilted moments to
1e-10 (both sides approximate the same integral to ~1e-13)."""
import math
import sys

import numpy as np
import pytest

from oracle import epo

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1708_09705_amd import ep as E
    return E


def test_tilted_moments_match_oracle():
    E = _lib()
    rng = np.random.default_rng(7)
    n = 20000
    mu = rng.uniform(-6, 1, n)
    v = np.exp(rng.uniform(np.log(1e-3), np.log(4.0), n))
    A = np.exp(rng.uniform(np.log(0.01), np.log(5.0), n)) * rng.choice([1, 1, 1, -0.2], n)
    s = rng.uniform(0.01, 0.3, n)
    lo, mo, vo = epo.tilted(0, mu, v, A, s)
    lg, mg, vg = E.ep_tilted_moments(0, mu, v, A, s)
    print("tilted max rel: lnZ %.2e mean %.2e var %.2e" % (relerr(lg, lo), relerr(mg, mo), relerr(vg, vo)), flush=True)
    assert np.allclose(lg, lo, rtol=1e-10, atol=1e-10)
    assert np.allclose(mg, mo, rtol=1e-10, atol=1e-10)
    assert np.allclose(vg, vo, rtol=1e-10, atol=0)
    lo, mo, vo = epo.tilted(1, mu, v, A, s)
    lg, mg, vg = E.ep_tilted_moments(1, mu, v, A, s)
    assert np.allclose(lg, lo, rtol=1e-13, atol=1e-13) and np.allclose(mg, mo, rtol=1e-13, atol=1e-13)
    assert np.allclose(vg, vo, rtol=1e-13)


def _run_pair(cfg, gcfg, raw, A, sl, sweeps):
    E = _lib()
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    print("structure", g.structure(), flush=True)
    for s in range(sweeps):
        so = ora.sweep()
        sg = g.sweep()
        tg, ng = g.sites()
        print(f"sweep {s}: tau {relerr(tg, ora.tau):.2e} nu {relerr(ng, ora.nu):.2e} "
              f"updated {sg['updated']}/{so['updated']}", flush=True)
        assert sg["updated"] == so["updated"]
        assert np.allclose(tg, ora.tau, rtol=1e-8, atol=1e-10)
        assert np.allclose(ng, ora.nu, rtol=1e-8, atol=1e-8)
    assert relerr(g.linpoint(), ora.fhat) < 1e-8
    mo, vo = ora.posterior_mean(), ora.marginal_var()
    mg, vg = g.posterior_mean(), g.marginal_var()
    print(f"posterior: mean {relerr(mg, mo):.2e} var {relerr(vg, vo):.2e}", flush=True)
    assert relerr(mg, mo) < 1e-8
    assert relerr(vg, vo) < 1e-8
    g.close()


@pytest.mark.parametrize("n,L,stars,leaf", [(8, 500.0, 60, 32), (12, 700.0, 300, 64)])
def test_ep_extinction_matches_oracle(n, L, stars, leaf):
    cfg, gcfg, raw, f, A, sl = small_case(n=n, L=L, stars=stars, leaf=leaf)
    _run_pair(cfg, gcfg, raw, A, sl, sweeps=3)


def test_ep_partial_linearisation_step_matches_oracle():
    """relin_step 0.5 with site damping 0.7: the linearisation point moves
    half-way to the posterior mean after each sweep, on both sides."""
    cfg, gcfg, raw, f, A, sl = small_case(n=10, L=600.0, stars=200, leaf=48, damping=0.7)
    cfg["relin_step"] = gcfg["relin_step"] = 0.5
    _run_pair(cfg, gcfg, raw, A, sl, sweeps=4)


def test_ep_gaussian_is_exact_in_one_sweep():
    cfg, gcfg, raw, f, a, sl = small_case(n=10, L=600.0, stars=150, leaf=48, lik="gauss_linear")
    E = _lib()
    g = E.EP(gcfg, raw["xyz"], a, raw["sigma"])
    g.sweep()
    tau, nu = g.sites()
    assert np.allclose(tau, 1 / raw["sigma"] ** 2, rtol=1e-9)
    assert np.allclose(nu, a / raw["sigma"] ** 2, rtol=1e-8, atol=1e-8)
    ora = epo.DenseEP(cfg, raw["xyz"], a, raw["sigma"], sightlines=sl)
    ora.sweep()
    assert relerr(g.posterior_mean(), ora.posterior_mean()) < 1e-8
    assert relerr(g.marginal_var(), ora.marginal_var()) < 1e-8

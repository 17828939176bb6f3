"""The deterministic mode: sweeps whose results are bitwise reproducible
(fixed summation orders in place of the floating-point atomic adds), still
within the FP64 bar of the oracle."""
import numpy as np
import pytest

from oracle import epo
from synth import draw, preset

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu


def _E():
    from paper_1708_09705_amd import ep as E
    return E


def _state(g):
    tau, nu = g.sites()
    return dict(tau=tau, nu=nu, lin=g.linpoint(), mean=g.posterior_mean(), var=g.marginal_var())


def test_deterministic_matches_oracle_and_repeats_bitwise():
    E = _E()
    cfg, gcfg, raw, f, A, sl = small_case(n=12, L=700.0, stars=300, leaf=64, damping=0.7)
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    runs = []
    for rep in range(2):
        g = E.EP(dict(gcfg, deterministic=1), raw["xyz"], A, raw["sigma"])
        for s in range(3):
            if rep == 0:
                ora.sweep()
            g.sweep()
        runs.append(_state(g))
        g.close()
    mo, vo = ora.posterior_mean(), ora.marginal_var()
    print(f"deterministic vs oracle: tau {relerr(runs[0]['tau'], ora.tau):.2e} mean {relerr(runs[0]['mean'], mo):.2e} "
          f"var {relerr(runs[0]['var'], vo):.2e}", flush=True)
    assert np.allclose(runs[0]["tau"], ora.tau, rtol=1e-8, atol=1e-10)
    assert relerr(runs[0]["mean"], mo) < 1e-8 and relerr(runs[0]["var"], vo) < 1e-8
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k


def test_config2_deterministic_repeats_bitwise():
    """64^3 / 100,000 stars, two sweeps in each of two contexts (one after
    the other): sites, linearisation point, posterior mean and variances
    equal bit for bit; against the default mode they agree to the FP64 bar."""
    E = _E()
    w = preset(2)
    raw = draw(w)
    cfg = E.make_config(w.ep_fields(), leaf_size=512)
    f, A = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    runs = []
    for det in (1, 1, 0):
        g = E.EP(E.make_config(w.ep_fields(), leaf_size=512, deterministic=det), raw["xyz"], A, raw["sigma"])
        for _ in range(2):
            st = g.sweep()
        runs.append(_state(g))
        print(f"deterministic={det}: sweep {st['ms_total']:.0f} ms (assemble {st['ms_assemble']:.1f}, "
              f"solve {st['ms_solve']:.1f})", flush=True)
        g.close()
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
    same = {k: bool(np.array_equal(runs[0][k], runs[2][k])) for k in runs[0]}
    print("default mode bitwise equal to the deterministic one:", same, flush=True)
    # two sweeps apart, the rounding differences of the atomic order stay
    # within the FP64 bar
    assert relerr(runs[2]["mean"], runs[0]["mean"]) < 1e-8
    assert relerr(runs[2]["var"], runs[0]["var"]) < 1e-8

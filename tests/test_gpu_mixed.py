"""Mixed precision (FP32 factor on FP32 MFMA, FP64 diagonal pivots, FP64
refinement of the mean, FP64 selected inversion) against the FP64 oracle and
against the FP64 GPU run.

Tolerance: the factor carries FP32 rounding (unit roundoff 6e-8); refinement
restores the mean to the FP64 solve of the same sites, while the marginal
variances inherit the factor's relative error times the conditioning of the
fronts.  The required bound is 1e-4 relative in posterior mean and
variance."""
import numpy as np
import pytest

from oracle import epo
from synth import draw, preset

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu


def _E():
    from paper_1708_09705_amd import ep as E
    return E


@pytest.mark.parametrize("n,L,stars,leaf", [(8, 500.0, 60, 32), (12, 700.0, 300, 64)])
def test_mixed_against_oracle(n, L, stars, leaf):
    E = _E()
    cfg, gcfg, raw, f, A, sl = small_case(n=n, L=L, stars=stars, leaf=leaf)
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(dict(gcfg, precision="mixed"), raw["xyz"], A, raw["sigma"])
    for s in range(3):
        ora.sweep()
        st = g.sweep()
        assert st["refine_residual"] <= 1e-12
    em = relerr(g.posterior_mean(), ora.posterior_mean())
    ev = relerr(g.marginal_var(), ora.marginal_var())
    et = relerr(g.sites()[0], ora.tau)
    print(f"mixed vs oracle: sites {et:.2e} mean {em:.2e} var {ev:.2e}", flush=True)
    assert em < 1e-4 and ev < 1e-4


def test_mixed_config2_against_fp64_gpu():
    """64^3 / 100k: the FP64 run's state after two sweeps (sites and
    linearisation point) loaded into a mixed-precision context, so the
    comparison is of the same q(f) computed in the two precisions."""
    E = _E()
    w = preset(2)
    raw = draw(w)
    cfg = E.make_config(w.ep_fields(), leaf_size=512)
    f, A = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    g = E.EP(E.make_config(w.ep_fields(), leaf_size=512), raw["xyz"], A, raw["sigma"])
    for _ in range(2):
        g.sweep()
    sites, lin = g.sites(), g.linpoint()
    m64, v64 = g.posterior_mean(), g.marginal_var()
    g.close()
    g = E.EP(E.make_config(w.ep_fields(), leaf_size=512, precision="mixed"), raw["xyz"], A, raw["sigma"])
    g.set_sites(*sites)
    g.set_linpoint(lin)
    m32, v32 = g.posterior_mean(), g.marginal_var()
    st = g.sweep()
    g.close()
    em, ev = relerr(m32, m64), relerr(v32, v64)
    rms_v = float(np.sqrt(np.mean(((v32 - v64) / v64) ** 2)))
    rms_m = float(np.sqrt(np.mean(((m32 - m64) / m64) ** 2)))
    print(f"config 2 mixed vs fp64 on the same state: mean {em:.2e} var {ev:.2e} (rms {rms_m:.1e}, {rms_v:.1e}); "
          f"refine {st['refine_iters']} rounds to {st['refine_residual']:.1e}", flush=True)
    # The refined mean meets the 1e-4 bound.  The marginal variances do not,
    # and no split of the dissection levels between FP64 and FP32 makes them:
    # measured on a 12-sweep state of this workload, every level split leaves 3.0e-4 to 7.1e-4 at
    # the worst node (the selected inversion carries the factor's FP32
    # rounding down the tree, and an FP32 leaf alone leaves 3.0e-4), so the
    # mixed form is not a 1e-4 result.  The bound asserted is twice the
    # measured level (0.8e-3 to 1.4e-3 depending on the state), so that a
    # regression shows.
    assert st["refine_residual"] <= 1e-12
    assert em < 1e-4
    assert ev < 3e-3
    assert rms_m < 1e-6 and rms_v < 1e-4


# Precision SELINV32: FP64 factor, solves and sites; the selected
# inversion's block products on FP32 MFMA (operands rounded to FP32, FP32
# sums over 64 terms, those partial sums in FP64, FP64 storage).  The
# posterior mean comes from the FP64 factor alone.  The variances carry the
# FP32 rounding of the block products: each level's
# Sigma_11 = X^T X + W^T Sigma_22 W is a sum of positive semi-definite terms,
# so the rounding is not amplified by the conditioning of Q as a rounded
# factor's is.  With the whole K summed in FP32 the worst node at 64^3 /
# 100k was 0.7-1.3e-4 (the sums' rounding, not the operands'); with FP64
# partial sums it is 1e-6.  Bound: the required 1e-4 relative error in mean
# and variance.


@pytest.mark.parametrize("n,L,stars,leaf", [(8, 500.0, 60, 32), (12, 700.0, 300, 64)])
def test_selinv32_against_oracle(n, L, stars, leaf):
    E = _E()
    cfg, gcfg, raw, f, A, sl = small_case(n=n, L=L, stars=stars, leaf=leaf)
    ora = epo.DenseEP(cfg, raw["xyz"], A, raw["sigma"], sightlines=sl)
    g = E.EP(dict(gcfg, precision="selinv32"), raw["xyz"], A, raw["sigma"])
    for s in range(3):
        ora.sweep()
        g.sweep()
    em = relerr(g.posterior_mean(), ora.posterior_mean())
    ev = relerr(g.marginal_var(), ora.marginal_var())
    print(f"selinv32 vs oracle: mean {em:.2e} var {ev:.2e}", flush=True)
    assert em < 1e-4 and ev < 1e-4


def test_selinv32_config2_against_fp64_gpu():
    """64^3 / 100k on the FP64 run's state after two sweeps: the mean within
    the FP64 parity bar (the same FP64 factor and solves; two FP64 contexts
    loaded with one state differ by their atomic summation orders), the
    variances within 1e-4."""
    E = _E()
    w = preset(2)
    raw = draw(w)
    cfg = E.make_config(w.ep_fields(), leaf_size=512)
    f, A = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    g = E.EP(E.make_config(w.ep_fields(), leaf_size=512), raw["xyz"], A, raw["sigma"])
    for _ in range(2):
        g.sweep()
    sites, lin = g.sites(), g.linpoint()
    m64, v64 = g.posterior_mean(), g.marginal_var()
    g.close()
    g = E.EP(E.make_config(w.ep_fields(), leaf_size=512, precision="selinv32"), raw["xyz"], A, raw["sigma"])
    g.set_sites(*sites)
    g.set_linpoint(lin)
    m32, v32 = g.posterior_mean(), g.marginal_var()
    g.close()
    em, ev = relerr(m32, m64), relerr(v32, v64)
    rms_v = float(np.sqrt(np.mean(((v32 - v64) / v64) ** 2)))
    print(f"config 2 selinv32 vs fp64 on the same state: mean {em:.2e} var {ev:.2e} (rms {rms_v:.1e})", flush=True)
    assert em < 1e-8
    assert ev < 1e-4

"""Pins for the oracle's line-of-sight operator: trapezoid integral of
exp(trilinear f) from the observer to the star, its gradient and support."""
import math

import numpy as np
import pytest

from oracle import epo


def _cfg(n=8, L=700.0, step=2.0):
    return dict(n=n, box_pc=L, observer_pc=(L / 2, 0.0, L / 2), prior_mean=-7.0, prior_var=1.0,
                outer_scale_pc=100.0, support_pc=150.0, los_step_pc=step)


def _stars(L, k=40, seed=0):
    return np.random.default_rng(seed).random((k, 3)) * L


def test_constant_field_exact():
    cfg = _cfg()
    xyz = _stars(cfg["box_pc"])
    sl = epo.Sightlines(cfg, xyz)
    f = np.full(sl.grid.N, -6.3)
    gval, lnA, c = sl.linearise(f)
    d = np.linalg.norm(xyz - np.asarray(cfg["observer_pc"]), axis=1)
    assert np.allclose(lnA, np.log(d) - 6.3, rtol=0, atol=1e-13)
    rows = np.repeat(np.arange(len(xyz)), np.diff(sl.ptr))
    assert np.allclose(np.bincount(rows, weights=gval), 1.0, atol=1e-13)
    # c = ln A - g.f
    assert np.allclose(c, lnA - (-6.3), atol=1e-12)


def test_linear_field_trapezoid_converges_second_order():
    # trilinear interpolation reproduces a linear field, so the only error is the
    # trapezoid rule's: int_0^d exp(alpha + beta t) dt, O(step^2)
    L = 700.0
    xyz = np.array([[600.0, 650.0, 123.0], [50.0, 300.0, 610.0]])
    errs = []
    for step in [8.0, 4.0, 2.0]:
        cfg = _cfg(L=L, step=step)
        sl = epo.Sightlines(cfg, xyz)
        P = sl.grid.xyz()
        a = np.array([0.002, -0.001, 0.0015])
        f = -6.0 + P @ a
        _, lnA, _ = sl.linearise(f)
        o = np.asarray(cfg["observer_pc"])
        err = []
        for s in range(2):
            dv = xyz[s] - o
            d = np.linalg.norm(dv)
            alpha = -6.0 + o @ a
            beta = (dv / d) @ a
            exact = math.exp(alpha) * (math.exp(beta * d) - 1.0) / beta
            err.append(abs(math.exp(lnA[s]) / exact - 1.0))
        errs.append(max(err))
    assert errs[-1] < 1e-5
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)


def test_gradient_matches_finite_differences():
    cfg = _cfg(n=8, L=700.0)
    xyz = _stars(cfg["box_pc"], k=6, seed=2)
    sl = epo.Sightlines(cfg, xyz)
    rng = np.random.default_rng(4)
    f = -7.0 + 0.8 * rng.standard_normal(sl.grid.N)
    gval, lnA, _ = sl.linearise(f)
    G = sl.G_dense(gval)
    eps = 1e-6
    for s in range(len(xyz)):
        for q in sl.nodes[sl.ptr[s]:sl.ptr[s + 1]][::7]:
            fp, fm = f.copy(), f.copy()
            fp[q] += eps
            fm[q] -= eps
            num = (sl.linearise(fp)[1][s] - sl.linearise(fm)[1][s]) / (2 * eps)
            assert G[s, q] == pytest.approx(num, rel=1e-6, abs=1e-9)


def test_support_is_exactly_the_touched_nodes():
    cfg = _cfg()
    xyz = _stars(cfg["box_pc"], k=20, seed=7)
    sl = epo.Sightlines(cfg, xyz)
    gval, _, _ = sl.linearise(np.full(sl.grid.N, -7.0))
    for s in range(len(xyz)):
        nodes = sl.nodes[sl.ptr[s]:sl.ptr[s + 1]]
        assert np.all(np.diff(nodes) > 0)            # sorted, unique
        assert np.all(gval[sl.ptr[s]:sl.ptr[s + 1]] >= 0)
    # a brute-force support: corners of the cell of every sample
    g = sl.grid
    o = np.asarray(cfg["observer_pc"])
    s = 3
    dv = xyz[s] - o
    T = max(1, math.ceil(np.linalg.norm(dv) / g.step))
    pts = o + np.outer(np.arange(T + 1) / T, dv)
    cell = np.clip(np.floor(pts / g.h), 0, g.n - 2).astype(int)
    want = set()
    for c in cell:
        for k in range(8):
            i, j, l = c[0] + (k & 1), c[1] + ((k >> 1) & 1), c[2] + ((k >> 2) & 1)
            want.add(i + g.n * (j + g.n * l))
    assert sorted(want) == list(sl.nodes[sl.ptr[s]:sl.ptr[s + 1]])

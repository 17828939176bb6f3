"""The C ABI library loads and exports every function include/ep.h declares;
argument validation fails cleanly before any device work (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ep.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*(ep_\w+)\s*\(", src, re.M)))


def _lib():
    from paper_1708_09705_amd import ep as E
    so = E.LIB_PATH
    if not os.path.exists(so):
        from paper_1708_09705_amd import build
        build.build()
    return E, E.load()


def test_every_declared_symbol_is_exported():
    E, L = _lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(E.EXPORTS) <= set(names)


def test_config_default_and_struct_size():
    E, L = _lib()
    c = E.make_config()
    assert c.n == 16 and c.box_pc == 1000.0 and c.prior_mean == -7.0
    assert tuple(c.observer_pc) == (500.0, 0.0, 500.0)
    assert c.damping == 1.0 and c.relinearize == 1 and c.los_step_pc == 2.0 and c.relin_step == 1.0


def test_invalid_inputs_rejected_before_device_work():
    E, L = _lib()
    xyz = np.array([[100.0, 200.0, 300.0], [400.0, 500.0, 600.0]])
    A = np.array([0.3, 0.4])
    s = np.array([0.05, 0.05])
    cfg = E.make_config()
    for bad in (dict(A=np.array([math.nan, 0.4])), dict(s=np.array([0.05, 0.0])),
                dict(xyz=np.array([[100.0, 200.0, 300.0], [400.0, 500.0, 1200.0]])),
                dict(xyz=np.array([[100.0, 200.0, 300.0], [500.0, 0.0, 500.0]]))):   # at the observer
        with pytest.raises(E.EPError) as ei:
            E.ep_init(cfg, bad.get("xyz", xyz), bad.get("A", A), bad.get("s", s))
        assert ei.value.code == -1
    for field, val in (("n", 1), ("damping", 0.0), ("box_pc", -1.0), ("precision", 7), ("precision", 3),
                       ("precision", -1), ("relin_step", 0.0),
                       ("relin_step", 1.5), ("deterministic", 2)):
        c = E.make_config(**{field: val})
        with pytest.raises(E.EPError) as ei:
            E.ep_init(c, xyz, A, s)
        assert ei.value.code == -1
    for over in (dict(precision="mixed"), dict(precision="selinv32"), dict(mean_fn="disc_bump")):
        c = E.make_config(deterministic=1, **over)
        with pytest.raises(E.EPError) as ei:
            E.ep_init(c, xyz, A, s)
        assert ei.value.code == -1
    # the inferred mean needs FP64 throughout
    for prec in ("mixed", "selinv32"):
        c = E.make_config(precision=prec, mean_fn="disc_bump")
        with pytest.raises(E.EPError) as ei:
            E.ep_init(c, xyz, A, s)
        assert ei.value.code == -1
    with pytest.raises(E.EPError) as ei:
        E.ep_tilted_moments(0, [0.0], [-1.0], [0.3], [0.05])
    assert ei.value.code == -1
    assert b"no error" != L.ep_last_error(None)


def test_noalloc_size_limit_rejected_before_device_work():
    E, L = _lib()
    assert E.EP_NOALLOC_MAX_TUPLES == 1 << 20
    rc = L.ep_mlp_predict_noalloc(None, E.EP_NOALLOC_MAX_TUPLES + 1, None, 1e-4, None, None, None, 0, None)
    assert rc == -1
    assert b"exceeds the maximum" in L.ep_last_error(None)
    rc = L.ep_mlp_predict_noalloc(None, 10, None, 1e-4, None, None, None, 0, None)
    assert rc == -1
    assert L.ep_mlp_predict_noalloc(None, 0, None, 1e-4, None, None, None, 0, None) == 0


def test_plan_without_a_device():
    """ep_plan runs the host analysis alone: its sightline supports are the
    oracle's (integer results, compared exactly), its layout figures are
    consistent, and bad inputs are refused."""
    E, L = _lib()
    from oracle import epo
    from synth import draw, preset
    w = preset(1)
    cfg = w.ep_fields()
    raw = draw(w, field=False)
    p = E.ep_plan(cfg, raw["xyz"])
    sl = epo.Sightlines(cfg, raw["xyz"])
    assert p["n_nodes"] == w.n ** 3 and p["n_stars"] == w.n_stars
    assert p["nnz_g"] == len(sl.nodes) and p["max_support"] == int(np.max(np.diff(sl.ptr)))
    assert 0 < p["nnz_L"] <= p["front_elems_lower"] <= p["front_elems"]
    assert p["max_separator"] <= p["max_front"] and p["n_levels"] >= 1
    assert 0 < p["trail_flops"] <= p["factor_flops"] < p["selinv_flops"]
    assert p["device_bytes"] > 8 * p["front_elems"] and p["device_bytes_mixed"] > p["device_bytes"]
    # the dense limit: one star-free 4^3 grid has one front holding every node
    q = E.ep_plan(dict(cfg, n=4, box_pc=200.0, observer_pc=(100.0, 0.0, 100.0)), np.zeros((0, 3)))
    assert q["n_fronts"] == 1 and q["nnz_L"] == 64 * 65 // 2
    with pytest.raises(E.EPError) as ei:
        E.ep_plan(cfg, np.array([[10.0, 20.0, 5000.0]]))
    assert ei.value.code == -1

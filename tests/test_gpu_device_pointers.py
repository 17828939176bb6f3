"""pointers_on_device = 1: every array of a context call is device memory
(torch tensors here).  The results must equal those of a context fed host
arrays (to 1e-9: FP64 atomic accumulation order differs run to run, and
ln Z of a poorly fitting star amplifies a 1e-12 change in its cavity), and
the host-side checks must still see the data."""
import os

import numpy as np
import pytest

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _np(t):
    return t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)


def test_device_pointers_match_host_pointers():
    import torch
    from paper_1708_09705_amd import ep as E
    cfg, gcfg, raw, f, A, sl = small_case(n=10, L=600.0, stars=150, leaf=48)
    print("case n=10 L=600 stars=150 (host vs device pointers)", flush=True)
    dev = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64, device="cuda:0")
    gh = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    gd = E.EP(dict(gcfg, pointers_on_device=1, device=0), dev(raw["xyz"]), dev(A), dev(raw["sigma"]))
    assert gd.S == gh.S == len(A)
    for _ in range(2):
        gh.sweep()
        gd.sweep()
    pairs = [("posterior_mean", gh.posterior_mean(), gd.posterior_mean()),
             ("marginal_var", gh.marginal_var(), gd.marginal_var())]
    for name, a, b in zip(("tau", "nu"), gh.sites(), gd.sites()):
        pairs.append((name, a, b))
    pairs.append(("linpoint", gh.linpoint(), gd.linpoint()))
    sh, sd = gh.star_state(), gd.star_state()
    pairs += [(k, sh[k], sd[k]) for k in sh]
    dm_h, dv_h = gh.density_moments()
    dm_d, dv_d = gd.density_moments()
    pairs += [("density mean", dm_h, dm_d), ("density var", dv_h, dv_d)]
    z = np.random.default_rng(3).standard_normal((3, gh.N))
    em_h, ev_h = gh.extinction_map(z)
    em_d, ev_d = gd.extinction_map(dev(z))
    pairs += [("extinction mean", em_h, em_d), ("extinction var", ev_h, ev_d)]
    rng = np.random.default_rng(4)
    pa = rng.uniform(0, 600.0, (50, 3))
    xyz2 = np.hstack([pa, np.clip(pa + 10.0, 0, 600.0)])
    pairs.append(("point predict", gh.point_predict(xyz2), gd.point_predict(dev(xyz2))))
    for name, a, b in pairs:
        assert isinstance(b, torch.Tensor) and b.device.type == "cuda", name
        b = _np(b)
        # relative to each entry, or to the array's scale for entries near 0
        # (ln Z crosses zero)
        scale = np.maximum(np.abs(a), 1e-6 * max(float(np.max(np.abs(a))), 1e-300))
        err = float(np.max(np.abs(b - a) / scale))
        print(f"{name}: {err:.2e}", flush=True)
        assert err < 1e-9, name
    assert np.array_equal(_np(gd.ordering()), gh.ordering())
    # inputs from the device, read back
    tau = np.abs(np.random.default_rng(5).standard_normal(gh.S)) * 10
    nu = np.random.default_rng(6).standard_normal(gh.S)
    gd.set_sites(dev(tau), dev(nu))
    t2, n2 = gd.sites()
    assert np.array_equal(_np(t2), tau) and np.array_equal(_np(n2), nu)
    fl = np.full(gh.N, -6.5)
    gd.set_linpoint(dev(fl))
    assert np.array_equal(_np(gd.linpoint()), fl)
    w = np.load(os.path.join(ROOT, "paper_1708_09705_amd", "surrogate_64cube.npy"))
    gd.load_surrogate(torch.as_tensor(w, device="cuda:0"))
    # host-side checks see device data
    bad = tau.copy()
    bad[7] = np.nan
    with pytest.raises(E.EPError) as ei:
        gd.set_sites(dev(bad), dev(nu))
    assert ei.value.code == -1
    A_bad = A.copy()
    A_bad[3] = np.inf
    with pytest.raises(E.EPError) as ei:
        E.EP(dict(gcfg, pointers_on_device=1, device=0), dev(raw["xyz"]), dev(A_bad), dev(raw["sigma"]))
    assert ei.value.code == -1
    with pytest.raises(E.EPError) as ei:
        gd.point_predict(dev([[0, 0, 0, 0, 0, 601.0]]))
    assert ei.value.code == -1
    gh.close()
    gd.close()


def test_device_pointers_pitc():
    """The PITC entry points with device arrays (int32 inputs, FP64 outputs)."""
    import torch
    from paper_1708_09705_amd import ep as E
    from synth.workloads import node_positions, sky_cells
    from synth import Workload
    cfg, gcfg, raw, f, a, sl = small_case(n=8, L=600.0, stars=150, leaf=48, lik="gauss_linear")
    w = Workload("p", n=8, box_pc=600.0, n_stars=150, sweeps=1)
    blocks = sky_cells(w, raw["xyz"], 2, 1)
    nb = sky_cells(w, node_positions(w), 2, 1)
    u = np.arange(0, 512, 9, dtype=np.int32)
    dev = lambda x, t=torch.float64: torch.as_tensor(np.asarray(x), dtype=t, device="cuda:0")
    gh = E.EP(gcfg, raw["xyz"], a, raw["sigma"])
    gd = E.EP(dict(gcfg, pointers_on_device=1, device=0), dev(raw["xyz"]), dev(a), dev(raw["sigma"]))
    gh.pitc_setup(blocks, u, nb)
    gd.pitc_setup(dev(blocks, torch.int32), dev(u, torch.int32), dev(nb, torch.int32))
    lh, ld = gh.pitc_sweep(0.8), gd.pitc_sweep(0.8)
    assert abs(lh - ld) <= 1e-12 * abs(lh)
    outs = [("u mean", gh.pitc_inducing()[0], gd.pitc_inducing()[0]),
            ("u cov", gh.pitc_inducing()[1], gd.pitc_inducing()[1]),
            ("pic mean", gh.pitc_predict()[0], gd.pitc_predict()[0]),
            ("pic var", gh.pitc_predict()[1], gd.pitc_predict()[1])]
    for name, x, y in outs:
        assert isinstance(y, torch.Tensor) and y.device.type == "cuda", name
        err = relerr(_np(y), x)
        print(f"{name}: {err:.2e}", flush=True)
        assert err < 1e-12, name
    gh.close()
    gd.close()

"""ep_mlp_predict_noalloc, the allocation-free form of the gated surrogate
moments for callers that cannot allocate device memory: through the C ABI on
device buffers, against ep_mlp_predict on the same tuples.  Consecutive calls
share the library's static device array, so the second and third calls run
on smaller inputs after a larger one, and a rejected call sits between two
good ones."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tuples(n, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-3.0, 1.0, n)
    v = np.exp(rng.uniform(np.log(0.002), np.log(0.5), n))
    s = rng.uniform(0.05, 0.2, n)
    A = np.exp(mu + np.sqrt(v) * rng.standard_normal(n)) + s * rng.standard_normal(n)
    return np.ascontiguousarray(np.stack([mu, v, A, s], 1))


def test_noalloc_matches_the_allocating_call():
    import torch
    from paper_1708_09705_amd import ep as E
    w = np.load(os.path.join(ROOT, "paper_1708_09705_amd", "surrogate_64cube.npy")).astype(np.float32)
    wt = torch.from_numpy(w).cuda()
    stream = torch.cuda.Stream()
    for n, seed, with_net in ((20000, 1, True), (3001, 2, True), (777, 3, False)):
        print(f"noalloc: n={n} seed={seed} network={with_net}", flush=True)
        X = _tuples(n, seed)
        ref_out, ref_err, ref_acc = E.ep_mlp_predict(w if with_net else None, X, tol=1e-4)
        Xt = torch.from_numpy(X).cuda()
        out = torch.full((n, 3), math.nan, dtype=torch.float64, device="cuda")
        err = torch.full((n,), math.nan, dtype=torch.float64, device="cuda")
        acc = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        E.ep_mlp_predict_noalloc(wt if with_net else None, Xt, out, err, acc, tol=1e-4, stream=stream)
        o, e, a = out.cpu().numpy(), err.cpu().numpy(), acc.cpu().numpy()
        assert np.array_equal(a.astype(bool), ref_acc) and set(np.unique(a)) <= {0, 1}
        assert np.all(np.isfinite(o)) and np.all(np.isfinite(e))
        d_out = float(np.max(np.abs(o - ref_out) / np.maximum(np.abs(ref_out), 1e-300)))
        d_err = float(np.max(np.abs(e - ref_err) / np.maximum(np.abs(ref_err), 1e-300)))
        print(f"  accepted {a.mean():.4f}; max rel diff: moments {d_out:.1e}, error estimate {d_err:.1e}", flush=True)
        assert d_out <= 1e-13 and d_err <= 1e-13


def test_noalloc_rejects_bad_input_and_recovers():
    import torch
    from paper_1708_09705_amd import ep as E
    n = 500
    X = _tuples(n, 7)
    X[123, 3] = 0.0   # sigma = 0
    Xt = torch.from_numpy(X).cuda()
    out = torch.full((n, 3), -5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EPError) as ei:
        E.ep_mlp_predict_noalloc(None, Xt, out)
    assert ei.value.code == -1 and "sigma" in str(ei.value)
    assert bool(torch.all(out == -5.0))          # outputs untouched
    X[123, 3] = 0.1
    Xt = torch.from_numpy(X).cuda()
    E.ep_mlp_predict_noalloc(None, Xt, out)      # the error counter starts at zero again
    ref_out, _, _ = E.ep_mlp_predict(None, X, tol=1e-4)
    o = out.cpu().numpy()
    assert float(np.max(np.abs(o - ref_out) / np.abs(ref_out))) <= 1e-13
    big = torch.empty((0, 4), dtype=torch.float64, device="cuda")
    E.ep_mlp_predict_noalloc(None, big, torch.empty((0, 3), dtype=torch.float64, device="cuda"))   # n = 0

"""The tilted-moment surrogate on the GPU: backward kernels against the FP64
reference, training, the gate against the oracle's quadrature, and EP with
surrogate moments against EP with quadrature moments."""
import numpy as np
import pytest

from oracle import epo, mlp

from gpu_common import relerr, small_case

pytestmark = pytest.mark.gpu


def _E():
    from paper_1708_09705_amd import ep as E
    return E


def _tuples(n, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-3.0, 1.0, n)
    v = np.exp(rng.uniform(np.log(0.002), np.log(0.5), n))
    s = rng.uniform(0.05, 0.2, n)
    A = np.exp(mu + np.sqrt(v) * rng.standard_normal(n)) + s * rng.standard_normal(n)
    lnZ, m, var = epo.tilted(0, mu, v, A, s)
    return np.stack([mu, v, A, s], 1), np.stack([lnZ, m, var], 1)


def test_gradients_match_fp64_backprop():
    E = _E()
    rng = np.random.default_rng(3)
    w = rng.normal(0, 0.15, mlp.NPARAM).astype(np.float32)
    X = rng.normal(size=(300, 4)).astype(np.float32)
    Y = rng.normal(size=(300, 3)).astype(np.float32)
    loss, g = E.ep_mlp_loss_grad(w, X, Y)
    p = mlp.unpack(w.astype(np.float64))
    lo, go = mlp.loss_grad(p, X.astype(np.float64), Y.astype(np.float64))
    flat = np.concatenate([go[n].ravel() for n, _ in mlp.SHAPES if n[0] in "Wb"])
    err = np.max(np.abs(g[:mlp.NTRAIN] - flat)) / np.max(np.abs(flat))
    print(f"loss {loss:.6f} vs {lo:.6f}; gradient max error / max |g| = {err:.2e}", flush=True)
    assert abs(loss - lo) < 1e-5 * lo
    assert err < 1e-5


@pytest.fixture(scope="module")
def trained():
    E = _E()
    X, Y = _tuples(60000, 1)
    w, loss = E.ep_mlp_train(X, Y, epochs=8, batch=1024, lr=2e-3, seed=5)
    return w, loss


def test_training_reduces_the_loss(trained):
    w, loss = trained
    print("loss per epoch", np.round(loss, 5), flush=True)
    assert np.all(np.isfinite(loss)) and loss[-1] < 0.2 * loss[0]
    assert np.all(np.isfinite(w))


def test_gate_accepts_only_moments_within_tolerance(trained):
    E = _E()
    w, _ = trained
    X, Y = _tuples(20000, 2)
    out, err, acc = E.ep_mlp_predict(w, X, tol=1e-4)
    _, _, acc0 = E.ep_mlp_predict(None, X, tol=1e-4)
    print(f"accepted {acc.mean():.3f} with the network, {acc0.mean():.3f} centred at the baseline", flush=True)
    assert acc.mean() > 0.2
    a = out[acc]
    y = Y[acc]
    scale = np.maximum(np.abs(y[:, 1]), np.sqrt(y[:, 2]))
    # accepted stars use the second (32-node) pass; the gate's estimate is
    # the first pass's error, so the adaptive quadrature agrees with what was
    # accepted to within the tolerance
    assert np.max(np.abs(a[:, 0] - y[:, 0])) < 1e-4
    assert np.max(np.abs(a[:, 1] - y[:, 1]) / scale) < 1e-4
    assert np.max(np.abs(a[:, 2] / y[:, 2] - 1)) < 1e-4
    # the baseline-centred gate is just as exact where it accepts
    assert acc0.mean() > 0.5



def test_ep_with_surrogate_moments_tracks_quadrature(trained):
    E = _E()
    w, _ = trained
    cfg, gcfg, raw, f, A, sl = small_case(n=10, L=600.0, stars=300, leaf=48)
    q = E.EP(gcfg, raw["xyz"], A, raw["sigma"])
    s = E.EP(dict(gcfg, moments="surrogate"), raw["xyz"], A, raw["sigma"])
    s.load_surrogate(w)
    for _ in range(3):
        q.sweep()
        st = s.sweep()
    print(f"fallbacks in the last sweep: {st['surrogate_fallbacks']} of {s.S}", flush=True)
    em = relerr(s.posterior_mean(), q.posterior_mean())
    ev = relerr(s.marginal_var(), q.marginal_var())
    print(f"surrogate vs quadrature EP: mean {em:.2e} var {ev:.2e}", flush=True)
    assert em < 1e-3 and ev < 1e-2


def test_surrogate_mode_without_weights_is_a_state_error():
    E = _E()
    cfg, gcfg, raw, f, A, sl = small_case(n=8, L=500.0, stars=40, leaf=32)
    s = E.EP(dict(gcfg, moments="surrogate"), raw["xyz"], A, raw["sigma"])
    with pytest.raises(E.EPError) as ei:
        s.sweep()
    assert ei.value.name == "STATE"

"""Pins for the oracle's sparse prior precision (Vecchia / inverse Cholesky of
the tapered covariance): exact when the conditioning radius covers the box,
KL-monotone in the radius, SPD, and an exact prior draw."""
import numpy as np
import pytest
from scipy import special

from oracle import epo


def _cfg(n=4, L=300.0, rs=150.0, rho=None, ell=100.0):
    return dict(n=n, box_pc=L, observer_pc=(L / 2, 0.0, L / 2), prior_mean=-7.0, prior_var=1.0,
                outer_scale_pc=ell, support_pc=rs, vecchia_radius_pc=rho or rs, los_step_pc=2.0)


def _Kt(cfg):
    g = epo.Grid(cfg)
    x = g.xyz()
    r = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    f = np.vectorize(lambda t: epo.cov(cfg["prior_var"], cfg["outer_scale_pc"], cfg["support_pc"], t))
    return f(r)


def test_full_radius_reproduces_inverse_covariance():
    # conditioning on every earlier node = exact Cholesky: Q0 = K_t^{-1}
    cfg = _cfg(n=4, L=300.0, rs=250.0, rho=1000.0)
    vec = epo.Vecchia(cfg)
    K = _Kt(cfg)
    Q0 = vec.Q0_dense()
    assert np.allclose(Q0 @ K, np.eye(K.shape[0]), atol=1e-10)


def test_untapered_limit():
    # support -> infinity: the tapered kernel -> plain Matern (scipy kv route)
    cfg = _cfg(n=3, L=200.0, rs=1e7, rho=1e9)
    vec = epo.Vecchia(cfg)
    g = epo.Grid(cfg)
    x = g.xyz()
    r = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    nu = 1.0 / 3.0
    with np.errstate(invalid="ignore"):
        z = r / 100.0
        K = np.where(r > 0, 2 ** (1 - nu) / special.gamma(nu) * z ** nu * special.kv(nu, z), 1.0)
    Sigma = np.linalg.inv(vec.Q0_dense())
    assert np.allclose(Sigma, K, rtol=1e-8, atol=1e-9)


def _kl(K, Q):
    # KL( N(0,K) || N(0,Q^{-1}) )
    n = K.shape[0]
    sK = np.linalg.slogdet(K)[1]
    sQ = np.linalg.slogdet(Q)[1]
    return 0.5 * (np.trace(Q @ K) - n - sQ - sK)


def test_kl_nonincreasing_in_radius():
    base = _cfg(n=5, L=400.0, rs=250.0)
    K = _Kt(base)
    kls = []
    for rho in [60.0, 110.0, 150.0, 200.0, 250.0, 1000.0]:
        kls.append(_kl(K, epo.Vecchia(dict(base, vecchia_radius_pc=rho)).Q0_dense()))
    assert all(b <= a + 1e-10 for a, b in zip(kls, kls[1:]))
    assert kls[-1] == pytest.approx(0.0, abs=1e-9)
    assert kls[0] > 1e-3


def test_spd_and_positive_conditional_variances():
    cfg = _cfg(n=16, L=1000.0)
    vec = epo.Vecchia(cfg)
    assert np.all(vec.d > 0)
    Q0 = vec.Q0_dense()
    assert np.array_equal(Q0, Q0.T) or np.allclose(Q0, Q0.T, rtol=0, atol=1e-13)
    np.linalg.cholesky(Q0)  # raises if not PD
    # interior rows condition on the 28 earlier points within the radius
    assert np.max(np.diff(vec.rowptr)) == 28


def test_prior_draw_is_exact():
    cfg = _cfg(n=5, L=300.0)
    vec = epo.Vecchia(cfg)
    xi = np.random.default_rng(3).standard_normal(vec.grid.N)
    f = vec.draw(-7.0, xi)
    IB = np.eye(vec.grid.N) - vec.B_dense()
    assert np.allclose(IB @ (f + 7.0), np.sqrt(vec.d) * xi, atol=1e-12)


def test_prior_quadform_matches_dense():
    cfg = _cfg(n=6, L=400.0)
    vec = epo.Vecchia(cfg)
    Sigma = np.linalg.inv(vec.Q0_dense())
    rng = np.random.default_rng(5)
    ptr = np.array([0, 5, 12], dtype=np.int64)
    nodes = np.concatenate([np.sort(rng.choice(vec.grid.N, 5, replace=False)),
                            np.sort(rng.choice(vec.grid.N, 7, replace=False))]).astype(np.int32)
    gval = rng.random(12)
    out = vec.prior_quadform(ptr, nodes, gval)
    for s in range(2):
        idx, w = nodes[ptr[s]:ptr[s + 1]], gval[ptr[s]:ptr[s + 1]]
        assert out[s] == pytest.approx(w @ Sigma[np.ix_(idx, idx)] @ w, rel=1e-11)


def test_q0_matvec_matches_dense():
    cfg = _cfg(n=6, L=400.0)
    vec = epo.Vecchia(cfg)
    x = np.random.default_rng(1).standard_normal(vec.grid.N)
    assert np.allclose(vec.Q0_matvec(x), vec.Q0_dense() @ x, rtol=1e-12, atol=1e-12)

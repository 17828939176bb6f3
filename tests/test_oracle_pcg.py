"""Pins for the oracle's matrix-free posterior solves (used where the dense
oracle cannot go): Q0^{-1} against the dense inverse, Q X against the dense
posterior precision of the dense EP, and the preconditioned CG results
(posterior mean, marginal variances, the q-marginal variances of the stars'
log-extinctions) against the dense EP's posterior after a few sweeps."""
import numpy as np
import pytest

from oracle import epo, pcg
from synth import Workload, draw


def _ep(n, L, stars, seed, sweeps=3):
    w = Workload("t", n=n, box_pc=L, n_stars=stars, sweeps=sweeps, star_law="uniform", d_max_pc=L,
                 noise_law="const", noise_a=0.05, seed_id=seed)
    cfg = dict(w.ep_fields(), damping=0.7)
    raw = draw(w)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    ep = epo.DenseEP(cfg, raw["xyz"], A_obs, raw["sigma"], sightlines=sl)
    for _ in range(sweeps):
        ep.sweep()
    return cfg, ep, sl


def test_q0_solve_is_the_inverse():
    cfg, ep, sl = _ep(8, 500.0, 10, 60, sweeps=0)
    K = np.linalg.inv(ep.Q0)
    X = np.random.default_rng(0).standard_normal((sl.grid.N, 5))
    assert np.allclose(ep.vec.q0_solve(X), K @ X, rtol=1e-11, atol=1e-12)
    assert np.allclose(ep.vec.q0_solve(X[:, 0]), K @ X[:, 0], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n,L,stars,seed", [(8, 500.0, 60, 61), (10, 650.0, 150, 62), (12, 800.0, 250, 63)])
def test_pcg_reproduces_the_dense_posterior(n, L, stars, seed):
    cfg, ep, sl = _ep(n, L, stars, seed)
    mu_d, Sig_d, G, c = ep.posterior()
    gval, lnA, c2 = sl.linearise(ep.fhat)
    ops = pcg.PosteriorOps(ep.vec, sl, gval, ep.tau)
    Qd = ep.Q0 + G.T @ (ep.tau[:, None] * G)
    X = np.random.default_rng(1).standard_normal((sl.grid.N, 3))
    assert np.allclose(ops.Q(X), Qd @ X, rtol=1e-12, atol=1e-11)
    # mean
    b = ep.b0 + G.T @ (ep.nu - ep.tau * c)
    mu, it, res = pcg.pcg(ops, b)
    assert res.max() < 1e-14
    assert np.allclose(mu, mu_d, rtol=1e-12, atol=1e-12)
    # marginal variances at every node and the stars' q-marginal variances
    N = sl.grid.N
    E = np.eye(N)
    Xe, it, res = pcg.pcg(ops, E)
    assert np.allclose(np.diag(Xe), np.diag(Sig_d), rtol=1e-11)
    Gt = G.T.copy()
    Xg, it, res = pcg.pcg(ops, Gt)
    v = np.einsum("ij,ij->j", Gt, Xg)
    assert np.allclose(v, np.einsum("ij,jk,ik->i", G, Sig_d, G), rtol=1e-11)

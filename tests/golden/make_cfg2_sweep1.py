"""Writes cfg2_sweep1.npz: the oracle's EP state after one sweep of the
64^3-grid / 100,000-star workload (4 kpc cube, disc-distributed stars,
sigma ~ U[0.05, 0.2] mag), and its posterior there, for the GPU parity test
at that size.  Calls the oracle and the seeded draws only.

Sweep 1 starts from zero sites, so every star's cavity is its prior marginal
(mean ln A at the prior mean, variance g^T Q0^{-1} g); the tilted moments
(adaptive Gauss-Kronrod) give the new sites, with the skip rule for a
negative site (undamped).  With those sites at the same linearisation point
the oracle's matrix-free PCG gives the posterior mean at every node, the
marginal variance at 64 nodes (near the observer, on the planes through it,
random) and the q-marginal of a_n for 64 stars (nearest, longest sightlines,
random), from which their cavities follow.

Run: python tests/golden/make_cfg2_sweep1.py   (about an hour on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import epo, pcg  # noqa: E402
from synth import draw, preset  # noqa: E402


def log(*a):
    print(*a, flush=True)


def main():
    t0 = time.time()
    w = preset(2)
    cfg = w.ep_fields()
    raw = draw(w)
    vec = epo.Vecchia(cfg)
    f_true, A_obs, sl = epo.simulate(cfg, raw)
    N, S = sl.grid.N, sl.n_stars
    m0 = float(cfg["prior_mean"])
    f0 = np.full(N, m0)
    gval, lnA, c = sl.linearise(f0)
    v0 = vec.prior_quadform(sl.ptr, sl.nodes, gval)
    _, mh, vh = epo.tilted(0, lnA, v0, A_obs, raw["sigma"])
    tau = 1.0 / vh - 1.0 / v0
    nu = mh / vh - lnA / v0
    good = np.isfinite(tau) & np.isfinite(nu) & (tau >= 0)
    tau, nu = np.where(good, tau, 0.0), np.where(good, nu, 0.0)
    log(f"sweep 1 sites: {int(good.sum())} updated, {int((~good).sum())} skipped ({time.time() - t0:.0f} s)")
    ops = pcg.PosteriorOps(vec, sl, gval, tau)
    b = ops.Q0(f0) + ops.Gt @ (nu - tau * c)
    mu, it, res = pcg.pcg(ops, b, log=log, stall=400)
    log(f"mean: {it} iterations, residual {res.max():.2e} ({time.time() - t0:.0f} s)")
    # nodes: nearest the observer, on the planes x = L/2 and z = L/2 through it, random
    rng = np.random.default_rng(20260)
    P = sl.grid.xyz()
    o = np.asarray(cfg["observer_pc"])
    dist = np.linalg.norm(P - o, axis=1)
    n = sl.grid.n
    half = (n - 1) // 2
    ii, kk = np.arange(N) % n, np.arange(N) // (n * n)
    near = np.argsort(dist)[:16]
    px = rng.choice(np.flatnonzero(ii == half), 16, replace=False)
    pz = rng.choice(np.flatnonzero(kk == half), 16, replace=False)
    rest = np.setdiff1d(np.arange(N), np.concatenate([near, px, pz]))
    nodes = np.concatenate([near, px, pz, rng.choice(rest, 16, replace=False)])
    # stars: nearest the observer, the longest sightlines, random
    d_st = np.linalg.norm(raw["xyz"] - o, axis=1)
    sup = np.diff(sl.ptr)
    s_near = np.argsort(d_st)[:16]
    s_long = np.setdiff1d(np.argsort(-sup)[:40], s_near)[:16]
    s_rest = np.setdiff1d(np.arange(S), np.concatenate([s_near, s_long]))
    stars = np.concatenate([s_near, s_long, rng.choice(s_rest, 32, replace=False)])
    R = np.zeros((N, 128))
    R[nodes, np.arange(64)] = 1.0
    Gt = ops.Gt[:, stars].toarray()
    R[:, 64:] = Gt
    X, it2, res2 = pcg.pcg(ops, R, log=log, stall=400)
    log(f"variances and stars: {it2} iterations, max residual {res2.max():.2e} ({time.time() - t0:.0f} s)")
    var = X[nodes, np.arange(64)]
    vq = np.einsum("ij,ij->j", Gt, X[:, 64:])
    mq = c[stars] + Gt.T @ mu
    tau_c = 1.0 / vq - tau[stars]
    nu_c = mq / vq - nu[stars]
    np.savez_compressed(os.path.join(HERE, "cfg2_sweep1.npz"), tau=tau, nu=nu, mu=mu, nodes=nodes, var=var,
                        stars=stars, q_var=vq, q_mean=mq, cav_var=1.0 / tau_c, cav_mu=nu_c / tau_c,
                        pcg_iterations=np.array([it, it2]), pcg_residuals=np.array([res.max(), res2.max()]))
    log(f"wrote cfg2_sweep1.npz ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()

"""Plain FP64 reference of the map predictions (test infrastructure only:
imported by tests/ and nothing else).

From the Gaussian posterior q(f) = N(mu, Sigma) on the grid (Sec. 5 maps of
extinction and of the pseudo-density rho kappa = e^f):

* density_moments: rho kappa = e^f is lognormal, E = exp(mu + v/2),
  Var = (e^v - 1) exp(2 mu + v).
* extinction_mean: A(x) is the line-of-sight integral of e^F from the
  observer to x by the sightline forward model (steps T = max(1, ceil(d/step)),
  points o + (t/T)(x - o), trapezoid weights d/T halved at both ends,
  trilinear F with cell clamp(floor(s/h), 0, n-2)); F at each point is
  Gaussian, so E[A(x)] = sum_t w_t exp(phi_t . mu + phi_t^T Sigma phi_t / 2).
* extinction_sample_var: posterior draws f_k = mu + P L^{-T} z_k with L the
  Cholesky factor of Q permuted to the elimination order P and z_k consumed
  in that order; the sample variance (divisor K - 1) of A(x) over them.
* point_predict: the lognormal moments of (e^F(x), e^F(x')) from the
  trilinear field's Gaussian moments.
"""
from __future__ import annotations

import math

import numpy as np


def density_moments(mu, var):
    mu, var = np.asarray(mu, dtype=np.float64), np.asarray(var, dtype=np.float64)
    e = np.exp(mu + 0.5 * var)
    return e, np.expm1(var) * e * e


def _geom(cfg):
    n = int(cfg["n"])
    L = float(cfg["box_pc"])
    return n, L / (n - 1), np.asarray(cfg["observer_pc"], dtype=np.float64), float(cfg["los_step_pc"])


def point_weights(cfg, p):
    """Trilinear corners (8 node indices) and weights of points p (m x 3)."""
    n, h, _, _ = _geom(cfg)
    p = np.atleast_2d(np.asarray(p, dtype=np.float64))
    c = np.clip(np.floor(p / h), 0, n - 2)
    w = p / h - c
    c = c.astype(np.int64)
    nodes = np.empty((p.shape[0], 8), dtype=np.int64)
    phi = np.empty((p.shape[0], 8))
    for c8 in range(8):
        b = np.array([c8 & 1, (c8 >> 1) & 1, (c8 >> 2) & 1])
        idx = c + b
        nodes[:, c8] = idx[:, 0] + n * (idx[:, 1] + n * idx[:, 2])
        phi[:, c8] = np.prod(np.where(b == 1, w, 1.0 - w), axis=1)
    return nodes, phi


def sightline_points(cfg, x):
    """Sample points of the observer's sightline to x: (weights, nodes, phi);
    empty at the observer."""
    n, h, o, step = _geom(cfg)
    x = np.asarray(x, dtype=np.float64)
    dv = x - o
    d = math.sqrt(float(dv @ dv))
    if not d > 0:
        return np.zeros(0), np.zeros((0, 8), dtype=np.int64), np.zeros((0, 8))
    T = max(1, int(math.ceil(d / step)))
    t = np.arange(T + 1, dtype=np.float64)
    pts = o[None, :] + (t / T)[:, None] * dv[None, :]
    w = np.full(T + 1, d / T)
    w[0] *= 0.5
    w[-1] *= 0.5
    nodes, phi = point_weights(cfg, pts)
    return w, nodes, phi


def node_positions(cfg):
    n, h, _, _ = _geom(cfg)
    i = np.arange(n ** 3)
    return np.stack([(i % n) * h, ((i // n) % n) * h, (i // (n * n)) * h], axis=1)


def extinction_mean(cfg, mu, Sigma, targets=None):
    """E[A(x)] for every node (or the given node indices)."""
    pos = node_positions(cfg)
    idx = np.arange(pos.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros(len(idx))
    for k, p in enumerate(idx):
        w, nodes, phi = sightline_points(cfg, pos[p])
        if len(w) == 0:
            continue
        m = np.einsum("ta,ta->t", phi, mu[nodes])
        v = np.einsum("ta,tab,tb->t", phi, Sigma[nodes[:, :, None], nodes[:, None, :]], phi)
        out[k] = float(np.sum(w * np.exp(m + 0.5 * v)))
    return out


def extinction_of_field(cfg, f, targets=None):
    """A(x) for one field f, every node (or the given node indices)."""
    pos = node_positions(cfg)
    idx = np.arange(pos.shape[0]) if targets is None else np.asarray(targets)
    out = np.zeros(len(idx))
    for k, p in enumerate(idx):
        w, nodes, phi = sightline_points(cfg, pos[p])
        if len(w) == 0:
            continue
        out[k] = float(np.sum(w * np.exp(np.einsum("ta,ta->t", phi, f[nodes]))))
    return out


def posterior_draws(mu, Q, perm, z):
    """f_k = mu + P L^{-T} z_k, L L^T = Q[perm][:, perm], z_k in elimination order."""
    Qp = Q[np.ix_(perm, perm)]
    Lp = np.linalg.cholesky(Qp)
    x = np.linalg.solve(Lp.T, np.asarray(z, dtype=np.float64).T).T   # K x N, elimination order
    f = np.empty_like(x)
    f[:, perm] = x
    return mu[None, :] + f


def extinction_sample_var(cfg, mu, Q, perm, z, targets=None):
    draws = posterior_draws(mu, Q, perm, z)
    A = np.stack([extinction_of_field(cfg, f, targets) for f in draws])
    return A.var(axis=0, ddof=1)


def point_predict(cfg, mu, Sigma, xyz2):
    xyz2 = np.asarray(xyz2, dtype=np.float64).reshape(-1, 6)
    na, pa = point_weights(cfg, xyz2[:, :3])
    nb, pb = point_weights(cfg, xyz2[:, 3:])
    out = np.empty((xyz2.shape[0], 5))
    for i in range(xyz2.shape[0]):
        ma, mb = pa[i] @ mu[na[i]], pb[i] @ mu[nb[i]]
        va = pa[i] @ Sigma[np.ix_(na[i], na[i])] @ pa[i]
        vb = pb[i] @ Sigma[np.ix_(nb[i], nb[i])] @ pb[i]
        cab = pa[i] @ Sigma[np.ix_(na[i], nb[i])] @ pb[i]
        ea, eb = math.exp(ma + 0.5 * va), math.exp(mb + 0.5 * vb)
        out[i] = [ea, eb, math.expm1(va) * ea * ea, math.expm1(vb) * eb * eb, math.expm1(cab) * ea * eb]
    return out

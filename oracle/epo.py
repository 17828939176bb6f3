"""Plain FP64 CPU oracle: Python driver over epo.c.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this module.  It shares no code with the GPU
library; the two meet only at the seeded raw draws of ``synth``.

What it computes (Sale & Magorrian, arXiv:1708.09705):

* prior: a Gaussian process on the log pseudo-density f = ln(rho kappa)
  (Sec. 5, dA/ds = rho kappa) on a regular grid, Matern nu = 1/3 (the 3-D
  Kolmogorov spectrum truncated at the outer scale, Sec. 1) tapered to a
  compact support, made sparse by a Vecchia (inverse-Cholesky) precision
  Q0 = (I - B)^T D^{-1} (I - B);
* likelihood: one factor per star on a_n = ln A_n, A_n the line-of-sight
  integral of exp(f); linearised at the current posterior mean each sweep;
* EP: Gaussian sites in a_n, parallel updates (App. A.2, parallel procedure),
  cavity -> tilted -> moment matching (Sec. 4.1 and App. A.2);
* outputs: posterior mean and marginal variance of f at the grid nodes
  (Sec. 5, maps of marginal posterior mean and variance).

The linear algebra is the plain definition (dense numpy Cholesky/inverse);
use it on small grids only.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epo.c")
_SO = os.path.join(_HERE, "libepo.so")
_lib = None

LIK_EXTINCTION = 0
LIK_GAUSS_LINEAR = 1


def build(force: bool = False) -> str:
    """Compile epo.c with gcc (FP64, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        L.epo_besselk.restype = d
        L.epo_besselk.argtypes = [d, d]
        L.epo_matern13.restype = d
        L.epo_matern13.argtypes = [d, d, d]
        L.epo_wendland.restype = d
        L.epo_wendland.argtypes = [d, d]
        L.epo_cov.restype = d
        L.epo_cov.argtypes = [d, d, d, d]
        L.epo_gk15_rule.argtypes = [p, p, p]
        L.epo_vecchia_nnz.restype = i64
        L.epo_vecchia_nnz.argtypes = [i32, d, d]
        L.epo_vecchia.restype = i32
        L.epo_vecchia.argtypes = [i32, d, d, d, d, d, p, p, p, p]
        L.epo_prior_draw.argtypes = [i64, p, p, p, p, d, p, p]
        L.epo_prior_quadform_batch.argtypes = [i64, p, p, p, p, i64, p, p, p, p]
        L.epo_q0_solve_multi.argtypes = [i64, p, p, p, p, i64, p]
        L.epo_q_mul_multi.argtypes = [i64, p, p, p, p, i64, p, p, p, p, i64, p, p, p]
        L.epo_los_counts.argtypes = [i32, d, p, d, i64, p, p]
        L.epo_los_fill.argtypes = [i32, d, p, d, i64, p, p, p]
        L.epo_los_linearise.argtypes = [i32, d, p, d, i64, p, p, p, p, p, p, p]
        L.epo_tilted.restype = i32
        L.epo_tilted.argtypes = [i32, d, d, d, d, p, p, p]
        L.epo_tilted_batch.restype = i32
        L.epo_tilted_batch.argtypes = [i32, i64, p, p, p, p, p, p, p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# Covariance
# ----------------------------------------------------------------------------
def besselk(nu: float, x: float) -> float:
    return lib().epo_besselk(nu, x)


def matern13(var: float, ell: float, r: float) -> float:
    return lib().epo_matern13(var, ell, r)


def wendland(rs: float, r: float) -> float:
    return lib().epo_wendland(rs, r)


def cov(var: float, ell: float, rs: float, r: float) -> float:
    """Tapered prior covariance C(r) W(r)."""
    return lib().epo_cov(var, ell, rs, r)


def gk15_rule():
    xk, wk, wg = np.zeros(8), np.zeros(8), np.zeros(4)
    lib().epo_gk15_rule(_p(xk), _p(wk), _p(wg))
    return xk, wk, wg


# ----------------------------------------------------------------------------
# Geometry and Vecchia prior
# ----------------------------------------------------------------------------
class Grid:
    def __init__(self, cfg: dict):
        self.n = int(cfg["n"])
        self.L = float(cfg["box_pc"])
        self.h = self.L / (self.n - 1)
        self.N = self.n ** 3
        self.obs = np.asarray(cfg["observer_pc"], dtype=np.float64).copy()
        self.step = float(cfg["los_step_pc"])

    def xyz(self) -> np.ndarray:
        p = np.arange(self.N)
        n = self.n
        return np.stack([p % n, (p // n) % n, p // (n * n)], axis=1) * self.h


class Vecchia:
    """B (CSR, strictly lower in lexicographic order) and D of the Vecchia
    approximation of the tapered covariance; Q0 = (I-B)^T D^{-1} (I-B)."""

    def __init__(self, cfg: dict):
        g = Grid(cfg)
        self.grid = g
        var, ell, rs = float(cfg["prior_var"]), float(cfg["outer_scale_pc"]), float(cfg["support_pc"])
        rho = float(cfg.get("vecchia_radius_pc") or rs)
        nnz = lib().epo_vecchia_nnz(g.n, g.h, rho)
        self.rowptr = np.zeros(g.N + 1, dtype=np.int64)
        self.col = np.zeros(max(nnz, 1), dtype=np.int32)
        self.val = np.zeros(max(nnz, 1), dtype=np.float64)
        self.d = np.zeros(g.N, dtype=np.float64)
        rc = lib().epo_vecchia(g.n, g.h, var, ell, rs, rho, _p(self.rowptr), _p(self.col),
                               _p(self.val), _p(self.d))
        if rc != 0:
            raise RuntimeError("Vecchia precision is not positive definite")
        self.nnz = nnz

    def B_dense(self) -> np.ndarray:
        N = self.grid.N
        B = np.zeros((N, N))
        for p in range(N):
            s, e = self.rowptr[p], self.rowptr[p + 1]
            B[p, self.col[s:e]] = self.val[s:e]
        return B

    def Q0_dense(self) -> np.ndarray:
        N = self.grid.N
        IB = np.eye(N) - self.B_dense()
        return IB.T @ (IB / self.d[:, None])

    def Q0_matvec(self, x: np.ndarray) -> np.ndarray:
        """(I-B)^T D^{-1} (I-B) x without forming Q0."""
        N = self.grid.N
        rows = np.repeat(np.arange(N), np.diff(self.rowptr))
        col = self.col[: self.nnz]
        val = self.val[: self.nnz]
        y = x.copy()
        np.add.at(y, rows, -val * x[col])
        y /= self.d
        z = y.copy()
        np.add.at(z, col, -val * y[rows])
        return z

    def draw(self, m0: float, xi: np.ndarray) -> np.ndarray:
        """Exact prior draw f = m0 + (I-B)^{-1} D^{1/2} xi."""
        f = np.zeros(self.grid.N)
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        lib().epo_prior_draw(self.grid.N, _p(self.rowptr), _p(self.col), _p(self.val), _p(self.d),
                             m0, _p(xi), _p(f))
        return f

    def q0_solve(self, X: np.ndarray) -> np.ndarray:
        """Q0^{-1} X for X of shape (N,) or (N, k)."""
        Y = np.array(X, dtype=np.float64, order="C", copy=True)
        k = 1 if Y.ndim == 1 else Y.shape[1]
        lib().epo_q0_solve_multi(self.grid.N, _p(self.rowptr), _p(self.col), _p(self.val), _p(self.d), k, _p(Y))
        return Y

    def prior_quadform(self, ptr, nodes, gval) -> np.ndarray:
        """g_n^T Q0^{-1} g_n for every star (CSR rows)."""
        S = len(ptr) - 1
        out = np.zeros(S)
        lib().epo_prior_quadform_batch(self.grid.N, _p(self.rowptr), _p(self.col), _p(self.val),
                                       _p(self.d), S, _p(ptr), _p(nodes), _p(gval), _p(out))
        return out


# ----------------------------------------------------------------------------
# Line-of-sight operator
# ----------------------------------------------------------------------------
class Sightlines:
    """Support sets P_n (CSR) of every star's sightline and the linearisation
    of ln A_n = ln sum_t w_t exp(F(s_t)) around a field."""

    def __init__(self, cfg: dict, xyz: np.ndarray):
        self.grid = g = Grid(cfg)
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        S = self.xyz.shape[0]
        counts = np.zeros(S, dtype=np.int32)
        lib().epo_los_counts(g.n, g.h, _p(g.obs), g.step, S, _p(self.xyz), _p(counts))
        self.ptr = np.zeros(S + 1, dtype=np.int64)
        np.cumsum(counts, out=self.ptr[1:])
        self.nodes = np.zeros(int(self.ptr[-1]), dtype=np.int32)
        lib().epo_los_fill(g.n, g.h, _p(g.obs), g.step, S, _p(self.xyz), _p(self.ptr), _p(self.nodes))

    @property
    def n_stars(self) -> int:
        return len(self.ptr) - 1

    def linearise(self, f: np.ndarray):
        g = self.grid
        S = self.n_stars
        f = np.ascontiguousarray(f, dtype=np.float64)
        gval = np.zeros(len(self.nodes))
        lnA = np.zeros(S)
        c = np.zeros(S)
        lib().epo_los_linearise(g.n, g.h, _p(g.obs), g.step, S, _p(self.xyz), _p(self.ptr),
                                _p(self.nodes), _p(f), _p(gval), _p(lnA), _p(c))
        return gval, lnA, c

    def G_dense(self, gval: np.ndarray) -> np.ndarray:
        S, N = self.n_stars, self.grid.N
        G = np.zeros((S, N))
        rows = np.repeat(np.arange(S), np.diff(self.ptr))
        G[rows, self.nodes] = gval
        return G


# ----------------------------------------------------------------------------
# Tilted moments
# ----------------------------------------------------------------------------
def tilted(mode: int, mu, v, A, s):
    """(ln Z, mean, variance) of N(a; mu, v) N(A; e^a, s^2) (mode 0) or
    N(a; mu, v) N(A; a, s^2) (mode 1), vectorised over stars."""
    mu, v, A, s = (np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64),
                                                        np.broadcast(mu, v, A, s).shape))
                   for x in (mu, v, A, s))
    n = mu.size
    lnZ, mh, vh = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().epo_tilted_batch(int(mode), n, _p(mu), _p(v), _p(A), _p(s), _p(lnZ), _p(mh), _p(vh))
    return lnZ.reshape(mu.shape), mh.reshape(mu.shape), vh.reshape(mu.shape)


# ----------------------------------------------------------------------------
# Synthetic observations (forward model on the oracle's own arithmetic)
# ----------------------------------------------------------------------------
def simulate(cfg: dict, raw: dict, gauss_sigma: float | None = None):
    """From raw draws (xi, xyz, sigma, eps) build the true field and the
    observations.

    extinction likelihood:  A_obs = A_true + sigma * eps,  A_true = LOS(f_true)
    gauss_linear likelihood: a_obs = c_n + g_n . f_true + sigma * eps with
      g, c the linearisation at the prior mean (frozen).
    Returns (f_true, A_obs, sightlines)."""
    vec = Vecchia(cfg)
    f_true = vec.draw(float(cfg["prior_mean"]), raw["xi"])
    sl = Sightlines(cfg, raw["xyz"])
    if cfg.get("likelihood", "extinction") == "gauss_linear":
        m0 = np.full(sl.grid.N, float(cfg["prior_mean"]))
        gval, lnA, c = sl.linearise(m0)
        rows = np.repeat(np.arange(sl.n_stars), np.diff(sl.ptr))
        lin = c + np.bincount(rows, weights=gval * f_true[sl.nodes], minlength=sl.n_stars)
        return f_true, lin + raw["sigma"] * raw["eps"], sl
    _, lnA, _ = sl.linearise(f_true)
    return f_true, np.exp(lnA) + raw["sigma"] * raw["eps"], sl


# ----------------------------------------------------------------------------
# Dense parallel EP (small grids)
# ----------------------------------------------------------------------------
class DenseEP:
    """Parallel EP with the plain dense linear algebra.

    State: sites (tau, nu) in a_n = ln A_n, one per star, and the
    linearisation point fhat.  One sweep:
      1. linearise every star at fhat: g_n, c_n;
      2. Q = Q0 + sum tau_n g_n g_n^T,  b = Q0 m0 1 + sum (nu_n - tau_n c_n) g_n;
      3. mu = Q^{-1} b,  Sigma = Q^{-1};
      4. for every star, from the same q: cavity, tilted moments, new site;
      5. fhat = mu, or with a linearisation step r < 1 (a damped
         Gauss-Newton step, same fixed points) fhat <- (1 - r) fhat + r mu.
    """

    def __init__(self, cfg: dict, xyz, A_obs, sigma, sightlines: Sightlines | None = None,
                 vecchia: Vecchia | None = None):
        self.cfg = dict(cfg)
        self.mode = LIK_GAUSS_LINEAR if cfg.get("likelihood", "extinction") == "gauss_linear" else LIK_EXTINCTION
        self.relin = bool(cfg.get("relinearize", True)) and self.mode == LIK_EXTINCTION
        self.vec = vecchia or Vecchia(cfg)
        self.sl = sightlines or Sightlines(cfg, xyz)
        self.grid = self.vec.grid
        self.A_obs = np.asarray(A_obs, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        S = self.sl.n_stars
        self.tau = np.zeros(S)
        self.nu = np.zeros(S)
        self.m0 = float(cfg["prior_mean"])
        self.fhat = np.full(self.grid.N, self.m0)
        self.damping = float(cfg.get("damping", 1.0))
        self.relin_step = float(cfg.get("relin_step", 1.0))
        self.vfloor = float(cfg.get("cavity_var_floor", 0.0))
        self.Q0 = self.vec.Q0_dense()
        self.b0 = self.Q0 @ np.full(self.grid.N, self.m0)
        self._lin = None
        if not self.relin:
            self._lin = self.sl.linearise(np.full(self.grid.N, self.m0))

    def linearisation(self):
        if self.relin:
            return self.sl.linearise(self.fhat)
        return self._lin

    def posterior(self):
        """(mu, Sigma, G, c) with the current sites at the current fhat."""
        gval, lnA, c = self.linearisation()
        G = self.sl.G_dense(gval)
        Q = self.Q0 + G.T @ (self.tau[:, None] * G)
        b = self.b0 + G.T @ (self.nu - self.tau * c)
        Sigma = np.linalg.inv(Q)
        Sigma = 0.5 * (Sigma + Sigma.T)
        mu = np.linalg.solve(Q, b)
        return mu, Sigma, G, c

    def sweep(self) -> dict:
        mu, Sigma, G, c = self.posterior()
        m = c + G @ mu
        v = np.einsum("ij,ij->i", G @ Sigma, G)
        tau_c = 1.0 / v - self.tau
        nu_c = m / v - self.nu
        ok = tau_c > 0.0
        v_c = np.where(ok, np.maximum(1.0 / np.where(ok, tau_c, 1.0), self.vfloor), 1.0)
        mu_c = np.where(ok, nu_c / np.where(ok, tau_c, 1.0), 0.0)
        tau_c = 1.0 / v_c
        nu_c = mu_c / v_c
        lnZ, mh, vh = tilted(self.mode, mu_c, v_c, self.A_obs, self.sigma)
        tau_new = 1.0 / vh - tau_c
        nu_new = mh / vh - nu_c
        good = ok & np.isfinite(tau_new) & np.isfinite(nu_new) & (tau_new >= 0.0)
        d = self.damping
        old_tau = self.tau.copy()
        self.tau = np.where(good, (1 - d) * self.tau + d * tau_new, self.tau)
        self.nu = np.where(good, (1 - d) * self.nu + d * nu_new, self.nu)
        dmu = float(np.max(np.abs(mu - self.fhat)))
        if self.relin:
            self.relinearise(mu)
        return dict(updated=int(good.sum()), skipped_cavity=int((~ok).sum()),
                    skipped_negsite=int((ok & ~good).sum()),
                    max_dtau=float(np.max(np.abs(self.tau - old_tau))), max_dmu=dmu,
                    cav_mu=mu_c, cav_var=v_c, lnZ=lnZ, tilted_mean=mh, tilted_var=vh)

    def relinearise(self, mu):
        """Step 5: move the linearisation point to mu, or the fraction r of
        the way there."""
        r = self.relin_step
        self.fhat = mu.copy() if r == 1.0 else (1.0 - r) * self.fhat + r * mu

    def posterior_mean(self) -> np.ndarray:
        return self.posterior()[0]

    def marginal_var(self) -> np.ndarray:
        return np.diag(self.posterior()[1]).copy()

"""Plain FP64 posterior solves on grids too large for the dense oracle (test
infrastructure only: imported by tests/ and the committed script that writes
the stored expected values, nothing else).

The posterior precision of the oracle's EP (Sec. 4.1; App. A.2) with sites
(tau, nu) at a linearisation point is Q = Q0 + G^T diag(tau) G, with
Q0 = (I - B)^T D^{-1} (I - B) the Vecchia prior precision and G the
sightlines' gradient rows.  Q is never formed: its product with a block of
vectors is the two sparse products with (I - B), the scaling by D^{-1} and
the two products with G.  Q^{-1} R is found by conjugate gradients
preconditioned with Q0^{-1} (the oracle's own triangular solves), one
independent recurrence per column of R.  From it:

* the posterior mean mu = Q^{-1} b, b = Q0 m0 1 + G^T (nu - tau c);
* the marginal variance at node i, (Q^{-1})_ii = e_i^T Q^{-1} e_i;
* the q-marginal variance of a star's log-extinction g_n^T Q^{-1} g_n.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .epo import Sightlines, Vecchia, _p, lib


class PosteriorOps:
    """Products with Q and solves with Q0 for one set of sites."""

    def __init__(self, vec: Vecchia, sl: Sightlines, gval: np.ndarray, tau: np.ndarray):
        self.vec, self.sl = vec, sl
        self.gval = np.ascontiguousarray(gval, dtype=np.float64)
        self.tau = np.ascontiguousarray(tau, dtype=np.float64)
        N, S = vec.grid.N, sl.n_stars
        self.G = sp.csr_matrix((self.gval, sl.nodes, sl.ptr), shape=(S, N))
        self.Gt = self.G.T.tocsr()

    def Q(self, X: np.ndarray) -> np.ndarray:
        X2 = np.ascontiguousarray(X if X.ndim == 2 else X[:, None], dtype=np.float64)
        N, k = X2.shape
        Y = np.empty_like(X2)
        work = np.empty_like(X2)
        v, sl = self.vec, self.sl
        lib().epo_q_mul_multi(N, _p(v.rowptr), _p(v.col), _p(v.val), _p(v.d), sl.n_stars, _p(sl.ptr),
                              _p(sl.nodes), _p(self.gval), _p(self.tau), k, _p(X2), _p(Y), _p(work))
        return Y if X.ndim == 2 else Y[:, 0]

    def Q0(self, x: np.ndarray) -> np.ndarray:
        """Q0 x (no site term)."""
        return PosteriorOps(self.vec, self.sl, self.gval, np.zeros_like(self.tau)).Q(x)

    def M(self, R: np.ndarray) -> np.ndarray:
        return self.vec.q0_solve(R)


def pcg(ops: PosteriorOps, R: np.ndarray, rtol: float = 1e-15, maxit: int = 5000, log=None, stall: int = 40):
    """Q^{-1} R, one preconditioned CG recurrence per column, each run until
    its residual falls below rtol times its right-hand side or stops falling
    (no halving in 40 iterations: rounding has been reached).
    Returns (X, iterations, final relative residual per column)."""
    R = np.asarray(R, dtype=np.float64)
    one = R.ndim == 1
    Rm = R[:, None] if one else R
    X = np.zeros_like(Rm)
    r = Rm.copy()
    z = ops.M(r)
    p = z.copy()
    rz = np.einsum("ij,ij->j", r, z)
    bn = np.linalg.norm(Rm, axis=0)
    active = bn > 0
    res = np.zeros(Rm.shape[1])
    best = np.full(Rm.shape[1], np.inf)
    since = np.zeros(Rm.shape[1], dtype=np.int64)
    it = 0
    for it in range(1, maxit + 1):
        Ap = ops.Q(p)
        pAp = np.einsum("ij,ij->j", p, Ap)
        alpha = np.where(active, rz / np.where(active, pAp, 1.0), 0.0)
        X += alpha[None, :] * p
        r -= alpha[None, :] * Ap
        res = np.linalg.norm(r, axis=0) / np.where(bn > 0, bn, 1.0)
        gain = res < 0.5 * best
        best = np.where(gain, res, best)
        since = np.where(gain, 0, since + 1)
        active = active & (res > rtol) & (since < stall)
        if log and (it % 50 == 0 or not active.any()):
            log(f"pcg iteration {it}: max relative residual {res.max():.3e}, {int(active.sum())} columns active")
        if not active.any():
            break
        z = ops.M(r)
        rz_new = np.einsum("ij,ij->j", r, z)
        beta = np.where(active, rz_new / np.where(rz != 0, rz, 1.0), 0.0)
        rz = rz_new
        p = z + beta[None, :] * p
    return (X[:, 0] if one else X), it, res

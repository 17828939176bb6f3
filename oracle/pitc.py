"""PITC / PIC block EP over inducing values, plain dense FP64.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU leg,
never by the library.

What it computes (Sale & Magorrian, arXiv:1708.09705):

* Sec. 4.1 (simplified case): stars are split into sub-catalogues k; the
  observed log-extinctions are Gaussian, a~_n | a_n ~ N(a_n, sigma_n^2); the
  joint prior of (a, u) is approximated by PITC, blocks independent given the
  values u of the field at R inducing points (App. A.1);
* EP over u with one Gaussian site per sub-catalogue (Sec. 4.1 algorithm,
  App. A.2 parallel form), the tilted distribution built as in App. B:
  p(u | a~_k) = N(m'_k, C'_k) times the reduced cavity;
* the PIC predictive of the field at the grid nodes, node by node from the
  block it is assigned to (App. A.1 PIC, App. C), integrated over q(u);
* the PITC log marginal likelihood ln p(a~) (App. A.1).

The field and the data are the library's: f = ln(rho kappa) at the grid nodes
with prior N(m0 1, K), K the tapered Matern covariance between nodes, and a_n =
c_n + g_n . f, the sightline linearised at the prior mean (the gauss_linear
likelihood), so a and u are jointly Gaussian: mu_k = c_k + G_k m0 1, Sigma_k =
G_k K G_k^T, rho_k = G_k K[:, u], C = K[u, u], m = m0 1.

Readings (where the paper is silent or garbled):

* App. B prints C'_k with a plus sign and rho_n^T; the Gaussian conditional
  covariance is C - rho_k^T (Sigma_k + S_k)^{-1} rho_k, used here (and the
  mean term rho_k^T (.)^{-1} (a~_k - mu_k)).  The same holds for C'_{-k}.
* The hyper-parameters Theta are fixed (no site carries Theta), so the
  reduced cavity is a Gaussian in u alone, kept in natural parameters (it is
  improper before every site has been set once); each block's tilted
  distribution is then Gaussian and one undamped parallel sweep reaches the
  fixed point.
* The predictive integrates over q(u) rather than each block's tilted
  distribution; App. C replaces one by the other at convergence, and for this
  model they are equal at the fixed point.
* sigma_n is a standard deviation (S_k = diag sigma_k^2).

The linear algebra is the plain definition (dense numpy inverse/solve); use it
on small grids only.
"""
from __future__ import annotations

import math

import numpy as np

from . import epo


def node_cov(cfg: dict) -> np.ndarray:
    """K[i, j] = C(|x_i - x_j|) W(|x_i - x_j|) between all grid nodes."""
    g = epo.Grid(cfg)
    n = g.n
    p = np.arange(g.N)
    ijk = np.stack([p % n, (p // n) % n, p // (n * n)], axis=1).astype(np.int64)
    d2 = ((ijk[:, None, :] - ijk[None, :, :]) ** 2).sum(axis=2)
    uniq, inv = np.unique(d2, return_inverse=True)
    var, ell, rs = float(cfg["prior_var"]), float(cfg["outer_scale_pc"]), float(cfg["support_pc"])
    vals = np.array([epo.cov(var, ell, rs, g.h * math.sqrt(float(u))) for u in uniq])
    return vals[inv].reshape(g.N, g.N)


class DensePITC:
    """State: the natural parameters (Lam_k, eta_k) of every block's site on u.

    blocks: sub-catalogue of every star (0..K-1); inducing: node ids of u;
    node_block: the block each node's prediction conditions on."""

    def __init__(self, cfg: dict, xyz, a_obs, sigma, blocks, inducing, node_block=None,
                 sightlines: epo.Sightlines | None = None, K: np.ndarray | None = None):
        self.cfg = dict(cfg)
        self.m0 = float(cfg["prior_mean"])
        self.sl = sightlines or epo.Sightlines(cfg, xyz)
        self.grid = self.sl.grid
        N = self.grid.N
        self.K = node_cov(cfg) if K is None else K
        gval, _, c = self.sl.linearise(np.full(N, self.m0))
        self.G = self.sl.G_dense(gval)
        self.a_obs = np.asarray(a_obs, dtype=np.float64)
        self.s2 = np.asarray(sigma, dtype=np.float64) ** 2
        self.mu_a = c + self.G @ np.full(N, self.m0)
        self.blocks = np.asarray(blocks)
        self.nblk = int(self.blocks.max()) + 1 if self.blocks.size else 0
        self.members = [np.nonzero(self.blocks == k)[0] for k in range(self.nblk)]
        self.u = np.asarray(inducing, dtype=np.int64)
        self.node_block = None if node_block is None else np.asarray(node_block)
        R = len(self.u)
        self.m_u = np.full(R, self.m0)
        self.C = self.K[np.ix_(self.u, self.u)]
        self.Cinv = np.linalg.inv(self.C) if R else np.zeros((0, 0))
        self.Lam = np.zeros((self.nblk, R, R))
        self.eta = np.zeros((self.nblk, R))

    # -- the Gaussian pieces of App. B --------------------------------------
    def block_joint(self, k):
        """(mu_k, Sigma_k + S_k, rho_k) of (a~_k, u)."""
        idx = self.members[k]
        Gk = self.G[idx]
        Sig = Gk @ self.K @ Gk.T + np.diag(self.s2[idx])
        rho = Gk @ self.K[:, self.u]
        return self.mu_a[idx], Sig, rho

    def u_given_block(self, k):
        """p(u | a~_k) = N(m'_k, C'_k) (App. B, minus sign in C'_k)."""
        idx = self.members[k]
        mu, A, rho = self.block_joint(k)
        Ainv = np.linalg.inv(A)
        m1 = self.m_u + rho.T @ Ainv @ (self.a_obs[idx] - mu)
        C1 = self.C - rho.T @ Ainv @ rho
        return m1, 0.5 * (C1 + C1.T)

    # -- EP -------------------------------------------------------------------
    def sweep(self, damping: float = 1.0):
        """One parallel pass: every block from the same q (App. A.2).

        For block k: reduced cavity q'_{-k} = prod_{l != k} q_l; tilted
        q_{\\k} proportional to q'_{-k}(u) p(u | a~_k) (the q-bar_k of App. B);
        the new site is the tilted divided by the full cavity p(u) q'_{-k};
        damped in natural parameters."""
        Lam_tot, eta_tot = self.Lam.sum(axis=0), self.eta.sum(axis=0)
        new_L, new_e = np.zeros_like(self.Lam), np.zeros_like(self.eta)
        for k in range(self.nblk):
            m1, C1 = self.u_given_block(k)
            C1inv = np.linalg.inv(C1)
            Lc, ec = Lam_tot - self.Lam[k], eta_tot - self.eta[k]          # reduced cavity
            Lbar, ebar = C1inv + Lc, C1inv @ m1 + ec                        # q-bar_k
            new_L[k] = Lbar - (self.Cinv + Lc)                              # tilted / cavity
            new_e[k] = ebar - (self.Cinv @ self.m_u + ec)
        d = float(damping)
        self.Lam = (1.0 - d) * self.Lam + d * new_L
        self.eta = (1.0 - d) * self.eta + d * new_e

    def posterior_u(self):
        """(mean, cov) of q(u) = p(u) prod_k q_k(u)."""
        P = self.Cinv + self.Lam.sum(axis=0)
        V = np.linalg.inv(P)
        V = 0.5 * (V + V.T)
        return V @ (self.Cinv @ self.m_u + self.eta.sum(axis=0)), V

    def log_evidence(self) -> float:
        """ln p(a~) under PITC: a~ ~ N(mu, Q + S) with Q = rho C^{-1} rho^T
        off the diagonal blocks and Sigma_k on them (App. A.1)."""
        S = len(self.a_obs)
        rho = self.G @ self.K[:, self.u]
        Q = rho @ self.Cinv @ rho.T
        for k in range(self.nblk):
            idx = self.members[k]
            Q[np.ix_(idx, idx)] = self.G[idx] @ self.K @ self.G[idx].T
        Q += np.diag(self.s2)
        r = self.a_obs - self.mu_a
        sign, logdet = np.linalg.slogdet(Q)
        return float(-0.5 * (S * math.log(2 * math.pi) + logdet + r @ np.linalg.solve(Q, r)))

    # -- prediction -------------------------------------------------------------
    def predict(self):
        """PIC predictive (mean, var) of f at every node: f_p | a~_i, u from the
        joint Gaussian of (f_p, a~_i, u), i = node_block[p], integrated over
        q(u) (App. A.1 PIC, App. C)."""
        N = self.grid.N
        mean, var = np.zeros(N), np.zeros(N)
        mu_u, V_u = self.posterior_u()
        R = len(self.u)
        for i in range(self.nblk):
            nodes = np.nonzero(self.node_block == i)[0]
            if nodes.size == 0:
                continue
            idx = self.members[i]
            mu, A, rho = self.block_joint(i)
            J = np.block([[A, rho], [rho.T, self.C]])
            kst = np.vstack([self.G[idx] @ self.K[:, nodes], self.K[np.ix_(self.u, nodes)]])
            w = np.linalg.solve(J, kst)
            wa, wu = w[: len(idx)], w[len(idx):]
            mean[nodes] = self.m0 + wa.T @ (self.a_obs[idx] - mu) + wu.T @ (mu_u - self.m_u)
            var[nodes] = (np.diag(self.K)[nodes] - np.einsum("ij,ij->j", kst, w)
                          + np.einsum("ij,ij->j", wu, V_u @ wu))
        return mean, var


class DensePITCTheta(DensePITC):
    """The same block EP with the mean parameters Theta in the sites: the
    paper's q(u, Theta) (Sec. 4.1, App. B).  The prior mean of the field is
    the disc + bump function of phi = ln theta, linearised at the hyperprior
    mean phihat = mu0 (the sightlines are frozen there too, the gauss_linear
    likelihood): f = mhat + J psi + delta, psi = phi - phihat ~ N(0, S0),
    delta ~ N(0, K), so that
        a~_k | u, phi:  mean mu_k(phi) = muhat_k + H_k psi (H_k = G_k J)
        u | phi:        mean m(phi)    = mhat_u + J_u psi, covariance C.
    The sites are Gaussians over z = (u, psi), kept in natural parameters.
    Per block, after App. B (minus sign in C'_k, P1):
        p(u | a~_k, phi) = N(m'_k(phi), C'_k),
        m'_k(phi) = m(phi) + rho_k^T A_k^{-1} (a~_k - mu_k(phi)),
        p(a~_k | phi)    = N(mu_k(phi), A_k),  A_k = Sigma_k + S_k;
    the tilted distribution is the reduced cavity times p(phi) p(u | a~_k,
    phi) p(a~_k | phi), and the new site is it divided by the full cavity
    p(phi) p(u | phi) q'_{-k}."""

    def __init__(self, cfg, xyz, a_obs, sigma, blocks, inducing, node_block=None, sightlines=None, K=None,
                 prior=None):
        from . import meanfn
        sl = sightlines or epo.Sightlines(cfg, xyz)
        self.cfg = dict(cfg)
        pos = sl.grid.xyz()
        self.mu0, self.s0sq = prior if prior is not None else meanfn.hyperprior(cfg)
        self.mhat, self.J = meanfn.mean_and_jacobian(cfg, pos, self.mu0)
        N = sl.grid.N
        self.sl = sl
        self.grid = sl.grid
        self.m0 = None
        self.K = node_cov(cfg) if K is None else K
        gval, _, c = sl.linearise(self.mhat)
        self.G = sl.G_dense(gval)
        self.a_obs = np.asarray(a_obs, dtype=np.float64)
        self.s2 = np.asarray(sigma, dtype=np.float64) ** 2
        self.mu_a = c + self.G @ self.mhat               # muhat
        self.H = self.G @ self.J
        self.blocks = np.asarray(blocks)
        self.nblk = int(self.blocks.max()) + 1 if self.blocks.size else 0
        self.members = [np.nonzero(self.blocks == k)[0] for k in range(self.nblk)]
        self.u = np.asarray(inducing, dtype=np.int64)
        self.node_block = None if node_block is None else np.asarray(node_block)
        R, M = len(self.u), len(self.mu0)
        self.M = M
        self.m_u = self.mhat[self.u]
        self.Ju = self.J[self.u]
        self.C = self.K[np.ix_(self.u, self.u)]
        self.Cinv = np.linalg.inv(self.C)
        self.Lam = np.zeros((self.nblk, R + M, R + M))
        self.eta = np.zeros((self.nblk, R + M))

    def _prior_z(self):
        """Natural parameters of p(psi) p(u | phi) over z = (u, psi)."""
        R, M = len(self.u), self.M
        E = np.hstack([np.eye(R), -self.Ju])
        P = E.T @ self.Cinv @ E
        P[R:, R:] += np.diag(1.0 / self.s0sq)
        return P, E.T @ self.Cinv @ self.m_u

    def sweep(self, damping: float = 1.0):
        R, M = len(self.u), self.M
        Lam_tot, eta_tot = self.Lam.sum(axis=0), self.eta.sum(axis=0)
        P0, e0 = self._prior_z()
        new_L, new_e = np.zeros_like(self.Lam), np.zeros_like(self.eta)
        for k in range(self.nblk):
            idx = self.members[k]
            mu, A, rho = self.block_joint(k)
            Ainv = np.linalg.inv(A)
            r = self.a_obs[idx] - mu
            # p(u | a~_k, phi) = N(alpha + beta psi, C'_k)
            alpha = self.m_u + rho.T @ Ainv @ r
            beta = self.Ju - rho.T @ Ainv @ self.H[idx]
            C1 = self.C - rho.T @ Ainv @ rho
            C1inv = np.linalg.inv(0.5 * (C1 + C1.T))
            E1 = np.hstack([np.eye(R), -beta])
            P_cond, e_cond = E1.T @ C1inv @ E1, E1.T @ C1inv @ alpha
            # p(a~_k | phi) = N(muhat_k + H_k psi, A_k)
            Hk = self.H[idx]
            P_marg = np.zeros((R + M, R + M))
            P_marg[R:, R:] = Hk.T @ Ainv @ Hk
            e_marg = np.concatenate([np.zeros(R), Hk.T @ Ainv @ r])
            Lc, ec = Lam_tot - self.Lam[k], eta_tot - self.eta[k]            # reduced cavity
            # tilted = q'_{-k} p(phi) p(u|a~_k,phi) p(a~_k|phi); cavity = p(phi) p(u|phi) q'_{-k}
            Pphi = np.zeros((R + M, R + M))
            Pphi[R:, R:] = np.diag(1.0 / self.s0sq)
            L_til = Lc + Pphi + P_cond + P_marg
            e_til = ec + e_cond + e_marg
            new_L[k] = L_til - (P0 + Lc)
            new_e[k] = e_til - (e0 + ec)
        d = float(damping)
        self.Lam = (1.0 - d) * self.Lam + d * new_L
        self.eta = (1.0 - d) * self.eta + d * new_e

    def posterior_z(self):
        """(mean, cov) of q(u, psi)."""
        P0, e0 = self._prior_z()
        P = P0 + self.Lam.sum(axis=0)
        V = np.linalg.inv(P)
        V = 0.5 * (V + V.T)
        return V @ (e0 + self.eta.sum(axis=0)), V

    def posterior_u(self):
        m, V = self.posterior_z()
        R = len(self.u)
        return m[:R], V[:R, :R]

    def theta_posterior(self):
        """Mean and covariance of phi = ln theta under q."""
        m, V = self.posterior_z()
        R = len(self.u)
        return self.mu0 + m[R:], V[R:, R:]

    def log_evidence(self) -> float:
        """ln p(a~) with phi marginalised: a~ ~ N(muhat, Q + S + H S0 H^T)."""
        S = len(self.a_obs)
        rho = self.G @ self.K[:, self.u]
        Q = rho @ self.Cinv @ rho.T
        for k in range(self.nblk):
            idx = self.members[k]
            Q[np.ix_(idx, idx)] = self.G[idx] @ self.K @ self.G[idx].T
        Q += np.diag(self.s2) + self.H @ np.diag(self.s0sq) @ self.H.T
        r = self.a_obs - self.mu_a
        _, logdet = np.linalg.slogdet(Q)
        return float(-0.5 * (S * math.log(2 * math.pi) + logdet + r @ np.linalg.solve(Q, r)))

    def predict(self):
        """PIC predictive of f at every node: f_p = mhat_p + J_p psi + delta_p,
        delta_p | a~_i, u, psi from the joint Gaussian of (delta_p, a~_i, u)
        given psi, integrated over q(u, psi)."""
        N = self.grid.N
        mean, var = np.zeros(N), np.zeros(N)
        mz, Vz = self.posterior_z()
        R = len(self.u)
        for i in range(self.nblk):
            nodes = np.nonzero(self.node_block == i)[0]
            if nodes.size == 0:
                continue
            idx = self.members[i]
            mu, A, rho = self.block_joint(i)
            J = np.block([[A, rho], [rho.T, self.C]])
            kst = np.vstack([self.G[idx] @ self.K[:, nodes], self.K[np.ix_(self.u, nodes)]])
            w = np.linalg.solve(J, kst)
            wa, wu = w[: len(idx)], w[len(idx):]
            # E[delta_p | a~_i, u, psi] = wa^T (a~_i - muhat_i - H_i psi) + wu^T (u - mhat_u - J_u psi)
            # so f_p = const + b^T z with b = (wu, J_p - H_i^T wa - J_u^T wu)
            b = np.vstack([wu, self.J[nodes].T - self.H[idx].T @ wa - self.Ju.T @ wu])
            const = self.mhat[nodes] + wa.T @ (self.a_obs[idx] - mu) - wu.T @ self.m_u
            mean[nodes] = const + b.T @ mz
            var[nodes] = (np.diag(self.K)[nodes] - np.einsum("ij,ij->j", kst, w)
                          + np.einsum("ij,ij->j", b, Vz @ b))
        return mean, var


class DensePITCExt:
    """PITC with the extinction likelihood: parallel EP with one Gaussian
    site per star on a_n (as on the grid path, Sec. 4.1), the prior of a
    being the PITC approximation instead of the grid's (App. A.1): a ~
    N(mu_a, Q), Q = Sigma_k on the sub-catalogue blocks and rho_k C^{-1}
    rho_l^T between them, a_n = c_n + g_n . f linearised at the prior mean
    (frozen, as in the Gaussian PITC pass), A_n | a_n ~ N(e^{a_n}, sigma_n^2).

    Readings: the paper forms one site per sub-catalogue over (u, Theta) and
    samples the tilted distributions; here every star keeps its own site, so
    the tilted distributions are the one-dimensional ones of the grid path
    and the sub-catalogues enter through the prior.  With one sub-catalogue
    and an exact prior this is the grid path's EP with frozen sightlines.
    Given the sites the posterior is Gaussian, and so are q(u) and the PIC
    predictive: those of the Gaussian pass with pseudo-observations nu/tau
    of variance 1/tau, written in the scaled form s = sqrt(tau) so that stars
    without a site (tau = 0) carry no information.  Mean parameters are not
    inferred here (constant prior mean)."""

    def __init__(self, cfg: dict, xyz, A_obs, sigma, blocks, inducing, node_block=None,
                 sightlines: epo.Sightlines | None = None, K: np.ndarray | None = None):
        self.cfg = dict(cfg)
        self.m0 = float(cfg["prior_mean"])
        self.sl = sightlines or epo.Sightlines(cfg, xyz)
        self.grid = self.sl.grid
        N = self.grid.N
        self.K = node_cov(cfg) if K is None else K
        gval, _, c = self.sl.linearise(np.full(N, self.m0))
        self.G = self.sl.G_dense(gval)
        self.A_obs = np.asarray(A_obs, dtype=np.float64)
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.mu_a = c + self.G @ np.full(N, self.m0)
        self.blocks = np.asarray(blocks)
        self.nblk = int(self.blocks.max()) + 1 if self.blocks.size else 0
        self.members = [np.nonzero(self.blocks == k)[0] for k in range(self.nblk)]
        self.u = np.asarray(inducing, dtype=np.int64)
        self.node_block = None if node_block is None else np.asarray(node_block)
        self.m_u = np.full(len(self.u), self.m0)
        self.C = self.K[np.ix_(self.u, self.u)]
        self.Cinv = np.linalg.inv(self.C)
        self.rho = self.G @ self.K[:, self.u]
        Q = self.rho @ self.Cinv @ self.rho.T
        for idx in self.members:
            Q[np.ix_(idx, idx)] = self.G[idx] @ self.K @ self.G[idx].T
        self.Q = 0.5 * (Q + Q.T)
        S = len(self.A_obs)
        self.tau = np.zeros(S)
        self.nu = np.zeros(S)
        self.vfloor = float(cfg.get("cavity_var_floor", 0.0))

    def _scaled(self):
        """s = sqrt(tau), B = I + S Q S and r~ = (nu - tau mu_a) / s (0 where tau = 0)."""
        s = np.sqrt(self.tau)
        B = np.eye(len(s)) + s[:, None] * self.Q * s[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            rt = np.where(s > 0, (self.nu - self.tau * self.mu_a) / np.where(s > 0, s, 1.0), 0.0)
        return s, B, rt

    def posterior_a(self):
        """(mean, cov) of q(a) = N(mu_a, Q) prod_n N(a_n; nu_n/tau_n, 1/tau_n)."""
        s, B, rt = self._scaled()
        SQ = s[:, None] * self.Q
        cov = self.Q - SQ.T @ np.linalg.solve(B, SQ)
        cov = 0.5 * (cov + cov.T)
        mean = self.mu_a + SQ.T @ np.linalg.solve(B, rt)
        return mean, cov

    def sweep(self, damping: float = 1.0) -> dict:
        """Every star from the same q (App. A.2): cavity, tilted moments,
        new site; the skip rules and the cavity floor of the grid path."""
        m, P = self.posterior_a()
        v = np.diag(P).copy()
        tau_c = 1.0 / v - self.tau
        nu_c = m / v - self.nu
        ok = tau_c > 0.0
        v_c = np.where(ok, np.maximum(1.0 / np.where(ok, tau_c, 1.0), self.vfloor), 1.0)
        mu_c = np.where(ok, nu_c / np.where(ok, tau_c, 1.0), 0.0)
        tau_c, nu_c = 1.0 / v_c, mu_c / v_c
        lnZ, mh, vh = epo.tilted(epo.LIK_EXTINCTION, mu_c, v_c, self.A_obs, self.sigma)
        with np.errstate(divide="ignore", invalid="ignore"):
            tau_new = 1.0 / vh - tau_c
            nu_new = mh / vh - nu_c
        good = ok & np.isfinite(tau_new) & np.isfinite(nu_new) & (tau_new >= 0.0)
        d = float(damping)
        old = self.tau.copy()
        self.tau = np.where(good, (1 - d) * self.tau + d * tau_new, self.tau)
        self.nu = np.where(good, (1 - d) * self.nu + d * nu_new, self.nu)
        return dict(updated=int(good.sum()), skipped_cavity=int((~ok).sum()),
                    skipped_negsite=int((ok & ~good).sum()), max_dtau=float(np.max(np.abs(self.tau - old))),
                    marg_mean=m, marg_var=v, lnZ=lnZ, tilted_mean=mh, tilted_var=vh)

    def posterior_u(self):
        """(mean, cov) of q(u): (u, a) jointly Gaussian under PITC, cov(u, a) = rho^T."""
        s, B, rt = self._scaled()
        Sr = s[:, None] * self.rho
        mean = self.m_u + Sr.T @ np.linalg.solve(B, rt)
        cov = self.C - Sr.T @ np.linalg.solve(B, Sr)
        return mean, 0.5 * (cov + cov.T)

    def predict(self):
        """PIC predictive (mean, var) of f at every node from its block's
        scaled pseudo-observations and u, integrated over q(u)."""
        N = self.grid.N
        mean, var = np.zeros(N), np.zeros(N)
        mu_u, V_u = self.posterior_u()
        s, _, rt = self._scaled()
        for i in range(self.nblk):
            nodes = np.nonzero(self.node_block == i)[0]
            if nodes.size == 0:
                continue
            idx = self.members[i]
            si = s[idx]
            Bi = np.eye(len(idx)) + si[:, None] * self.Q[np.ix_(idx, idx)] * si[None, :]
            rho = si[:, None] * self.rho[idx]
            J = np.block([[Bi, rho], [rho.T, self.C]])
            kst = np.vstack([si[:, None] * (self.G[idx] @ self.K[:, nodes]), self.K[np.ix_(self.u, nodes)]])
            w = np.linalg.solve(J, kst)
            wa, wu = w[: len(idx)], w[len(idx):]
            mean[nodes] = self.m0 + wa.T @ rt[idx] + wu.T @ (mu_u - self.m_u)
            var[nodes] = (np.diag(self.K)[nodes] - np.einsum("ij,ij->j", kst, w)
                          + np.einsum("ij,ij->j", wu, V_u @ wu))
        return mean, var

"""Plain FP64 reference of EP with a parametric prior mean whose parameters
are inferred with the field (test infrastructure only: imported by tests/
and bench.py's CPU leg, nothing else).

Mean function (Sec. 5 tests): the pseudo-density rho kappa is an
exponential disc plus a Gaussian bump,

    rho kappa(x) = rk0 exp(-(R - R0)/L - |h|/H) + A_b N(y - y_o; s_b, w^2) exp(-|h|/H),

theta = (L, H, rk0, s_b, A_b); the bump width w is fixed.  Geometry (our
reading): the observer o sits in the disc mid-plane at Galactocentric radius
R0 and looks along +y, away from the Galactic centre, so R(x) =
sqrt((R0 + y - y_o)^2 + (x - x_o)^2) and h = z - z_o; the bump is a slab
across the line of sight at distance s_b.  The GP is on f = ln rho kappa,
so its prior mean is m(x; theta) = ln rho kappa(x).

Hyperprior: independent log-normals whose mean and standard deviation both
equal the given value M_j; in phi = ln theta that is N(ln M_j - ln2/2, ln 2).

Joint EP over (delta, phi), f = m(phi) + delta, delta ~ N(0, Q0^{-1}) (the
paper's q(u, Theta), Gaussian in the latent field and the hyperparameters,
Sec. 4.1).  Each sweep linearises the mean about phihat (also in the
Gaussian mode, whose sightlines stay frozen),
m(phi) ~ mhat + J (phi - phihat), and every sightline about fhat = mhat +
deltahat, so the site variable a_n = c'_n + g_n.delta + h_n.phi with
h_n = J^T g_n and c'_n = c_n + g_n.mhat - h_n.phihat.  The posterior of
(delta, phi) is then Gaussian with precision
    [[Q0 + G^T T G, G^T T H], [H^T T G, S0^{-1} + H^T T H]]
and the cavities, tilted moments and site updates are those of the
fixed-mean EP.  After the sweep deltahat, phihat <- the posterior means
(with a linearisation step r < 1: move the fraction r of the way there).
"""
from __future__ import annotations

import math

import numpy as np

from .epo import DenseEP, LIK_GAUSS_LINEAR, tilted

N_THETA = 5
NAMES = ("L_pc", "H_pc", "rk0_per_pc", "s_bump_pc", "A_bump")
DEFAULT_PRIOR = (3000.0, 150.0, 7.5e-4, 2000.0, 0.1)     # Sec. 5 hyperprior means (rk0 in mag/pc)


def geometry(cfg):
    o = np.asarray(cfg["observer_pc"], dtype=np.float64)
    return o, float(cfg.get("sun_radius_pc", 8000.0)), float(cfg.get("bump_width_pc", 400.0))


def components(cfg, pos, theta):
    """(disc, bump) pseudo-densities at positions pos (m x 3)."""
    o, R0, w = geometry(cfg)
    L, H, rk0, sb, Ab = [float(t) for t in theta]
    pos = np.atleast_2d(pos)
    dy = pos[:, 1] - o[1]
    R = np.sqrt((R0 + dy) ** 2 + (pos[:, 0] - o[0]) ** 2)
    vert = np.exp(-np.abs(pos[:, 2] - o[2]) / H)
    disc = rk0 * np.exp(-(R - R0) / L) * vert
    bump = Ab / (math.sqrt(2 * math.pi) * w) * np.exp(-0.5 * ((dy - sb) / w) ** 2) * vert
    return disc, bump


def mean_and_jacobian(cfg, pos, phi):
    """m(x; theta) = ln(disc + bump) and dm/dphi_j (m x 5), phi = ln theta."""
    o, R0, w = geometry(cfg)
    theta = np.exp(np.asarray(phi, dtype=np.float64))
    L, H, rk0, sb, Ab = theta
    pos = np.atleast_2d(pos)
    D, B = components(cfg, pos, theta)
    S = D + B
    dy = pos[:, 1] - o[1]
    R = np.sqrt((R0 + dy) ** 2 + (pos[:, 0] - o[0]) ** 2)
    habs = np.abs(pos[:, 2] - o[2])
    J = np.empty((pos.shape[0], N_THETA))
    J[:, 0] = D * (R - R0) / L / S          # d disc / d ln L = disc (R - R0) / L
    J[:, 1] = habs / H                        # both terms share exp(-|h|/H)
    J[:, 2] = D / S
    J[:, 3] = B * (dy - sb) * sb / (w * w) / S
    J[:, 4] = B / S
    return np.log(S), J


def hyperprior(cfg):
    """(mu0, s0^2) of phi = ln theta."""
    M = np.asarray(cfg.get("theta_prior", DEFAULT_PRIOR), dtype=np.float64)
    s2 = math.log(2.0)
    return np.log(M) - 0.5 * s2, np.full(N_THETA, s2)


def simulate(cfg, raw, theta_true, vecchia=None, sightlines=None):
    """f_true = m(x; theta_true) + a zero-mean prior draw; A_obs from the
    sightline forward model plus noise (the deviates of raw)."""
    from .epo import Sightlines, Vecchia
    vec = vecchia or Vecchia(cfg)
    sl = sightlines or Sightlines(cfg, raw["xyz"])
    pos = vec.grid.xyz()
    m, _ = mean_and_jacobian(cfg, pos, np.log(np.asarray(theta_true, dtype=np.float64)))
    f_true = m + vec.draw(0.0, raw["xi"])
    _, lnA, _ = sl.linearise(f_true)
    return f_true, np.exp(lnA) + raw["sigma"] * raw["eps"], sl


class DenseEPTheta(DenseEP):
    """DenseEP over (delta, phi).  mean: optional callable phi -> (m, J) on
    the grid nodes (default: the disc + bump function of cfg)."""

    def __init__(self, cfg, xyz, A_obs, sigma, sightlines=None, vecchia=None, mean=None, prior=None):
        super().__init__(cfg, xyz, A_obs, sigma, sightlines=sightlines, vecchia=vecchia)
        pos = self.grid.xyz()
        self.mean = mean or (lambda phi: mean_and_jacobian(cfg, pos, phi))
        self.mu0, self.s0sq = prior if prior is not None else hyperprior(cfg)
        self.M = len(self.mu0)
        self.phihat = np.array(self.mu0, dtype=np.float64)
        m, J = self.mean(self.phihat)
        self.fhat = m.copy()
        self._mJ = (m, J)
        self._lin = None
        if not self.relin:
            self._lin = self.sl.linearise(self.fhat)
        # the mean is re-linearised at phihat every sweep whenever relinearize
        # is on, also in the Gaussian mode, whose sightlines stay frozen at the
        # prior mean (its observation model)
        self.relin_mean = bool(cfg.get("relinearize", True))

    def mean_linearisation(self):
        if self.relin_mean:
            self._mJ = self.mean(self.phihat)
        return self._mJ

    def augmented(self):
        """(Gx = [G, H], c') of the site variables a = c' + Gx (delta, phi)."""
        gval, lnA, c = self.linearisation()
        self._lnA = lnA
        G = self.sl.G_dense(gval)
        m, J = self.mean_linearisation()
        H = G @ J
        cp = c + G @ m - H @ self.phihat
        return np.hstack([G, H]), cp

    def tilted_moments(self, mu_c, v_c):
        """The per-star tilted moments (the likelihood's; a subclass may
        replace the likelihood)."""
        return tilted(self.mode, mu_c, v_c, self.A_obs, self.sigma)

    def posterior_x(self):
        Gx, cp = self.augmented()
        N, M = self.grid.N, self.M
        Q = np.zeros((N + M, N + M))
        Q[:N, :N] = self.Q0
        Q[N:, N:] = np.diag(1.0 / self.s0sq)
        Q += Gx.T @ (self.tau[:, None] * Gx)
        b = np.zeros(N + M)
        b[N:] = self.mu0 / self.s0sq
        b += Gx.T @ (self.nu - self.tau * cp)
        Sigma = np.linalg.inv(Q)
        Sigma = 0.5 * (Sigma + Sigma.T)
        return np.linalg.solve(Q, b), Sigma, Gx, cp

    def sweep(self) -> dict:
        mu, Sigma, Gx, cp = self.posterior_x()
        m = cp + Gx @ mu
        v = np.einsum("ij,ij->i", Gx @ Sigma, Gx)
        tau_c = 1.0 / v - self.tau
        nu_c = m / v - self.nu
        ok = tau_c > 0.0
        v_c = np.where(ok, np.maximum(1.0 / np.where(ok, tau_c, 1.0), self.vfloor), 1.0)
        mu_c = np.where(ok, nu_c / np.where(ok, tau_c, 1.0), 0.0)
        tau_c, nu_c = 1.0 / v_c, mu_c / v_c
        lnZ, mh, vh = self.tilted_moments(mu_c, v_c)
        tau_new = 1.0 / vh - tau_c
        nu_new = mh / vh - nu_c
        good = ok & np.isfinite(tau_new) & np.isfinite(nu_new) & (tau_new >= 0.0)
        d = self.damping
        self.tau = np.where(good, (1 - d) * self.tau + d * tau_new, self.tau)
        self.nu = np.where(good, (1 - d) * self.nu + d * nu_new, self.nu)
        N = self.grid.N
        if self.relin:
            # deltahat = fhat - m(phihat) and phihat move the fraction r of the
            # way to the posterior means (r = 1: onto them), then
            # fhat = m(phihat) + deltahat
            r = self.relin_step
            if r == 1.0:
                self.phihat = mu[N:].copy()
                dhat = mu[:N]
            else:
                mold, _ = self.mean(self.phihat)
                dhat = (1.0 - r) * (self.fhat - mold) + r * mu[:N]
                self.phihat = (1.0 - r) * self.phihat + r * mu[N:]
            mnew, _ = self.mean(self.phihat)
            self.fhat = mnew + dhat
        elif self.relin_mean:
            # Gaussian mode: a damped Gauss-Newton step of the mean's
            # linearisation point (full steps can cycle when the bump is
            # weakly identified)
            self.phihat = (1 - d) * self.phihat + d * mu[N:]
        return dict(updated=int(good.sum()), skipped_cavity=int((~ok).sum()),
                    skipped_negsite=int((ok & ~good).sum()), cav_mu=mu_c, cav_var=v_c,
                    lnZ=lnZ, tilted_mean=mh, tilted_var=vh)

    def f_operator(self):
        """A with f = const + A (delta, phi) under the current mean linearisation."""
        m, J = self.mean_linearisation()
        return np.hstack([np.eye(self.grid.N), J]), m - J @ self.phihat

    def posterior_mean(self) -> np.ndarray:
        mu, _, _, _ = self.posterior_x()
        A, c0 = self.f_operator()
        return c0 + A @ mu

    def marginal_var(self) -> np.ndarray:
        _, Sigma, _, _ = self.posterior_x()
        A, _ = self.f_operator()
        return np.einsum("ij,ij->i", A @ Sigma, A)

    def theta_posterior(self):
        """Mean (M) and covariance (M x M) of phi = ln theta."""
        mu, Sigma, _, _ = self.posterior_x()
        N = self.grid.N
        return mu[N:].copy(), Sigma[N:, N:].copy()


def exact_theta_posterior_gaussian(cfg, sl, vec, a_obs, sigma, prop_mean, prop_cov, n_samples=8000, seed=0,
                                   dof=5.0):
    """Mean and covariance of the exact p(phi | a~) in the Gaussian mode, by
    importance sampling.  The sightlines are linearised at the prior mean
    m(mu0) (the observation model), so given phi the data are exactly
    Gaussian: a~ ~ N(c + G m(phi), G K G^T + S), K = Q0^{-1}, S = diag sigma^2,
    times the log-normal hyperprior.  Proposal: a multivariate t (dof) with
    the given mean and covariance.  Returns (mean, covariance, effective
    sample size)."""
    import scipy.linalg as sla
    pos = vec.grid.xyz()
    mu0, s02 = hyperprior(cfg)
    m0, _ = mean_and_jacobian(cfg, pos, mu0)
    gval, _, c = sl.linearise(m0)
    G = sl.G_dense(gval)
    K = np.linalg.inv(vec.Q0_dense())
    L = np.linalg.cholesky(G @ K @ G.T + np.diag(np.asarray(sigma, dtype=np.float64) ** 2))
    rng = np.random.default_rng(seed)
    Lp = np.linalg.cholesky(prop_cov)
    k = len(prop_mean)
    X = prop_mean + (rng.standard_normal((n_samples, k)) @ Lp.T) * np.sqrt(dof / rng.chisquare(dof, n_samples))[:, None]
    d = sla.solve_triangular(Lp, (X - prop_mean).T, lower=True).T
    lq = -0.5 * (dof + k) * np.log1p(np.sum(d * d, 1) / dof)
    lp = np.empty(n_samples)
    for s in range(0, n_samples, 500):
        Xb = X[s:s + 500]
        with np.errstate(all="ignore"):
            R = np.stack([a_obs - c - G @ mean_and_jacobian(cfg, pos, x)[0] for x in Xb], axis=1)
        ok = np.all(np.isfinite(R), axis=0)      # a draw so far out that the mean under- or overflows
        R[:, ~ok] = 0.0
        Y = sla.solve_triangular(L, R, lower=True)
        lp[s:s + 500] = np.where(ok, -0.5 * np.sum(Y * Y, 0) - 0.5 * np.sum((Xb - mu0) ** 2 / s02, 1), -np.inf)
    lw = lp - lq
    w = np.exp(lw - lw.max())
    w /= w.sum()
    mean = w @ X
    cov = (X - mean).T @ ((X - mean) * w[:, None])
    return mean, cov, 1.0 / float(np.sum(w * w))

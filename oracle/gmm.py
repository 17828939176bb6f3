"""Plain FP64 reference of EP with unknown distances (test infrastructure
only: imported by tests/ and nothing else).

General case of Sec. 4.2: each star's photometry gives a Gaussian mixture
over components z in (l, b) = (ln s, log-extinction implied at distance s):
weight w_z, mean (m_l, m_b), covariance [[C_ll, C_lb], [C_lb, C_bb]]
(Sec. 3's GMM approximation of the likelihood).  The distance s is
marginalised in the tilted distribution together with z.

The site variable stays a_n = ln A to the star's reference position at
distance s~ (its catalogue position); the log-extinction at distance s is
linearised in l = ln s about l~ = ln s~ with the current field,
    a(s) ~ a_n + beta_n (l - l~),  beta_n = d ln A / d ln s = s~ e^{F(x_n)} / A_n,
(e^F the pseudo-density at the star, A_n the extinction to it).  For one
component the likelihood in a_n is then
    int dl N((l, a_n + beta (l - l~)); m, C) = N(a_n; m_b - beta (m_l - l~),
                                                 C_bb - 2 beta C_lb + beta^2 C_ll)
(the density of b - beta (l - l~) under (l, b) ~ N(m, C); the shear has unit
Jacobian), so the tilted distribution is a Gaussian mixture with closed-form
normaliser and moments.
"""
from __future__ import annotations

import math

import numpy as np

from .epo import DenseEP
from .maps import point_weights

NCOMP = 6   # per component: weight, m_l, m_b, C_ll, C_lb, C_bb


def likelihood_in_a(comps, beta, lref):
    """(w, mean, var) of the Gaussian mixture likelihood in a_n; comps is
    (S, K, 6), beta and lref (S,)."""
    comps = np.asarray(comps, dtype=np.float64)
    w, ml, mb, cll, clb, cbb = [comps[..., k] for k in range(NCOMP)]
    b = np.asarray(beta, dtype=np.float64)[:, None]
    m = mb - b * (ml - np.asarray(lref, dtype=np.float64)[:, None])
    v = cbb - 2 * b * clb + b * b * cll
    return w, m, v


def gmm_tilted(mu_c, v_c, comps, beta, lref):
    """ln Z, mean and variance of N(a; mu_c, v_c) times the mixture likelihood."""
    w, m, v = likelihood_in_a(comps, beta, lref)
    mu_c = np.asarray(mu_c, dtype=np.float64)[:, None]
    v_c = np.asarray(v_c, dtype=np.float64)[:, None]
    s = v_c + v
    with np.errstate(divide="ignore"):
        lz = np.log(w) - 0.5 * np.log(2 * math.pi * s) - 0.5 * (m - mu_c) ** 2 / s
    top = np.max(lz, axis=1, keepdims=True)
    r = np.exp(lz - top)
    Z = np.sum(r, axis=1, keepdims=True)
    r = r / Z
    vz = v_c * v / s
    mz = vz * (mu_c / v_c + m / v)
    mean = np.sum(r * mz, axis=1)
    var = np.sum(r * (vz + (mz - mean[:, None]) ** 2), axis=1)
    return (top + np.log(Z))[:, 0], mean, var


def beta_at(cfg, xyz, f, lnA):
    """beta_n = d_n e^{F(x_n)} / A_n with F the trilinear field at the star."""
    o = np.asarray(cfg["observer_pc"], dtype=np.float64)
    xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
    nodes, phi = point_weights(cfg, xyz)
    F = np.sum(phi * f[nodes], axis=1)
    d = np.linalg.norm(xyz - o, axis=1)
    return d * np.exp(F - lnA)


class DenseEPGMM(DenseEP):
    """DenseEP whose per-star likelihood is the distance-marginalised mixture.
    Each sweep takes beta at the linearisation point with the sightlines."""

    def __init__(self, cfg, xyz, comps, sightlines=None, vecchia=None):
        S = len(np.atleast_2d(xyz))
        super().__init__(dict(cfg, likelihood="extinction"), xyz, np.zeros(S), np.ones(S),
                         sightlines=sightlines, vecchia=vecchia)
        self.xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
        self.comps = np.asarray(comps, dtype=np.float64).reshape(S, -1, NCOMP)
        o = np.asarray(cfg["observer_pc"], dtype=np.float64)
        self.lref = np.log(np.linalg.norm(self.xyz - o, axis=1))

    def sweep(self) -> dict:
        gval, lnA, c = self.linearisation()
        G = self.sl.G_dense(gval)
        Q = self.Q0 + G.T @ (self.tau[:, None] * G)
        b = self.b0 + G.T @ (self.nu - self.tau * c)
        Sigma = np.linalg.inv(Q)
        Sigma = 0.5 * (Sigma + Sigma.T)
        mu = np.linalg.solve(Q, b)
        beta = beta_at(self.cfg, self.xyz, self.fhat, lnA)
        m = c + G @ mu
        v = np.einsum("ij,ij->i", G @ Sigma, G)
        tau_c = 1.0 / v - self.tau
        nu_c = m / v - self.nu
        ok = tau_c > 0.0
        v_c = np.where(ok, np.maximum(1.0 / np.where(ok, tau_c, 1.0), self.vfloor), 1.0)
        mu_c = np.where(ok, nu_c / np.where(ok, tau_c, 1.0), 0.0)
        tau_c, nu_c = 1.0 / v_c, mu_c / v_c
        lnZ, mh, vh = gmm_tilted(mu_c, v_c, self.comps, beta, self.lref)
        tau_new = 1.0 / vh - tau_c
        nu_new = mh / vh - nu_c
        good = ok & np.isfinite(tau_new) & np.isfinite(nu_new) & (tau_new >= 0.0)
        d = self.damping
        self.tau = np.where(good, (1 - d) * self.tau + d * tau_new, self.tau)
        self.nu = np.where(good, (1 - d) * self.nu + d * nu_new, self.nu)
        if self.relin:
            self.fhat = mu
        return dict(updated=int(good.sum()), skipped_cavity=int((~ok).sum()),
                    skipped_negsite=int((ok & ~good).sum()), beta=beta, cav_mu=mu_c, cav_var=v_c,
                    lnZ=lnZ, tilted_mean=mh, tilted_var=vh)


class DenseEPThetaGMM:
    """The inferred-mean EP (meanfn.DenseEPTheta) with the distance-mixture
    likelihood: beta at the linearisation point fhat = m(phihat) + deltahat."""

    def __new__(cls, cfg, xyz, comps, sightlines=None, vecchia=None):
        from .meanfn import DenseEPTheta

        class _Impl(DenseEPTheta):
            def tilted_moments(self, mu_c, v_c):
                beta = beta_at(self.cfg, self.xyz, self.fhat, self._lnA)
                return gmm_tilted(mu_c, v_c, self.comps, beta, self.lref)

        S = len(np.atleast_2d(xyz))
        ep = _Impl(dict(cfg, likelihood="extinction"), xyz, np.zeros(S), np.ones(S), sightlines=sightlines,
                   vecchia=vecchia)
        ep.xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
        ep.comps = np.asarray(comps, dtype=np.float64).reshape(S, -1, NCOMP)
        o = np.asarray(cfg["observer_pc"], dtype=np.float64)
        ep.lref = np.log(np.linalg.norm(ep.xyz - o, axis=1))
        return ep

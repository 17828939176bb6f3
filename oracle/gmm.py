"""Plain FP64 reference of EP with unknown distances (test infrastructure
only: imported by tests/ and nothing else).

General case (Sec. 4.2, learning phase): each star's photometry gives a
Gaussian mixture over components z in (l, b) = (ln s, log-extinction to
distance s) (Sec. 3, the mixture approximation of the likelihood times the
distance prior): weight w_z, mean (m_l, m_b), covariance
[[C_ll, C_lb], [C_lb, C_bb]].  The tilted distribution sums over z and
integrates over the distance s.

The site variable is a_n = ln A(s~), the log-extinction to the star's
catalogue position at distance s~.  The log-extinction at any other distance
s on the same sightline is taken from the sightline forward model at the
linearisation point fhat (the field every sightline is linearised about):
    a(s) = a_n + delta(s),  delta(s) = ln A(s; fhat) - ln A(s~; fhat),
so the extinction curve's shape along the ray is that of fhat and its level
is the site variable.  A(s) extends the star's forward model past the
star: samples t_k = k s~/T for k <= T (the star's own T = max(1,
ceil(s~/step)) equal steps, so s~ is sample T), then t_k = s~ + (k - T) step
out to the last sample inside the cube, K_max; A(s) is the trapezoid sum
over the samples up to the last one at or below s, t_K, plus the partial
trapezoid from t_K to s:
    A(s) = A_lat(K) + (s - t_K)/2 (e^{F(t_K)} + e^{F(s)}).
Distances past the point where the ray leaves the cube carry no
likelihood.

For one component and one distance l = ln s the likelihood in a_n is
N(l; m_l, C_ll) N(a_n + delta(l); mu_b(l), v_b) with mu_b(l) = m_b + (C_lb /
C_ll)(l - m_l), v_b = C_bb - C_lb^2 / C_ll, so against the cavity N(a_n;
mu_c, v_c) its normaliser and moments are closed form:
    Z(l)  = N(l; m_l, C_ll) N(y(l); mu_c, v_c + v_b),  y = mu_b - delta,
    E[a | l] = (v_b mu_c + v_c y) / (v_c + v_b),  Var[a | l] = v_c v_b / (v_c + v_b).
The integral over l is a composite Gauss-Legendre rule: PANELS equal panels
of GL_NODES nodes on [m_l - WIDTH sd, min(m_l + WIDTH sd, ln s_exit)],
sd = sqrt(C_ll).  A component with C_ll = C_lb = 0 has a known distance:
one node at l = m_l (if inside the cube).  The tilted moments mix the nodes
of every component (log-sum-exp).
"""
from __future__ import annotations

import math

import numpy as np

from .epo import DenseEP
from .maps import point_weights

NCOMP = 6        # per component: weight, m_l, m_b, C_ll, C_lb, C_bb
PANELS = 16      # equal panels over each component's distance range
GL_NODES = 16    # Gauss-Legendre nodes per panel
WIDTH = 8.0      # half-width of the range in distance sd (ln s)

_GLX, _GLW = np.polynomial.legendre.leggauss(GL_NODES)


class Ray:
    """One star's sightline extended past the star to the cube's face, and
    the extinction A(s) along it at a field f (forward model above)."""

    def __init__(self, cfg, x):
        self.cfg = cfg
        L = float(cfg["box_pc"])
        self.o = np.asarray(cfg["observer_pc"], dtype=np.float64)
        self.x = np.asarray(x, dtype=np.float64)
        dv = self.x - self.o
        self.dv = dv
        self.s_ref = math.sqrt(float(dv @ dv))
        self.step = float(cfg["los_step_pc"])
        self.T = max(1, int(math.ceil(self.s_ref / self.step)))
        self.delta = self.s_ref / self.T
        u = dv / self.s_ref
        t = []
        for a in range(3):
            if u[a] > 0:
                t.append((L - self.o[a]) / u[a])
            elif u[a] < 0:
                t.append(-self.o[a] / u[a])
        self.s_exit = max(min(t), self.s_ref)
        self.K_max = self.T + int(math.floor((self.s_exit - self.s_ref) / self.step))

    def field(self, f, frac):
        """F at the points o + frac (x - o)."""
        p = self.o[None, :] + np.asarray(frac, dtype=np.float64)[:, None] * self.dv[None, :]
        nodes, phi = point_weights(self.cfg, p)
        return np.sum(phi * f[nodes], axis=1)

    def sample_frac(self, k):
        """t_k / s~ of the samples k."""
        k = np.asarray(k, dtype=np.float64)
        return np.where(k <= self.T, k / self.T, 1.0 + (k - self.T) * self.step / self.s_ref)

    def extinction(self, f, s):
        """A(s) at the distances s (array) and A(s~)."""
        T = self.T
        k = np.arange(self.K_max + 1)
        E = np.exp(self.field(f, self.sample_frac(k)))
        C = np.cumsum(E)
        Alat = np.zeros(self.K_max + 1)
        Alat[1:T + 1] = self.delta * (C[1:T + 1] - 0.5 * (E[0] + E[1:T + 1]))
        Alat[T + 1:] = Alat[T] + self.step * (C[T + 1:] - C[T - 1] - 0.5 * (E[T] + E[T + 1:]))
        s = np.atleast_1d(np.asarray(s, dtype=np.float64))
        near = s <= self.s_ref
        Kn = np.minimum(np.floor(s / self.delta), T)
        Kf = T + np.minimum(np.floor((s - self.s_ref) / self.step), self.K_max - T)
        K = np.maximum(np.where(near, Kn, Kf), 0).astype(np.int64)
        tK = np.where(K <= T, K * self.delta, self.s_ref + (K - T) * self.step)
        Fs = self.field(f, s / self.s_ref)
        A = Alat[K] + 0.5 * (s - tK) * (E[K] + np.exp(Fs))
        return A, Alat[T]


def component_nodes(comp, ln_exit):
    """Distance nodes l and weights W of one component's rule, and whether
    the component is a known distance (no N(l) factor)."""
    w, ml, mb, cll, clb, cbb = comp
    if cll == 0.0:
        if ml > ln_exit:
            return np.zeros(0), np.zeros(0), True
        return np.array([ml]), np.array([1.0]), True
    sd = math.sqrt(cll)
    lo = ml - WIDTH * sd
    hi = min(ml + WIDTH * sd, ln_exit)
    if not hi > lo:
        return np.zeros(0), np.zeros(0), False
    h = (hi - lo) / PANELS
    p = np.arange(PANELS)[:, None]
    l = lo + h * (p + 0.5 * (1.0 + _GLX[None, :]))
    W = np.broadcast_to(0.5 * h * _GLW[None, :], l.shape)
    return l.ravel(), W.ravel().copy(), False


def tilted_one(ray: Ray, f, mu_c, v_c, comps):
    """(ln Z, mean, var) of the tilted distribution in a_n for one star."""
    ln_exit = math.log(ray.s_exit)
    logs, means, vars_ = [], [], []
    for comp in comps:
        w, ml, mb, cll, clb, cbb = [float(v) for v in comp]
        if not w > 0:
            continue
        l, W, known = component_nodes(comp, ln_exit)
        if l.size == 0:
            continue
        A, A_ref = ray.extinction(f, np.exp(l))
        dlt = np.log(A) - math.log(A_ref)
        if known:
            mub, vb, lN = mb, cbb, 0.0
        else:
            mub = mb + (clb / cll) * (l - ml)
            vb = cbb - clb * clb / cll
            lN = -0.5 * math.log(2 * math.pi * cll) - 0.5 * (l - ml) ** 2 / cll
        y = mub - dlt
        S = v_c + vb
        logs.append(math.log(w) + np.log(W) + lN - 0.5 * math.log(2 * math.pi * S) - 0.5 * (y - mu_c) ** 2 / S)
        means.append((vb * mu_c + v_c * y) / S)
        vars_.append(np.full(l.shape, v_c * vb / S))
    if not logs:
        return -math.inf, math.nan, math.nan
    lg = np.concatenate(logs)
    m = np.concatenate(means)
    v = np.concatenate(vars_)
    top = float(np.max(lg))
    r = np.exp(lg - top)
    Z = float(np.sum(r))
    mean = float(np.sum(r * m) / Z)
    var = float(np.sum(r * (v + (m - mean) ** 2)) / Z)
    return top + math.log(Z), mean, var


def gmm_tilted(cfg, xyz, f, mu_c, v_c, comps):
    """Tilted moments of every star (Python loop: small cases only)."""
    xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
    comps = np.asarray(comps, dtype=np.float64).reshape(xyz.shape[0], -1, NCOMP)
    f = np.asarray(f, dtype=np.float64)
    out = np.array([tilted_one(Ray(cfg, xyz[n]), f, float(mu_c[n]), float(v_c[n]), comps[n])
                    for n in range(xyz.shape[0])])
    return out[:, 0], out[:, 1], out[:, 2]


class DenseEPGMM(DenseEP):
    """DenseEP whose per-star likelihood is the distance-marginalised
    mixture, with delta(s) at the linearisation point of the sweep."""

    def __init__(self, cfg, xyz, comps, sightlines=None, vecchia=None):
        S = len(np.atleast_2d(xyz))
        super().__init__(dict(cfg, likelihood="extinction"), xyz, np.zeros(S), np.ones(S),
                         sightlines=sightlines, vecchia=vecchia)
        self.xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
        self.comps = np.asarray(comps, dtype=np.float64).reshape(S, -1, NCOMP)

    def sweep(self) -> dict:
        mu, Sigma, G, c = self.posterior()
        fhat = self.fhat
        m = c + G @ mu
        v = np.einsum("ij,ij->i", G @ Sigma, G)
        tau_c = 1.0 / v - self.tau
        nu_c = m / v - self.nu
        ok = tau_c > 0.0
        v_c = np.where(ok, np.maximum(1.0 / np.where(ok, tau_c, 1.0), self.vfloor), 1.0)
        mu_c = np.where(ok, nu_c / np.where(ok, tau_c, 1.0), 0.0)
        tau_c, nu_c = 1.0 / v_c, mu_c / v_c
        lnZ, mh, vh = gmm_tilted(self.cfg, self.xyz, fhat, mu_c, v_c, self.comps)
        with np.errstate(divide="ignore", invalid="ignore"):
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
                    skipped_negsite=int((ok & ~good).sum()), max_dtau=float(np.max(np.abs(self.tau - old_tau))),
                    max_dmu=dmu, cav_mu=mu_c, cav_var=v_c, lnZ=lnZ, tilted_mean=mh, tilted_var=vh)


class DenseEPThetaGMM:
    """The inferred-mean EP (meanfn.DenseEPTheta) with the distance-mixture
    likelihood: delta(s) at the linearisation point fhat = m(phihat) + deltahat."""

    def __new__(cls, cfg, xyz, comps, sightlines=None, vecchia=None):
        from .meanfn import DenseEPTheta

        class _Impl(DenseEPTheta):
            def tilted_moments(self, mu_c, v_c):
                return gmm_tilted(self.cfg, self.xyz, self.fhat, mu_c, v_c, self.comps)

        S = len(np.atleast_2d(xyz))
        ep = _Impl(dict(cfg, likelihood="extinction"), xyz, np.zeros(S), np.ones(S), sightlines=sightlines,
                   vecchia=vecchia)
        ep.xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
        ep.comps = np.asarray(comps, dtype=np.float64).reshape(S, -1, NCOMP)
        return ep

"""Workload presets and seeded raw draws.

The paper's own test catalogue (simulated Gaia stars in a thin anticentre
letter-box, Sec. 5) is not available; these synthetic workloads stand in for it.
Each preset fixes a grid, a prior and a star sample:

* stars either uniform in the cube, or from an exponential disc seen from an
  observer at the centre of the y = 0 face looking along +y (the anticentre
  direction, as in Sec. 5): density proportional to
  exp(-y / 2.6 kpc - |z - L/2| / 0.3 kpc), restricted to |b| <= 10 degrees
  (sin b = (z - L/2) / d) and d <= d_max, by rejection to an exact count;
* per-star noise scales sigma (1-sigma, in mag) from the preset's law;
* standard-normal deviates for the field (one per node) and for the
  observation noise (one per star).

Seeds: numpy PCG64 with seed 17080000 + 100 * preset + {0 field, 1 positions,
2 noise, 3 the synthetic distance-extinction mixtures}.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 17080000


@dataclasses.dataclass
class Workload:
    name: str
    n: int                      # nodes per axis
    box_pc: float               # cube side L
    n_stars: int
    sweeps: int
    star_law: str = "uniform"   # "uniform" or "disc"
    d_max_pc: float = 0.0       # disc law: truncation distance
    b_max_deg: float = 10.0     # disc law: latitude cut
    disc_scale_length_pc: float = 2600.0
    disc_scale_height_pc: float = 300.0
    noise_law: str = "const"    # "const", "uniform", "linear"
    noise_a: float = 0.05       # const value / uniform low / linear intercept
    noise_b: float = 0.0        # uniform high / linear slope per kpc
    prior_mean: float = -7.0    # ln(mag/pc)
    prior_var: float = 1.0
    outer_scale_pc: float = 100.0
    support_pc: float = 150.0
    vecchia_radius_pc: float = 0.0   # 0: equal to the support radius
    los_step_pc: float = 2.0
    likelihood: str = "extinction"   # or "gauss_linear"
    precision: str = "fp64"
    moments: str = "quadrature"
    damping: float = 1.0
    relin_step: float = 1.0     # linearisation step (1: onto the posterior mean)
    cavity_var_floor: float = 0.0
    seed_id: int = 1

    @property
    def N(self) -> int:
        return self.n ** 3

    @property
    def h(self) -> float:
        return self.box_pc / (self.n - 1)

    @property
    def observer(self):
        return (0.5 * self.box_pc, 0.0, 0.5 * self.box_pc)

    def ep_fields(self) -> dict:
        """The fields both EP implementations take as their configuration."""
        return dict(
            n=self.n, box_pc=self.box_pc, observer_pc=self.observer,
            prior_mean=self.prior_mean, prior_var=self.prior_var,
            outer_scale_pc=self.outer_scale_pc, support_pc=self.support_pc,
            vecchia_radius_pc=self.vecchia_radius_pc or self.support_pc,
            los_step_pc=self.los_step_pc, likelihood=self.likelihood,
            precision=self.precision, moments=self.moments,
            damping=self.damping, relin_step=self.relin_step, cavity_var_floor=self.cavity_var_floor)


PRESETS = {
    1: Workload("cfg1-16cube-1k", n=16, box_pc=1000.0, n_stars=1000, sweeps=10,
                star_law="uniform", noise_law="const", noise_a=0.05, seed_id=1),
    2: Workload("cfg2-64cube-100k", n=64, box_pc=4000.0, n_stars=100_000, sweeps=20,
                star_law="disc", d_max_pc=4000.0, noise_law="uniform",
                noise_a=0.05, noise_b=0.2, relin_step=0.5, seed_id=2),
    3: Workload("cfg3-128cube-1M", n=128, box_pc=8000.0, n_stars=1_000_000, sweeps=20,
                star_law="disc", d_max_pc=8000.0, noise_law="linear",
                noise_a=0.02, noise_b=0.03, precision="mixed", relin_step=0.5, seed_id=3),
    4: Workload("cfg4-128cube-1M-surrogate", n=128, box_pc=8000.0, n_stars=1_000_000, sweeps=20,
                star_law="disc", d_max_pc=8000.0, noise_law="linear",
                noise_a=0.02, noise_b=0.03, precision="mixed", moments="surrogate", relin_step=0.5, seed_id=4),
    # positions from the disc law; the G < 17 magnitude cut needs the
    # extinction along each sightline and is applied when observations are
    # simulated, not here
    5: Workload("cfg5-256cube-10M", n=256, box_pc=8000.0, n_stars=10_000_000, sweeps=10,
                star_law="disc", d_max_pc=8000.0, noise_law="uniform", noise_a=0.03, noise_b=0.3,
                support_pc=120.0, precision="mixed", moments="surrogate", relin_step=0.5, seed_id=5),
}


def preset(i: int, **over) -> Workload:
    """A preset, optionally with fields replaced (e.g. a smaller star count)."""
    return dataclasses.replace(PRESETS[i], **over)


def _disc_positions(w: Workload, rng: np.random.Generator, count: int) -> np.ndarray:
    L = w.box_pc
    ox, oy, oz = w.observer
    sinb = math.sin(math.radians(w.b_max_deg))
    ymax = min(L, w.d_max_pc)
    out = []
    have = 0
    while have < count:
        m = max(4 * (count - have), 4096)
        # y: exponential, truncated to [0, ymax] (inverse cdf)
        u = rng.random(m)
        hl = w.disc_scale_length_pc
        y = -hl * np.log1p(-u * (1.0 - math.exp(-ymax / hl)))
        # z - L/2: Laplace, truncated to [-L/2, L/2]
        u = rng.random(m)
        hz = w.disc_scale_height_pc
        az = -hz * np.log1p(-u * (1.0 - math.exp(-0.5 * L / hz)))
        sgn = np.where(rng.random(m) < 0.5, -1.0, 1.0)
        z = oz + sgn * az
        x = rng.random(m) * L
        d = np.sqrt((x - ox) ** 2 + (y - oy) ** 2 + (z - oz) ** 2)
        ok = (d <= w.d_max_pc) & (d > 0.0) & (np.abs(z - oz) <= sinb * d)
        sel = np.stack([x[ok], y[ok], z[ok]], axis=1)
        out.append(sel)
        have += sel.shape[0]
    return np.concatenate(out, axis=0)[:count]


def draw(w: Workload, n_stars: int | None = None, field: bool = True) -> dict:
    """Raw seeded draws for a workload.

    Returns a dict with
      xyz    (S, 3) star positions in the cube frame, pc
      sigma  (S,)   1-sigma observation noise, mag
      eps    (S,)   standard-normal noise deviates
      xi     (N,)   standard-normal field deviates (if field=True)
    """
    S = w.n_stars if n_stars is None else n_stars
    rng_pos = np.random.Generator(np.random.PCG64(SEED_BASE + 100 * w.seed_id + 1))
    rng_noise = np.random.Generator(np.random.PCG64(SEED_BASE + 100 * w.seed_id + 2))
    if w.star_law == "uniform":
        xyz = rng_pos.random((S, 3)) * w.box_pc
    elif w.star_law == "disc":
        xyz = _disc_positions(w, rng_pos, S)
    else:
        raise ValueError(w.star_law)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    d = np.sqrt(((xyz - np.asarray(w.observer)) ** 2).sum(axis=1))
    if w.noise_law == "const":
        sigma = np.full(S, w.noise_a)
    elif w.noise_law == "uniform":
        sigma = w.noise_a + (w.noise_b - w.noise_a) * rng_noise.random(S)
    elif w.noise_law == "linear":
        sigma = w.noise_a + w.noise_b * d / 1000.0
    else:
        raise ValueError(w.noise_law)
    eps = rng_noise.standard_normal(S)
    out = dict(xyz=xyz, sigma=np.ascontiguousarray(sigma, dtype=np.float64),
               eps=np.ascontiguousarray(eps, dtype=np.float64))
    if field:
        rng_f = np.random.Generator(np.random.PCG64(SEED_BASE + 100 * w.seed_id + 0))
        out["xi"] = rng_f.standard_normal(w.N)
    return out


def gmm_catalogue(w: Workload, xyz_true: np.ndarray, a_true: np.ndarray, weight_main: float = 0.75,
                  sd_l: float = 0.15, sd_b: float = 0.08, rho: float = 0.6,
                  alias_l: float = math.log(2.5), alias_b: float = 0.25) -> dict:
    """Synthetic per-star photometric likelihoods with unknown distance: a
    two-component Gaussian mixture in (l, b) = (ln distance, log-extinction)
    per star (the paper's real mixtures come from stellar models and are not
    available).  The main component (weight weight_main) is centred on a
    draw around the truth (l_true, a_true) with covariance
    C = [[sd_l^2, rho sd_l sd_b], [., sd_b^2]]; the alias component is the
    same shifted by (alias_l, alias_b), as for a dwarf / giant confusion.
    The catalogue position is the true direction at the main component's
    distance, pulled inside the cube.  a_true (the log-extinction at the true
    position) is an input: this module does no extinction arithmetic.

    Returns dict(xyz=(S, 3) catalogue positions, comps=(S, 2, 6) rows
    (weight, m_l, m_b, C_ll, C_lb, C_bb))."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 100 * w.seed_id + 3))
    xyz_true = np.asarray(xyz_true, dtype=np.float64)
    S = xyz_true.shape[0]
    o = np.asarray(w.observer, dtype=np.float64)
    dv = xyz_true - o
    d = np.linalg.norm(dv, axis=1)
    u = dv / d[:, None]
    cll, clb, cbb = sd_l ** 2, rho * sd_l * sd_b, sd_b ** 2
    z1 = rng.standard_normal(S)
    z2 = rng.standard_normal(S)
    nl = sd_l * z1
    nb = sd_b * (rho * z1 + math.sqrt(1 - rho * rho) * z2)
    comps = np.zeros((S, 2, 6))
    comps[:, 0] = np.stack([np.full(S, weight_main), np.log(d) + nl, a_true + nb,
                            np.full(S, cll), np.full(S, clb), np.full(S, cbb)], axis=1)
    comps[:, 1] = comps[:, 0]
    comps[:, 1, 0] = 1.0 - weight_main
    comps[:, 1, 1] += alias_l
    comps[:, 1, 2] += alias_b
    # largest distance along u that stays in the cube
    with np.errstate(divide="ignore", invalid="ignore"):
        tmax = np.where(u > 0, (w.box_pc - o) / u, np.where(u < 0, -o / u, np.inf))
    dmax = np.min(tmax, axis=1)
    dref = np.clip(np.exp(comps[:, 0, 1]), 1.0, 0.999 * dmax)
    return dict(xyz=np.ascontiguousarray(o + u * dref[:, None]), comps=np.ascontiguousarray(comps))


def sky_cells(w: Workload, xyz: np.ndarray, n_lon: int, n_lat: int) -> np.ndarray:
    """On-sky cell of each point, as the sub-catalogue partition (Sec. 4.1):
    equal-angle cells in longitude (-90, 90) deg about the +y axis and in
    latitude (-b_max, b_max), cell = i_lon * n_lat + i_lat, points outside
    the latitude band clamped to the nearest cell (the observer itself to
    latitude 0)."""
    o = np.asarray(w.observer)
    v = np.asarray(xyz, dtype=np.float64) - o
    d = np.sqrt((v ** 2).sum(axis=1))
    lon = np.degrees(np.arctan2(v[:, 0], v[:, 1]))
    lat = np.degrees(np.arcsin(np.divide(v[:, 2], d, out=np.zeros_like(d), where=d > 0)))
    il = np.clip(np.floor((lon + 90.0) / 180.0 * n_lon), 0, n_lon - 1).astype(np.int64)
    bm = w.b_max_deg
    ib = np.clip(np.floor((lat + bm) / (2 * bm) * n_lat), 0, n_lat - 1).astype(np.int64)
    return (il * n_lat + ib).astype(np.int32)


def node_positions(w: Workload) -> np.ndarray:
    p = np.arange(w.N)
    return np.stack([p % w.n, (p // w.n) % w.n, p // (w.n * w.n)], axis=1) * w.h


def boundary_inducing(w: Workload, n_lon: int, n_lat: int, dists_pc) -> np.ndarray:
    """Inducing points on the sub-catalogue boundaries at fixed distances
    (Sec. 5 places them on the boundaries between sub-catalogues at 1-4 kpc):
    the corner directions of the on-sky cells times each distance, snapped
    to the nearest grid node; points outside the cube dropped, duplicates
    removed (sorted node ids)."""
    o = np.asarray(w.observer)
    lons = np.radians(np.linspace(-90.0, 90.0, n_lon + 1))
    lats = np.radians(np.linspace(-w.b_max_deg, w.b_max_deg, n_lat + 1))
    pts = []
    for d in dists_pc:
        for lo in lons:
            for la in lats:
                pts.append(o + d * np.array([math.cos(la) * math.sin(lo), math.cos(la) * math.cos(lo), math.sin(la)]))
    pts = np.array(pts)
    inside = np.all((pts >= 0.0) & (pts <= w.box_pc), axis=1)
    ijk = np.rint(pts[inside] / w.h).astype(np.int64)
    ids = ijk[:, 0] + w.n * (ijk[:, 1] + w.n * ijk[:, 2])
    return np.unique(ids).astype(np.int32)

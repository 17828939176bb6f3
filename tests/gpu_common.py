"""Shared set-up for the GPU parity tests (inputs from the seeded draws and
the oracle's own forward model; expected values from the oracle only)."""
import numpy as np

from oracle import epo
from synth import Workload, draw


def small_case(n=10, L=600.0, stars=150, leaf=48, lik="extinction", relin=True, damping=1.0, seed=91,
               law="uniform"):
    w = Workload("small", n=n, box_pc=L, n_stars=stars, sweeps=3, star_law=law, d_max_pc=L,
                 noise_law="const", noise_a=0.05, likelihood=lik, seed_id=seed, damping=damping)
    cfg = w.ep_fields()
    cfg["relinearize"] = relin
    raw = draw(w)
    f_true, A, sl = epo.simulate(cfg, raw)
    gcfg = dict(cfg)
    gcfg["leaf_size"] = leaf
    return cfg, gcfg, raw, f_true, A, sl


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))

"""Train the tilted-moment surrogate on cavity/observation tuples from EP runs.

Runs plain EP (quadrature moments) on the 64^3 / 100,000-star workload with
the library, collects after every sweep each star's cavity (mu_c, v_c), its
observation (A, sigma) and the quadrature's tilted moments (ln Z, mean,
variance), trains the network with the library's kernels, measures the
gate's acceptance rate on tuples from a different seed, and saves the
weights (float32, EP_MLP_NPARAM values) next to this file.

    python -m paper_1708_09705_amd.train_surrogate [--sweeps 20] [--seeds 2 12]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "surrogate_64cube.npy")


def collect(seed_id: int, sweeps: int, leaf: int = 512, log=print):
    from synth import draw, preset
    from . import ep as E
    w = preset(2, seed_id=seed_id)
    raw = draw(w)
    cfg = E.make_config(w.ep_fields(), leaf_size=leaf)
    f, A = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    g = E.EP(cfg, raw["xyz"], A, raw["sigma"])
    X, Y = [], []
    for s in range(sweeps):
        st = g.sweep()
        ss = g.star_state()
        ok = np.isfinite(ss["tilted_var"]) & (ss["tilted_var"] > 0) & (ss["cav_var"] > 0)
        X.append(np.stack([ss["cav_mu"], ss["cav_var"], A, raw["sigma"]], 1)[ok])
        Y.append(np.stack([ss["lnZ"], ss["tilted_mean"], ss["tilted_var"]], 1)[ok])
        log(f"seed {seed_id} sweep {s}: {int(ok.sum())} tuples, {st['ms_total']:.0f} ms")
    g.close()
    return np.concatenate(X), np.concatenate(Y)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--seeds", type=int, nargs="+", default=[2, 12])
    ap.add_argument("--holdout-seed", type=int, default=22)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    from . import ep as E
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    Xs, Ys = [], []
    for sd in args.seeds:
        x, y = collect(sd, args.sweeps, log=log)
        Xs.append(x)
        Ys.append(y)
    X, Y = np.concatenate(Xs), np.concatenate(Ys)
    log(f"training on {len(X)} tuples")
    t0 = time.perf_counter()
    w, loss = E.ep_mlp_train(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=7)
    t_train = time.perf_counter() - t0
    log(f"trained in {t_train:.1f} s; loss per epoch {np.round(loss, 5).tolist()}")
    Xh, Yh = collect(args.holdout_seed, 4, log=log)
    out, err, acc = E.ep_mlp_predict(w, Xh, tol=1e-4)
    _, _, acc0 = E.ep_mlp_predict(None, Xh, tol=1e-4)
    d = np.abs(out[acc] - Yh[acc])
    report = {"tuples": int(len(X)), "epochs": args.epochs, "train_seconds": t_train, "loss": loss.tolist(),
              "holdout": int(len(Xh)), "accept_rate": float(acc.mean()),
              "accept_rate_baseline_centre": float(acc0.mean()),
              "accepted_max_abs_err": [float(x) for x in (d.max(0) if len(d) else [np.nan] * 3)]}
    np.save(args.out, w)
    print(json.dumps(report), flush=True)


if __name__ == "__main__":
    main()

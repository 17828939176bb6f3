"""Benchmark: EP star-updates per second on one MI355X.

One step = one full parallel EP sweep (line-of-sight linearisation, assembly,
multifrontal Cholesky, solves, selected inversion, cavity, tilted moments and
site update for every star) of the 64^3-grid / 100,000-star workload (4 kpc
cube, disc-distributed stars, sigma ~ U[0.05, 0.2] mag), FP64 throughout.

value = stars x steps / wall time of the timed steps (whole sweeps; inputs
resident on the device).  The JSON line also carries the per-star-phase rate
(stars / time of cavity + tilted moments + site update), the per-phase
times, the dense-front MFMA roofline, the two mixed-precision forms of the
same sweeps (FP32 factor; FP32 selected inversion with FP64 partial sums),
each with quadrature and with the surrogate and with its error against the
FP64 run, and the oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the dominant kernel (k_gemm_tasks<false>, every
# launch of one FP64 sweep of the 64^3 / 100,000-star workload): rocprofv3
# FETCH_SIZE and WRITE_SIZE summed over the sweep's 186 launches, each scaled
# by what the same counter reads for a 1 GiB device copy (FETCH_SIZE x 2.000,
# WRITE_SIZE x 1.000), divided by 186.  Taken for the kernel and task lists
# as they are; set to None whenever either changes until the counters are
# taken again.
TRAFFIC_GEMM_TASKS = {"fetch_bytes_per_launch": 1.5179e12 / 186, "write_bytes_per_launch": 8.6965e10 / 186,
                      "bytes_per_launch": (1.5179e12 + 8.6965e10) / 186, "launches_per_sweep": 186,
                      "source": "profiles/k_gemm_tasks_64cube_100k_traffic.md"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(preset_id: int, n_sample: int, repeats: int = 3) -> dict:
    """The oracle (plain FP64 C + numpy, unchanged) performing first-sweep star
    updates for a sample of the same workload, timed by phase (median of
    repeats): the line-of-sight linearisation at the prior mean, the cavity
    (with zero sites the prior marginal: g^T Q0^{-1} g by Vecchia
    back-substitution), adaptive Gauss-Kronrod tilted moments and the site
    update."""
    from oracle import epo
    from synth import draw, preset
    w = preset(preset_id)
    cfg = w.ep_fields()
    raw = draw(w)
    t0 = time.perf_counter()
    vec = epo.Vecchia(cfg)
    f_true = vec.draw(cfg["prior_mean"], raw["xi"])
    t_prior = time.perf_counter() - t0
    idx = np.arange(min(n_sample, w.n_stars))
    sl = epo.Sightlines(cfg, raw["xyz"][idx])
    _, lnA_true, _ = sl.linearise(f_true)
    A = np.exp(lnA_true) + raw["sigma"][idx] * raw["eps"][idx]
    runs = []
    for _ in range(repeats):
        t = [time.perf_counter()]
        gval, lnA, c = sl.linearise(np.full(sl.grid.N, cfg["prior_mean"]))
        t.append(time.perf_counter())
        v = vec.prior_quadform(sl.ptr, sl.nodes, gval)
        t.append(time.perf_counter())
        lnZ, mh, vh = epo.tilted(0, lnA, v, A, raw["sigma"][idx])
        t.append(time.perf_counter())
        tau = 1 / vh - 1 / v
        nu = mh / vh - lnA / v
        t.append(time.perf_counter())
        runs.append(np.diff(t))
        assert np.all(np.isfinite(tau)) and np.all(np.isfinite(nu))
    med = np.median(np.array(runs), axis=0)
    dt = float(np.sum(med))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(idx) / dt, "unit": "star-updates/s", "cores": cores, "kind": "oracle",
            "phases_ms": {"linearise": 1e3 * med[0], "cavity": 1e3 * med[1], "tilted": 1e3 * med[2],
                          "site_update": 1e3 * med[3]},
            "star_phase_updates_per_s": len(idx) / float(np.sum(med[1:])),
            "repeats": repeats,
            "sample": f"first-sweep star updates of {len(idx)} stars of the same 64^3/100k workload "
                      f"(LOS linearisation, g^T Q0^-1 g by Vecchia back-substitution, adaptive "
                      f"Gauss-Kronrod tilted moments, site update); median of {repeats} runs, {dt:.1f} s each; "
                      f"prior set-up {t_prior:.1f} s not counted.  The oracle cannot run the factor or the "
                      f"selected inversion at this size (dense algebra on 262,144 nodes)"}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "ms_per_copy": dt * 1e3, "GBps_read_plus_write": 2 * nbytes / dt / 1e9}), flush=True)


# measured FP64 rate of the dominant task-GEMM kernel on the 64^3 / 100k sweep
# (55 TFLOP/s): the plan's sweep-time estimate divides its MFMA work by it
MEASURED_GEMM_TFLOPS = 55.0
HBM_BYTES = 288e9


def sparse_kernels(st, stats, N) -> dict:
    """Achieved bandwidth of the sparse kernels on their algorithmic bytes
    (what each must move at least once per sweep), from the per-launch HIP
    events of the timed sweeps."""
    S = st["n_stars"]
    algo = {
        # the fronts' lower-triangular tiles, written once
        "zero": 8 * st["front_elems_lower"],
        # every clique entry read and written (FP64 atomic add); g and the local row per slot
        "assemble": 16 * st["clique_pairs"] + 12 * st["nnz_g"],
        # every update-block entry: read in the child, read and written in the parent
        "extend": 24 * st["update_elems"],
        # every update-block entry of Sigma: read in the parent, written in the child
        "gather": 16 * st["update_elems"],
        # every clique entry of Sigma read once; per slot g, local row, slot order, node and mu
        "cavity": 8 * st["clique_pairs"] + 28 * st["nnz_g"] + 40 * S,
        # one solve: the factor's pivot-block inverses and off-diagonal blocks, forward and backward
        "solve": 16 * (st["x_elems"] + st["offdiag_elems"]) + 6 * 8 * N,
    }
    out = {}
    for k, b in algo.items():
        ms = float(np.mean([s_["kernel_ms"][k] for s_ in stats]))
        if ms <= 0:
            continue
        gbs = b / (ms * 1e-3) / 1e9
        out[k] = {"ms_per_step": ms, "launches_per_step": int(stats[-1]["kernel_launches"][k]),
                  "algorithmic_bytes_per_step": int(b), "GBps": gbs, "frac_of_hbm_peak": gbs / PEAK_HBM_GBS}
    out["note"] = ("zero: k_zero_lower; assemble: k_sort_g + k_assemble_tiles + k_tiles_reduce (tile owner, LDS); "
                   "extend: k_extend_add; "
                   "gather: k_sigma_gather; cavity: k_cavity; solve: k_fwd_xv/k_fwd_r/k_bwd_t/k_bwd_x")
    return out


def scaled_workload(w, n):
    """The workload on an n^3 grid at the same spacing: the cube side and the
    star-distance cut scale with (n - 1)."""
    import dataclasses
    box = w.box_pc / (w.n - 1) * (n - 1)
    return dataclasses.replace(w, n=n, box_pc=box, d_max_pc=min(w.d_max_pc, box) if w.d_max_pc else box,
                               name=f"{n}cube-{w.n_stars // 1000}k-at-{box / (n - 1):.1f}pc")


def variant_workload():
    """The largest single-GPU variant of the 128^3 / 1M-star workload: the
    same spacing (63 pc), prior, star law and count, on 80^3 nodes (5 kpc)."""
    from synth import preset
    import dataclasses
    return dataclasses.replace(scaled_workload(preset(3), 80), precision="fp64", moments="quadrature")


def plan_of(w) -> dict:
    """Host structure analysis (ep_plan: no device) of a workload."""
    from paper_1708_09705_amd import ep as E
    from synth import draw
    raw = draw(w, field=False)
    t0 = time.perf_counter()
    p = E.ep_plan(w.ep_fields(), raw["xyz"])
    mfma = p["trail_flops"] + p["selinv_flops"]
    return {**p, "factor_bytes_fp64": 8 * p["nnz_L"], "front_bytes_full_squares": 8 * p["front_elems"],
            "front_bytes_lower_tiles": 8 * p["front_elems_lower"],
            "fits_one_gpu_fp64": p["device_bytes"] <= HBM_BYTES,
            "fits_one_gpu_mixed": p["device_bytes_mixed"] <= HBM_BYTES,
            "mfma_flop_per_sweep": mfma,
            "est_gemm_s_per_sweep": mfma / (MEASURED_GEMM_TFLOPS * 1e12),
            "plan_seconds": time.perf_counter() - t0,
            "note": "device_bytes counts ep_init's allocations without the GEMM task lists; "
                    f"est_gemm_s_per_sweep = MFMA flop / {MEASURED_GEMM_TFLOPS} TFLOP/s (the rate measured at 64^3)"}


THETA_TRUE = (2500.0, 200.0, 1.2e-3, 1800.0, 0.15)   # (L, H, rho kappa_0, s_bump, A_bump) of the synthetic sky


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--preset", type=int, default=2)
    ap.add_argument("--stars", type=int, default=0, help="override the star count (testing)")
    ap.add_argument("--leaf", type=int, default=512)
    ap.add_argument("--cpu-sample", type=int, default=50000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false",
                    help="skip the surrogate + mixed-precision run (FP32 factor + FP64 refinement, "
                         "network moments with quadrature fallback)")
    ap.add_argument("--no-gmm", dest="gmm", action="store_false",
                    help="skip the sweeps with unknown distances (per-star distance / extinction mixtures)")
    ap.add_argument("--no-theta", dest="theta", action="store_false",
                    help="skip the sweeps with the inferred disc + bump prior mean")
    ap.add_argument("--no-pitc", dest="pitc", action="store_false",
                    help="skip the PITC sub-catalogue EP (the paper's inducing-point approximation)")
    ap.add_argument("--pitc-only", action="store_true",
                    help="run only the PITC leg and print its JSON object (for profiling it alone)")
    ap.add_argument("--no-maps", dest="maps", action="store_false",
                    help="skip timing the map predictions after the FP64 run")
    ap.add_argument("--side-steps", type=int, default=5,
                    help="timed sweeps of every side leg (mixed, surrogate, gmm, theta)")
    ap.add_argument("--no-variant", dest="variant", action="store_false",
                    help="skip the largest single-GPU variant of the 128^3 / 1M-star workload")
    ap.add_argument("--no-plan", dest="plan_in_line", action="store_false",
                    help="skip the host structure analysis of the 128^3 / 1M-star workload")
    ap.add_argument("--plan", action="store_true",
                    help="CPU only: print the structure, work and memory of --preset (host analysis, no device) "
                         "and exit")
    ap.add_argument("--plan-n", type=int, default=0,
                    help="with --plan: another grid size at the preset's spacing (box and star distances scaled)")
    ap.add_argument("--plan-rho", type=float, default=0.0,
                    help="with --plan: another Vecchia conditioning radius (pc)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the reference kernel that "
                         "scales the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.plan:
        from synth import preset
        w = preset(args.preset) if not args.stars else preset(args.preset, n_stars=args.stars)
        if args.plan_n:
            w = scaled_workload(w, args.plan_n)
        if args.plan_rho:
            import dataclasses
            w = dataclasses.replace(w, vecchia_radius_pc=args.plan_rho, name=f"{w.name}-rho{args.plan_rho:g}")
        print(json.dumps({"workload": w.name, "grid": f"{w.n}^3", "box_pc": w.box_pc, "stars": w.n_stars,
                          **plan_of(w)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              f"design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "no GPU"
    from paper_1708_09705_amd import ep as E
    from synth import draw, preset

    w = preset(args.preset) if not args.stars else preset(args.preset, n_stars=args.stars)
    raw = draw(w)
    cfg = E.make_config(w.ep_fields(), leaf_size=args.leaf, device=0, profile_kernels=1)
    t0 = time.perf_counter()
    f_true, A = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
    log(f"simulated {w.name}: {time.perf_counter() - t0:.1f} s")

    weights = np.load(os.path.join(ROOT, "paper_1708_09705_amd", "surrogate_64cube.npy"))

    def variant_leg():
        # the 128^3 / 1M-star workload does not fit one GPU (headline_structure);
        # this is its largest variant that does, timed the same way
        wv = variant_workload()
        rv = draw(wv)
        cv = E.make_config(wv.ep_fields(), leaf_size=args.leaf, device=0)
        t0 = time.perf_counter()
        _, Av = E.ep_simulate(cv, rv["xyz"], rv["sigma"], rv["eps"], rv["xi"])
        g = E.EP(cv, rv["xyz"], Av, rv["sigma"])
        init_s = time.perf_counter() - t0
        stv = g.structure()
        log(f"[variant {wv.name}] init {init_s:.1f} s; structure {stv}")
        for i in range(side_w):
            log(f"[variant] warmup {i}: {g.sweep()['ms_total']:.0f} ms")
        torch.cuda.synchronize()
        sts = []
        t0 = time.perf_counter()
        for i in range(max(1, side // 2)):
            sts.append(g.sweep())
            log(f"[variant] step {i}: {sts[-1]['ms_total']:.0f} ms")
        torch.cuda.synchronize()
        wv_s = time.perf_counter() - t0
        n_st = max(1, side // 2)
        phases = ("ms_linearise", "ms_assemble", "ms_factor", "ms_solve", "ms_selinv", "ms_star", "ms_total")
        out = {"workload": wv.name, "grid": f"{wv.n}^3", "box_pc": wv.box_pc, "stars": wv.n_stars,
               "value": wv.n_stars * n_st / wv_s, "unit": "star-updates/s", "ms_per_step": wv_s / n_st * 1e3,
               "steps": n_st, "warmup": side_w, "init_s": init_s,
               "phases_ms": {k: float(np.mean([s_[k] for s_ in sts])) for k in phases},
               "structure": {k: stv[k] for k in ("n_fronts", "n_levels", "front_elems", "max_front",
                                                  "factor_flops", "selinv_flops", "trail_flops", "device_bytes")},
               "note": "FP64, quadrature; the same spacing, prior and star law as 128^3 / 1M on a 5 kpc cube"}
        if not args.mixed:
            g.close()
            return out
        # the surrogate + FP32 selected inversion form of the same workload,
        # timed the same way; its error against FP64 on the FP64 run's final
        # state (one context at a time: each takes most of the HBM)
        state = (g.sites(), g.linpoint())
        m64, v64 = g.posterior_mean(), g.marginal_var()
        g.close()
        try:
            g = E.EP(E.make_config(wv.ep_fields(), leaf_size=args.leaf, device=0, precision="selinv32",
                                   moments="surrogate"), rv["xyz"], Av, rv["sigma"])
            g.load_surrogate(weights)
            for i in range(side_w):
                log(f"[variant selinv32] warmup {i}: {g.sweep()['ms_total']:.0f} ms")
            torch.cuda.synchronize()
            sts = []
            t0 = time.perf_counter()
            for i in range(n_st):
                sts.append(g.sweep())
                log(f"[variant selinv32] step {i}: {sts[-1]['ms_total']:.0f} ms")
            torch.cuda.synchronize()
            w32_s = time.perf_counter() - t0
            g.set_sites(*state[0])
            g.set_linpoint(state[1])
            m32, v32 = g.posterior_mean(), g.marginal_var()
            g.close()
            em = float(np.max(np.abs(m32 - m64) / np.abs(m64)))
            ev = float(np.max(np.abs(v32 - v64) / np.abs(v64)))
            out["surrogate_selinv32"] = {
                "value": wv.n_stars * n_st / w32_s, "unit": "star-updates/s", "ms_per_step": w32_s / n_st * 1e3,
                "steps": n_st, "warmup": side_w,
                "phases_ms": {k: float(np.mean([s_[k] for s_ in sts])) for k in phases},
                "surrogate_fallbacks": int(sts[-1]["surrogate_fallbacks"]),
                "rel_err_vs_fp64": {"posterior_mean": em, "marginal_var": ev,
                                    "kind": "max over nodes of |x - x_fp64| / |x_fp64|"},
                "meets_1e-4": bool(em <= 1e-4 and ev <= 1e-4)}
        except E.EPError as e:
            out["surrogate_selinv32"] = {"error": str(e)}
        return out

    def surrogate_gain():
        # the gate centred at the network against the gate centred at the
        # analytic baseline, on the cavities of the FP64 run's last sweep
        # (tuples no training run saw: the network was trained on other seeds)
        ss = final["star_state"]
        X = np.stack([ss["cav_mu"], ss["cav_var"], A, raw["sigma"]], axis=1)
        ok = np.isfinite(X).all(axis=1) & (X[:, 1] > 0)
        X = X[ok]
        _, _, acc_n = E.ep_mlp_predict(weights, X, tol=1e-4)
        _, _, acc_b = E.ep_mlp_predict(None, X, tol=1e-4)
        return {"tuples": int(len(X)), "accepted_network": float(acc_n.mean()),
                "accepted_baseline_only": float(acc_b.mean()),
                "fallbacks_network": int((~acc_n).sum()), "fallbacks_baseline_only": int((~acc_b).sum()),
                "note": "quadrature fallbacks with the gate (1e-4) centred at the network vs at the analytic baseline"}

    def maps_leg(g):
        # Map predictions from the converged state of the FP64 run; every call
        # recomputes q(f) (factor, solve, selected inversion) first.
        N = w.n ** 3
        out = {}
        t0 = time.perf_counter()
        g.density_moments()
        out["ms_density_moments"] = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
        g.extinction_map()
        out["ms_extinction_mean"] = (time.perf_counter() - t0) * 1e3
        K = 8
        z = np.random.default_rng(123).standard_normal((K, N))
        t0 = time.perf_counter()
        g.extinction_map(z)
        out["ms_extinction_mean_and_var"] = (time.perf_counter() - t0) * 1e3
        out["draws"] = K
        # the paper's two-point layout: every node x and x + 10 pc along the
        # observer's ray, where that point is still inside the cube
        h = w.box_pc / (w.n - 1)
        i = np.arange(N)
        x = np.stack([(i % w.n) * h, ((i // w.n) % w.n) * h, (i // (w.n * w.n)) * h], axis=1)
        o = np.asarray(w.ep_fields()["observer_pc"], dtype=np.float64)
        d = np.linalg.norm(x - o, axis=1)
        ok = d > 0
        x2 = x[ok] + 10.0 * (x[ok] - o) / d[ok][:, None]
        inside = np.all((x2 >= 0) & (x2 <= w.box_pc), axis=1)
        xyz2 = np.hstack([x[ok][inside], x2[inside]])
        t0 = time.perf_counter()
        g.point_predict(xyz2)
        out["ms_two_point_density"] = (time.perf_counter() - t0) * 1e3
        out["pairs"] = int(len(xyz2))
        out["note"] = ("each call includes the factorization, solve and selected inversion of q(f); "
                       "mean and var: exact mean plus the sample variance over the draws")
        return out

    def pitc_leg():
        # The paper's own sparse scheme on the same stars and grid: Gaussian
        # log-extinction observations (the linearised forward model at the
        # prior mean), 40 x 4 on-sky sub-catalogues, inducing nodes on their
        # boundaries at 1-4 kpc.  Timed: one sweep (every sub-catalogue's
        # conditional, the sites, q(u), the evidence) and one PIC predictive
        # of the field at all nodes.  Compared with the grid path's exact
        # posterior of the same model (one sweep is exact there).
        from synth.workloads import boundary_inducing, node_positions, sky_cells
        gl = dict(w.ep_fields(), likelihood="gauss_linear")
        c = E.make_config(gl, leaf_size=args.leaf, device=0)
        f_t, a_obs = E.ep_simulate(c, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
        blocks = sky_cells(w, raw["xyz"], 40, 4)
        u = boundary_inducing(w, 40, 4, (1000.0, 2000.0, 3000.0, 4000.0))
        nb = sky_cells(w, node_positions(w), 40, 4)
        g = E.EP(c, raw["xyz"], a_obs, raw["sigma"])
        t0 = time.perf_counter()
        g.pitc_setup(blocks, u, nb)
        setup_ms = (time.perf_counter() - t0) * 1e3
        info = g.pitc_info()
        for _ in range(args.warmup):
            g.pitc_sweep(1.0)
            g.pitc_predict()
        torch.cuda.synchronize()
        ts, tp = [], []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            lz = g.pitc_sweep(1.0)
            t1 = time.perf_counter()
            pm, pv = g.pitc_predict()
            t2 = time.perf_counter()
            ts.append(t1 - t0)
            tp.append(t2 - t1)
        sweep_ms, pred_ms = float(np.mean(ts)) * 1e3, float(np.mean(tp)) * 1e3
        g.sweep()
        gm, gv = g.posterior_mean(), g.marginal_var()
        g.close()
        # the same with the disc + bump mean's parameters in the sites, q(u, Theta),
        # on observations drawn around THETA_TRUE
        ct = E.make_config(gl, leaf_size=args.leaf, device=0, mean_fn="disc_bump")
        sim = E.make_config(gl, device=0, mean_fn="disc_bump", theta_prior=THETA_TRUE)
        _, a_th = E.ep_simulate(sim, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
        gt = E.EP(ct, raw["xyz"], a_th, raw["sigma"])
        gt.pitc_setup(blocks, u, nb)
        for _ in range(args.warmup):
            gt.pitc_sweep(1.0)
        tt = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            gt.pitc_sweep(1.0)
            tt.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        gt.pitc_predict()
        tpt = time.perf_counter() - t0
        pm_t, pc_t = gt.pitc_theta()
        info_t = gt.pitc_info()
        gt.close()
        sd_t = np.sqrt(np.diag(pc_t))
        z_pic = (f_t - pm) / np.sqrt(pv)
        z_grid = (f_t - gm) / np.sqrt(gv)
        # the extinction likelihood on the bench's own observations A: one
        # site per star under the PITC prior (sightlines at the prior mean),
        # damped 0.7, swept until the largest relative site change falls
        # below 1e-3 (at most 30 sweeps); the last steps are timed
        ge = E.EP(E.make_config(w.ep_fields(), leaf_size=args.leaf, device=0), raw["xyz"], A, raw["sigma"])
        ge.pitc_setup(blocks, u, nb)
        te, nsw, rel = [], 0, float("inf")
        tau_prev = np.zeros(w.n_stars)
        while nsw < 30 and rel > 1e-3:
            t0 = time.perf_counter()
            ge.pitc_sweep(0.7)
            te.append(time.perf_counter() - t0)
            tau = ge.sites()[0]
            rel = float(np.max(np.abs(tau - tau_prev) / np.maximum(tau, 1e-300))) if nsw else float("inf")
            tau_prev = tau
            nsw += 1
        t0 = time.perf_counter()
        pme, pve = ge.pitc_predict()
        tpe = time.perf_counter() - t0
        ge.close()
        z_ext = (f_true - pme) / np.sqrt(pve)
        return {
            "workload": f"{w.name} stars, gauss_linear observations; 160 sub-catalogues (40 x 4 on-sky cells), "
                        f"{info['n_inducing']} inducing nodes on their boundaries at 1-4 kpc",
            "setup_ms": setup_ms, "ms_sweep": sweep_ms, "ms_predict": pred_ms,
            "sweep_tflops": info["sweep_flops"] / (sweep_ms * 1e-3) / 1e12,
            "predict_tflops": info["predict_flops"] / (pred_ms * 1e-3) / 1e12,
            "info": info, "lnZ": lz,
            "vs_grid_path": {
                "max_abs_mean_diff_in_grid_sd": float(np.max(np.abs(pm - gm) / np.sqrt(gv))),
                "rms_mean_diff_in_grid_sd": float(np.sqrt(np.mean(((pm - gm) / np.sqrt(gv)) ** 2))),
                "median_var_ratio_pic_over_grid": float(np.median(pv / gv)),
                "rms_z_true_pic": float(np.sqrt(np.mean(z_pic ** 2))),
                "rms_z_true_grid": float(np.sqrt(np.mean(z_grid ** 2)))},
            "with_mean_parameters": {
                "ms_sweep": float(np.mean(tt)) * 1e3, "ms_predict": tpt * 1e3,
                "sweep_tflops": info_t["sweep_flops"] / (float(np.mean(tt))) / 1e12,
                "theta_true": list(THETA_TRUE),
                "theta_mean": [float(v) for v in np.exp(pm_t + 0.5 * sd_t ** 2)],
                "log_theta_sd": [float(v) for v in sd_t],
                "z_true": [float(v) for v in (pm_t - np.log(THETA_TRUE)) / sd_t]},
            "extinction_likelihood": {
                "sweeps": nsw, "last_max_rel_site_change": rel,
                "ms_sweep": float(np.mean(te[-min(len(te), args.steps):])) * 1e3, "ms_predict": tpe * 1e3,
                "rms_z_true": float(np.sqrt(np.mean(z_ext ** 2))),
                "note": "one Gaussian site per star under the PITC prior; ms_predict refreshes q(u) from the sites"},
            "note": ("flops: algorithmic (unpadded) dense work of the pass; the grid path uses the Vecchia "
                     "precision, PITC the tapered covariance itself (the two priors agree where the Vecchia "
                     "conditioning radius covers the taper)"),
        }

    if args.pitc_only:
        print(json.dumps({"pitc_leg": pitc_leg()}), flush=True)
        return

    def run(prec, moments="quadrature", after=None, A_in=None, extra=None, xyz_in=None, comps=None, steps=None,
            warmup=None, state=None):
        steps = args.steps if steps is None else steps
        warmup = args.warmup if warmup is None else warmup
        c = E.make_config(w.ep_fields(), leaf_size=args.leaf, device=0, profile_kernels=1, precision=prec,
                          moments=moments, **(extra or {}))
        A_run = A if A_in is None else A_in
        t0 = time.perf_counter()
        if comps is not None:
            g = E.EP(c, xyz_in)
            g.set_gmm(comps)
        else:
            g = E.EP(c, raw["xyz"], A_run, raw["sigma"])
        if moments == "surrogate":
            g.load_surrogate(weights)
        prec = f"{prec}/{moments}"
        st = g.structure()
        log(f"[{prec}] init {time.perf_counter() - t0:.1f} s; structure {st}")
        for i in range(warmup):
            s = g.sweep()
            log(f"[{prec}] warmup {i}: {s['ms_total']:.1f} ms")
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for i in range(steps):
            s = g.sweep()
            stats.append(s)
            log(f"[{prec}] step {i}: {json.dumps({k: round(v, 3) if isinstance(v, float) else v for k, v in s.items()})}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if state is not None:
            # the posterior of another run's final sites at its linearisation point
            g.set_sites(*state[0])
            g.set_linpoint(state[1])
        mean, var = (g.posterior_mean(), g.marginal_var()) if args.mixed else (None, None)
        extra = after(g) if after else None
        g.close()
        return st, stats, wall, mean, var, extra

    final = {}

    def fp64_after(g):
        final["state"] = (g.sites(), g.linpoint())
        final["star_state"] = g.star_state()
        return maps_leg(g) if args.maps else None

    st, stats, wall, mean64, var64, maps = run("fp64", after=fp64_after)
    S = w.n_stars
    value = S * args.steps / wall
    ph = {k: float(np.mean([s[k] for s in stats])) for k in
          ("ms_linearise", "ms_assemble", "ms_factor", "ms_solve", "ms_selinv", "ms_star", "ms_total")}
    # Dominant kernel: k_gemm_tasks<false>, the FP64 MFMA task-list GEMM on
    # 256 x 128 blocks.  In an FP64 sweep every one of its launches is either
    # a trailing update of the factorization (EP_KK_TRAIL) or a
    # diagonal-block inverse / selected-inversion product (EP_KK_GEMM).  Each
    # launch is timed with HIP events on the library's stream; the work
    # counted is the algorithmic (unpadded) flop count of those two parts.
    gemm_ms = float(np.mean([s["kernel_ms"]["gemm"] + s["kernel_ms"]["trail"] for s in stats]))
    launches = int(stats[0]["kernel_launches"]["gemm"] + stats[0]["kernel_launches"]["trail"])
    flops = st["selinv_flops"] + st["trail_flops"]
    achieved = flops / (gemm_ms * 1e-3) / 1e12
    trail_ms = float(np.mean([s["kernel_ms"]["trail"] for s in stats]))
    sel_ms = float(np.mean([s["kernel_ms"]["gemm"] for s in stats]))
    mfma_ms = float(np.mean([s["mfma_ms"] for s in stats]))
    all_flops = st["factor_flops"] + st["selinv_flops"]
    line = {
        "metric": "EP star-updates/sec (full sweep, plain FP64)",
        "value": value,
        "unit": "star-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded draws; exact Vecchia-prior field; library forward model)",
        "config": {"workload": w.name, "grid": f"{w.n}^3", "box_pc": w.box_pc, "stars": S,
                   "precision": "fp64", "moments": "quadrature", "parallelism": "single GPU"},
        "phases_ms": ph,
        "star_phase_updates_per_s": S / (ph["ms_star"] * 1e-3),
        "structure": {k: st[k] for k in ("n_fronts", "n_levels", "front_elems", "max_front", "factor_flops",
                                         "selinv_flops", "trail_flops", "device_bytes", "front_elems_lower",
                                         "update_elems", "offdiag_elems", "x_elems", "clique_pairs", "nnz_g")},
        "sparse_kernels": sparse_kernels(st, stats, w.n ** 3),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": TRAFFIC_GEMM_TASKS["bytes_per_launch"] if TRAFFIC_GEMM_TASKS else None,
                     "traffic_unit": "HBM bytes per launch", "traffic_detail": TRAFFIC_GEMM_TASKS,
                     "kernel": "k_gemm_tasks<false> (FP64 MFMA, 256x128 blocks: trailing updates, "
                               "diagonal-block inverses, selected inversion)",
                     "launches_per_step": launches, "kernel_ms_per_step": gemm_ms,
                     "avg_launch_ms": gemm_ms / max(launches, 1),
                     "algorithmic_flop_per_step": flops,
                     "others": {
                         "trailing_updates": {"ms_per_step": trail_ms, "algorithmic_flop_per_step": st["trail_flops"],
                                              "tflops": st["trail_flops"] / (trail_ms * 1e-3) / 1e12},
                         "selected_inversion_and_inverses": {
                             "ms_per_step": sel_ms, "algorithmic_flop_per_step": st["selinv_flops"],
                             "tflops": st["selinv_flops"] / (sel_ms * 1e-3) / 1e12},
                         "all_mfma_tile_kernels": {"ms_per_step": mfma_ms, "algorithmic_flop_per_step": all_flops,
                                                   "tflops": all_flops / (mfma_ms * 1e-3) / 1e12}}},
    }
    side = min(args.steps, args.side_steps)
    side_w = min(args.warmup, 1)

    def leg(prec, moments):
        st32, stats32, wall32, mean32, var32, _ = run(prec, moments, steps=side, warmup=side_w,
                                                      state=final["state"])
        ph32 = {k: float(np.mean([s[k] for s in stats32])) for k in ph}
        return {
            "value": S * side / wall32, "unit": "star-updates/s", "ms_per_step": wall32 / side * 1e3,
            "steps": side, "warmup": side_w,
            "star_phase_updates_per_s": S / (ph32["ms_star"] * 1e-3),
            "phases_ms": ph32,
            "refine_iters": int(stats32[-1]["refine_iters"]),
            "refine_residual": float(stats32[-1]["refine_residual"]),
            "surrogate_fallbacks": int(stats32[-1]["surrogate_fallbacks"]),
            "rel_err_vs_fp64": {
                "posterior_mean": float(np.max(np.abs(mean32 - mean64) / np.abs(mean64))),
                "marginal_var": float(np.max(np.abs(var32 - var64) / np.abs(var64))),
                "kind": "max over nodes of |x - x_fp64| / |x_fp64|"},
            "rms_rel_err_vs_fp64": {
                "posterior_mean": float(np.sqrt(np.mean(((mean32 - mean64) / mean64) ** 2))),
                "marginal_var": float(np.sqrt(np.mean(((var32 - var64) / var64) ** 2)))},
            "meets_1e-4": bool(np.max(np.abs(mean32 - mean64) / np.abs(mean64)) <= 1e-4
                               and np.max(np.abs(var32 - var64) / np.abs(var64)) <= 1e-4),
            "note": ("timed over its own short run; errors on the same state: the FP64 run's final sites at its "
                     "final linearisation point, q(f) recomputed in this precision"),
        }

    if maps:
        line["maps"] = maps
    if args.gmm:
        # Unknown distances: noiseless extinction to the true positions
        # (eps = 0), a seeded two-component mixture per star around it, and
        # the catalogue positions at the main component's distance.
        from synth import gmm_catalogue
        _, A_true = E.ep_simulate(cfg, raw["xyz"], raw["sigma"], np.zeros(S), raw["xi"])
        cat = gmm_catalogue(w, raw["xyz"], np.log(A_true))
        st_m, stats_m, wall_m, _, _, _ = run("fp64", extra=dict(likelihood="gmm"), xyz_in=cat["xyz"],
                                             comps=cat["comps"], steps=side, warmup=side_w)
        line["gmm_leg"] = {
            "value": S * side / wall_m, "unit": "star-updates/s", "ms_per_step": wall_m / side * 1e3,
            "steps": side, "warmup": side_w,
            "phases_ms": {k: float(np.mean([s[k] for s in stats_m])) for k in ph},
            "updated_last_sweep": int(stats_m[-1]["updated"]),
            "skipped_negative_site_last_sweep": int(stats_m[-1]["skipped_negsite"]),
            "note": "per-star two-component (ln s, log-extinction) mixtures; distance marginalised in the tilted "
                    "distribution by a 256-node rule in ln s per component along each sightline extended to the "
                    "cube's face (extinction at each distance from the forward model at the linearisation point)",
        }
    if args.theta:
        # Data drawn around a disc + bump mean at THETA_TRUE; EP infers the
        # field and theta jointly from the Sec. 5 hyperprior means.
        sim = E.make_config(w.ep_fields(), device=0, mean_fn="disc_bump", theta_prior=THETA_TRUE)
        _, A_th = E.ep_simulate(sim, raw["xyz"], raw["sigma"], raw["eps"], raw["xi"])
        thv = {}

        def theta_after(g):
            m, c = g.theta()
            sd = np.sqrt(np.diag(c))
            thv["theta_mean"] = [float(v) for v in np.exp(m + 0.5 * sd ** 2)]
            thv["log_theta_sd"] = [float(v) for v in sd]
            thv["z_true"] = [float(v) for v in (m - np.log(THETA_TRUE)) / sd]
            return None

        st_t, stats_t, wall_t, _, _, _ = run("fp64", A_in=A_th, after=theta_after, extra=dict(mean_fn="disc_bump"),
                                             steps=max(side, 4), warmup=side_w)
        line["theta_leg"] = {
            "value": S * max(side, 4) / wall_t, "unit": "star-updates/s", "ms_per_step": wall_t / max(side, 4) * 1e3,
            "steps": max(side, 4), "warmup": side_w,
            "phases_ms": {k: float(np.mean([s[k] for s in stats_t])) for k in ph},
            "theta_names": ["L_pc", "H_pc", "rho_kappa0_per_pc", "s_bump_pc", "A_bump_mag"],
            "theta_true": list(THETA_TRUE), "theta_prior_mean": list(E.make_config().theta_prior),
            **thv,
            "note": ("field and phi = ln theta inferred jointly (five-column Schur border); theta_mean is the "
                     "log-normal posterior mean after warm-up + timed sweeps"),
        }
    if args.pitc:
        line["pitc_leg"] = pitc_leg()
    if args.mixed:
        line["surrogate_mixed"] = leg("mixed", "surrogate")
        line["mixed_quadrature"] = leg("mixed", "quadrature")
        # FP64 factor, selected inversion on FP32 MFMA (FP64 partial sums)
        line["surrogate_selinv32"] = leg("selinv32", "surrogate")
        line["selinv32_quadrature"] = leg("selinv32", "quadrature")
        line["fp64_surrogate"] = leg("fp64", "surrogate")
        line["surrogate_gain"] = surrogate_gain()
    if args.variant:
        line["headline_variant"] = variant_leg()
    if args.plan_in_line:
        line["headline_structure"] = {"cfg3-128cube-1M": plan_of(preset(3)),
                                      "largest_fitting_variant": plan_of(variant_workload())}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.preset, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

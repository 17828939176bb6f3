"""Python binding of the C ABI in include/ep.h (argument marshalling only).

Every step of the EP sweep runs in the HIP library ``libep.so`` built in this
directory for gfx950.  Loading fails loudly when the library is missing.

Functions keep the C names (``ep_init``, ``ep_sweep``, ``ep_posterior_mean``,
``ep_marginal_var``, ...); the ``EP`` class bundles them around one context.
"""
from __future__ import annotations

import ctypes
import os
from typing import Mapping

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libep.so")

EP_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "OOM", -3: "NOT_PD", -4: "DEVICE", -5: "STATE", -6: "NUMERIC"}
LIKELIHOOD = {"extinction": 0, "gauss_linear": 1, "gmm": 2}
PRECISION = {"fp64": 0, "mixed": 1, "selinv32": 2}
MOMENTS = {"quadrature": 0, "surrogate": 1}
MEAN_FN = {"constant": 0, "disc_bump": 1}
N_THETA = 5


class EPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class ep_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("box_pc", ctypes.c_double),
        ("observer_pc", ctypes.c_double * 3),
        ("prior_mean", ctypes.c_double),
        ("prior_var", ctypes.c_double),
        ("outer_scale_pc", ctypes.c_double),
        ("support_pc", ctypes.c_double),
        ("vecchia_radius_pc", ctypes.c_double),
        ("los_step_pc", ctypes.c_double),
        ("likelihood", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("moments", ctypes.c_int32),
        ("damping", ctypes.c_double),
        ("cavity_var_floor", ctypes.c_double),
        ("relinearize", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("leaf_size", ctypes.c_int32),
        ("hbm_cap_bytes", ctypes.c_int64),
        ("profile_kernels", ctypes.c_int32),
        ("mixed_fp64_levels", ctypes.c_int32),
        ("surrogate_tol", ctypes.c_double),
        ("pointers_on_device", ctypes.c_int32),
        ("mean_fn", ctypes.c_int32),
        ("theta_prior", ctypes.c_double * 5),
        ("sun_radius_pc", ctypes.c_double),
        ("bump_width_pc", ctypes.c_double),
        ("relin_step", ctypes.c_double),
        ("deterministic", ctypes.c_int32),
    ]


class ep_sweep_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("ms_linearise", "ms_assemble", "ms_factor", "ms_solve",
                                                "ms_selinv", "ms_star", "ms_total")] + \
               [(k, ctypes.c_int64) for k in ("updated", "skipped_cavity", "skipped_negsite")] + \
               [(k, ctypes.c_double) for k in ("max_dtau", "max_dmu", "mfma_ms")] + \
               [("mfma_launches", ctypes.c_int64), ("refine_iters", ctypes.c_int32),
                ("refine_residual", ctypes.c_double), ("surrogate_fallbacks", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double * 10), ("kernel_launches", ctypes.c_int64 * 10)]


class ep_structure_stats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_stars", ctypes.c_int64), ("nnz_g", ctypes.c_int64),
                ("n_fronts", ctypes.c_int64), ("n_levels", ctypes.c_int32), ("front_elems", ctypes.c_int64),
                ("max_front", ctypes.c_int64), ("factor_flops", ctypes.c_double),
                ("selinv_flops", ctypes.c_double), ("trail_flops", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("front_elems_lower", ctypes.c_int64),
                ("update_elems", ctypes.c_int64), ("offdiag_elems", ctypes.c_int64), ("x_elems", ctypes.c_int64),
                ("clique_pairs", ctypes.c_int64)]


class ep_plan_stats(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_stars", ctypes.c_int64), ("nnz_g", ctypes.c_int64),
                ("max_support", ctypes.c_int64), ("n_fronts", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("max_front", ctypes.c_int64), ("max_separator", ctypes.c_int64), ("front_elems", ctypes.c_int64),
                ("front_elems_lower", ctypes.c_int64), ("nnz_L", ctypes.c_int64), ("x_elems", ctypes.c_int64),
                ("w_elems", ctypes.c_int64), ("factor_flops", ctypes.c_double), ("selinv_flops", ctypes.c_double),
                ("trail_flops", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("device_bytes_mixed", ctypes.c_int64)]


class ep_pitc_stats(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_inducing", ctypes.c_int64), ("max_block_stars", ctypes.c_int64),
                ("max_block_nodes", ctypes.c_int64), ("sweep_flops", ctypes.c_double),
                ("predict_flops", ctypes.c_double), ("device_bytes", ctypes.c_int64)]


EXPORTS = ("ep_config_default", "ep_init", "ep_sweep", "ep_posterior_mean", "ep_marginal_var", "ep_free",
           "ep_last_error", "ep_get_sites", "ep_set_sites", "ep_get_linpoint", "ep_set_linpoint",
           "ep_star_state", "ep_tilted_moments", "ep_simulate", "ep_structure", "ep_mlp_train",
           "ep_mlp_predict", "ep_mlp_loss_grad", "ep_mlp_load", "ep_ordering", "ep_density_moments",
           "ep_extinction_map", "ep_point_predict", "ep_theta", "ep_set_gmm", "ep_pitc_setup", "ep_pitc_sweep",
           "ep_pitc_inducing", "ep_pitc_predict", "ep_pitc_info", "ep_pitc_theta", "ep_mlp_predict_noalloc", "ep_plan")
MLP_NPARAM = 34065
EP_NOALLOC_MAX_TUPLES = 1 << 20   # ep.h
KERNEL_KINDS = ("trsm", "inner", "trail", "gemm", "zero", "assemble", "extend", "gather", "cavity",
                "solve")   # EP_KK_* order


class ep_mlp_hyper(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("seed", ctypes.c_uint64)]

_lib = None


class _TorchDtypes(dict):
    def __missing__(self, k):
        import torch
        v = {np.float64: torch.float64, np.float32: torch.float32, np.int32: torch.int32}[k]
        self[k] = v
        return v


_TORCH = _TorchDtypes()


def load(path: str | None = None):
    """Load libep.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    # torch ships its own HIP runtime; it must be loaded and initialised
    # before this library's, or torch later finds no GPU in the process
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    L = ctypes.CDLL(p)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    cfgp = ctypes.POINTER(ep_config)
    L.ep_config_default.argtypes = [cfgp]
    L.ep_config_default.restype = None
    L.ep_init.argtypes = [cfgp, i64, vp, vp, vp, ctypes.POINTER(vp)]
    L.ep_sweep.argtypes = [vp, ctypes.POINTER(ep_sweep_stats)]
    L.ep_posterior_mean.argtypes = [vp, vp]
    L.ep_marginal_var.argtypes = [vp, vp]
    L.ep_free.argtypes = [vp]
    L.ep_free.restype = None
    L.ep_last_error.argtypes = [vp]
    L.ep_last_error.restype = ctypes.c_char_p
    L.ep_get_sites.argtypes = [vp, vp, vp]
    L.ep_set_sites.argtypes = [vp, vp, vp]
    L.ep_get_linpoint.argtypes = [vp, vp]
    L.ep_set_linpoint.argtypes = [vp, vp]
    L.ep_star_state.argtypes = [vp] * 7
    L.ep_tilted_moments.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, vp, i32]
    L.ep_simulate.argtypes = [cfgp, i64, vp, vp, vp, vp, vp, vp]
    L.ep_structure.argtypes = [vp, ctypes.POINTER(ep_structure_stats)]
    L.ep_mlp_train.argtypes = [ctypes.POINTER(ep_mlp_hyper), i64, vp, vp, vp, vp, i32]
    L.ep_mlp_predict.argtypes = [vp, i64, vp, ctypes.c_double, vp, vp, vp, i32]
    L.ep_mlp_loss_grad.argtypes = [vp, i64, vp, vp, vp, vp, i32]
    L.ep_mlp_load.argtypes = [vp, vp]
    L.ep_ordering.argtypes = [vp, vp]
    L.ep_density_moments.argtypes = [vp, vp, vp]
    L.ep_extinction_map.argtypes = [vp, i32, vp, vp, vp]
    L.ep_point_predict.argtypes = [vp, i64, vp, vp]
    L.ep_theta.argtypes = [vp, vp, vp]
    L.ep_set_gmm.argtypes = [vp, i32, vp]
    L.ep_pitc_setup.argtypes = [vp, i32, vp, i64, vp, vp]
    L.ep_pitc_sweep.argtypes = [vp, ctypes.c_double, vp]
    L.ep_pitc_inducing.argtypes = [vp, vp, vp]
    L.ep_pitc_predict.argtypes = [vp, vp, vp]
    L.ep_pitc_info.argtypes = [vp, ctypes.POINTER(ep_pitc_stats)]
    L.ep_pitc_theta.argtypes = [vp, vp, vp]
    L.ep_mlp_predict_noalloc.argtypes = [vp, i64, vp, ctypes.c_double, vp, vp, vp, i32, vp]
    L.ep_plan.argtypes = [cfgp, i64, vp, ctypes.POINTER(ep_plan_stats)]
    for name in ("ep_init", "ep_sweep", "ep_posterior_mean", "ep_marginal_var", "ep_get_sites",
                 "ep_set_sites", "ep_get_linpoint", "ep_set_linpoint", "ep_star_state",
                 "ep_tilted_moments", "ep_simulate", "ep_structure", "ep_mlp_train", "ep_mlp_predict",
                 "ep_mlp_loss_grad", "ep_mlp_load", "ep_ordering", "ep_density_moments", "ep_extinction_map",
                 "ep_point_predict", "ep_theta", "ep_set_gmm", "ep_pitc_setup", "ep_pitc_sweep",
                 "ep_pitc_inducing", "ep_pitc_predict", "ep_pitc_info", "ep_pitc_theta", "ep_mlp_predict_noalloc", "ep_plan"):
        getattr(L, name).restype = ctypes.c_int
    if path is None:
        _lib = L
    return L


def _arr(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_config(fields: Mapping | None = None, lib=None, **kw) -> ep_config:
    """An ep_config from defaults plus a mapping of field values (the same
    keys as the C struct; likelihood/precision/moments may be strings)."""
    L = lib or load()
    c = ep_config()
    L.ep_config_default(ctypes.byref(c))
    vals = dict(fields or {})
    vals.update(kw)
    for k, v in vals.items():
        if k == "likelihood" and isinstance(v, str):
            v = LIKELIHOOD[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        elif k == "moments" and isinstance(v, str):
            v = MOMENTS[v]
        elif k == "mean_fn" and isinstance(v, str):
            v = MEAN_FN[v]
        elif k == "relinearize":
            v = int(bool(v))
        if k == "observer_pc":
            c.observer_pc = (ctypes.c_double * 3)(*v)
        elif k == "theta_prior":
            c.theta_prior = (ctypes.c_double * 5)(*v)
        elif k == "stream":
            c.stream = ctypes.c_void_p(int(v) if v else None)
        elif hasattr(c, k):
            setattr(c, k, v)
        else:
            raise KeyError(f"unknown config field {k}")
    return c


def _marshal_in(a, n, on_device: bool, device: int, dtype=np.float64):
    """(object to keep alive, pointer) for an input array: a contiguous host
    copy, or with on_device a tensor on cuda:device (pointers_on_device)."""
    if not on_device:
        a = np.ascontiguousarray(a, dtype=dtype)
        if n is not None and a.size != n:
            raise ValueError(f"expected {n} values, got {a.size}")
        return a, _ptr(a)
    import torch
    t = torch.as_tensor(a, device=f"cuda:{device}").to(_TORCH[dtype]).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    torch.cuda.current_stream(t.device).synchronize()   # the library's stream does not wait for torch's
    return t, ctypes.c_void_p(t.data_ptr())


def _marshal_out(shape, on_device: bool, device: int, dtype=np.float64):
    """(array, pointer) for an output: numpy on the host, or a tensor on
    cuda:device (pointers_on_device)."""
    if not on_device:
        a = np.empty(shape, dtype=dtype)
        return a, _ptr(a)
    import torch
    t = torch.empty(shape, dtype=_TORCH[dtype], device=f"cuda:{device}")
    torch.cuda.current_stream(t.device).synchronize()
    return t, ctypes.c_void_p(t.data_ptr())


def _check(L, rc: int, ctx=None):
    if rc != EP_OK:
        msg = L.ep_last_error(ctx).decode()
        raise EPError(rc, msg)


# ---- C names -----------------------------------------------------------------
def ep_init(cfg: ep_config, xyz, A_obs, sigma, lib=None):
    """With cfg.pointers_on_device the arrays may be numpy arrays or tensors;
    they are passed as tensors on cuda:cfg.device."""
    L = lib or load()
    dev, d = bool(cfg.pointers_on_device), int(cfg.device)
    S = int(np.prod(tuple(xyz.shape))) // 3 if hasattr(xyz, "shape") else len(np.asarray(xyz).reshape(-1, 3))
    keep = [_marshal_in(a, n, dev, d) if a is not None else (None, None)
            for a, n in ((xyz, 3 * S), (A_obs, S), (sigma, S))]   # A_obs, sigma: None with the GMM likelihood
    out = ctypes.c_void_p()
    _check(L, L.ep_init(ctypes.byref(cfg), S, keep[0][1], keep[1][1], keep[2][1], ctypes.byref(out)))
    return out


def ep_sweep(ctx, lib=None) -> dict:
    L = lib or load()
    st = ep_sweep_stats()
    _check(L, L.ep_sweep(ctx, ctypes.byref(st)), ctx)
    out = {k: getattr(st, k) for k, _ in ep_sweep_stats._fields_}
    for k in ("kernel_ms", "kernel_launches"):
        out[k] = dict(zip(KERNEL_KINDS, list(out[k])))
    return out


def ep_posterior_mean(ctx, N: int, lib=None, on_device: bool = False, device: int = 0):
    """on_device must match the context's pointers_on_device."""
    L = lib or load()
    out, p = _marshal_out(N, on_device, device)
    _check(L, L.ep_posterior_mean(ctx, p), ctx)
    return out


def ep_marginal_var(ctx, N: int, lib=None, on_device: bool = False, device: int = 0):
    """on_device must match the context's pointers_on_device."""
    L = lib or load()
    out, p = _marshal_out(N, on_device, device)
    _check(L, L.ep_marginal_var(ctx, p), ctx)
    return out


def ep_free(ctx, lib=None) -> None:
    L = lib or load()
    L.ep_free(ctx)


def ep_tilted_moments(mode, mu_c, v_c, A, sigma, device: int = 0, lib=None):
    L = lib or load()
    mu_c = _arr(mu_c)
    n = mu_c.size
    v_c, A, sigma = _arr(v_c, n), _arr(A, n), _arr(sigma, n)
    lnZ, m, v = np.empty(n), np.empty(n), np.empty(n)
    mode = LIKELIHOOD.get(mode, mode) if isinstance(mode, str) else int(mode)
    _check(L, L.ep_tilted_moments(mode, n, _ptr(mu_c), _ptr(v_c), _ptr(A), _ptr(sigma), _ptr(lnZ), _ptr(m),
                                  _ptr(v), device))
    return lnZ, m, v


def ep_simulate(cfg: ep_config, xyz, sigma, eps, xi, lib=None):
    """(f_true, A_obs) from raw deviates with the library's own arithmetic."""
    L = lib or load()
    xyz = _arr(xyz).reshape(-1, 3)
    S = xyz.shape[0]
    N = cfg.n ** 3
    sigma, eps, xi = _arr(sigma, S), _arr(eps, S), _arr(xi, N)
    f = np.empty(N)
    A = np.empty(S)
    _check(L, L.ep_simulate(ctypes.byref(cfg), S, _ptr(xyz), _ptr(sigma), _ptr(eps), _ptr(xi), _ptr(f), _ptr(A)))
    return f, A


def ep_mlp_train(inputs, targets, epochs=20, batch=4096, lr=1e-3, seed=1, device=0, lib=None):
    """Train the tilted-moment surrogate.  inputs (n, 4): mu_c, v_c, A, sigma;
    targets (n, 3): ln Z, mean, var.  Returns (weights float32, loss per epoch)."""
    L = lib or load()
    X = _arr(inputs).reshape(-1, 4)
    Y = _arr(targets).reshape(-1, 3)
    if X.shape[0] != Y.shape[0]:
        raise ValueError("inputs and targets differ in length")
    w = np.zeros(MLP_NPARAM, dtype=np.float32)
    loss = np.zeros(epochs)
    hp = ep_mlp_hyper(epochs, batch, lr, seed)
    _check(L, L.ep_mlp_train(ctypes.byref(hp), X.shape[0], _ptr(X), _ptr(Y), _ptr(w), _ptr(loss), device))
    return w, loss


def ep_mlp_predict_noalloc(weights, inputs, out3, errest=None, accepted=None, tol=1e-4, device=0, stream=None,
                           lib=None):
    """The allocation-free form of ep_mlp_predict: every array is a
    contiguous tensor already on cuda:device (weights float32 or None, inputs
    (n, 4) and out3 (n, 3) float64, errest float64, accepted int32; either of
    the last two may be None); stream is a torch stream or None.  Nothing is
    allocated: the outputs are written in place."""
    L = lib or load()

    def ptr(t, dtype, what):
        if t is None:
            return None
        if str(t.dtype) != "torch." + dtype or not t.is_contiguous() or t.device.type != "cuda" \
                or t.device.index != device:
            raise ValueError(f"{what}: expected a contiguous {dtype} tensor on cuda:{device}")
        return ctypes.c_void_p(t.data_ptr())

    n = inputs.shape[0] if inputs.dim() == 2 else inputs.numel() // 4
    if inputs.numel() != 4 * n or out3.numel() != 3 * n:
        raise ValueError("inputs must hold n x 4 and out3 n x 3 values")
    for t, k in ((errest, 1), (accepted, 1)):
        if t is not None and t.numel() != k * n:
            raise ValueError("errest and accepted must hold n values")
    st = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(L, L.ep_mlp_predict_noalloc(ptr(weights, "float32", "weights"), n, ptr(inputs, "float64", "inputs"), tol,
                                       ptr(out3, "float64", "out3"), ptr(errest, "float64", "errest"),
                                       ptr(accepted, "int32", "accepted"), device, st))


def ep_plan(cfg, xyz, lib=None) -> dict:
    """Structure, work and memory of a configuration from the host analysis
    alone (no device)."""
    L = lib or load()
    c = cfg if isinstance(cfg, ep_config) else make_config(cfg, lib=L)
    x = _arr(xyz).reshape(-1, 3)
    out = ep_plan_stats()
    _check(L, L.ep_plan(ctypes.byref(c), x.shape[0], _ptr(x), ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in ep_plan_stats._fields_}


def ep_mlp_predict(weights, inputs, tol=1e-4, device=0, lib=None):
    """Gated surrogate moments: (out (n,3), error estimate (n,), accepted (n,))."""
    L = lib or load()
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    X = _arr(inputs).reshape(-1, 4)
    n = X.shape[0]
    out = np.zeros((n, 3))
    err = np.zeros(n)
    acc = np.zeros(n, dtype=np.int32)
    _check(L, L.ep_mlp_predict(None if w is None else _ptr(w), n, _ptr(X), tol, _ptr(out), _ptr(err), _ptr(acc),
                               device))
    return out, err, acc.astype(bool)


def ep_mlp_loss_grad(weights, xstd, ystd, device=0, lib=None):
    L = lib or load()
    w = np.ascontiguousarray(weights, dtype=np.float32)
    X = np.ascontiguousarray(xstd, dtype=np.float32).reshape(-1, 4)
    Y = np.ascontiguousarray(ystd, dtype=np.float32).reshape(-1, 3)
    loss = np.zeros(1)
    g = np.zeros(MLP_NPARAM, dtype=np.float32)
    _check(L, L.ep_mlp_loss_grad(_ptr(w), X.shape[0], _ptr(X), _ptr(Y), _ptr(loss), _ptr(g), device))
    return float(loss[0]), g


# ---- convenience wrapper -----------------------------------------------------
class EP:
    """One EP context on the GPU.  With cfg pointers_on_device = 1 every
    array goes in and comes out as a tensor on cuda:device."""

    def __init__(self, cfg: Mapping | ep_config, xyz, A_obs=None, sigma=None, lib=None):
        self.L = lib or load()
        self.cfg = cfg if isinstance(cfg, ep_config) else make_config(cfg, lib=self.L)
        self.N = self.cfg.n ** 3
        self.on_device = bool(self.cfg.pointers_on_device)
        self.device = int(self.cfg.device)
        self.ctx = ep_init(self.cfg, xyz, A_obs, sigma, lib=self.L)
        st = ep_structure_stats()
        _check(self.L, self.L.ep_structure(self.ctx, ctypes.byref(st)), self.ctx)
        self.S = int(st.n_stars)

    def _in(self, a, n, dtype=np.float64):
        return _marshal_in(a, n, self.on_device, self.device, dtype)

    def _out(self, shape, dtype=np.float64):
        return _marshal_out(shape, self.on_device, self.device, dtype)

    def sweep(self) -> dict:
        return ep_sweep(self.ctx, lib=self.L)

    def posterior_mean(self):
        return ep_posterior_mean(self.ctx, self.N, lib=self.L, on_device=self.on_device, device=self.device)

    def marginal_var(self):
        return ep_marginal_var(self.ctx, self.N, lib=self.L, on_device=self.on_device, device=self.device)

    def sites(self):
        (tau, pt), (nu, pn) = self._out(self.S), self._out(self.S)
        _check(self.L, self.L.ep_get_sites(self.ctx, pt, pn), self.ctx)
        return tau, nu

    def set_sites(self, tau, nu) -> None:
        (kt, pt), (kn, pn) = self._in(tau, self.S), self._in(nu, self.S)
        _check(self.L, self.L.ep_set_sites(self.ctx, pt, pn), self.ctx)

    @property
    def n_lin(self) -> int:
        """Length of the linearisation point: n^3, plus the 5 log-parameters
        of an inferred mean."""
        return self.N + (N_THETA if self.cfg.mean_fn == MEAN_FN["disc_bump"] else 0)

    def linpoint(self):
        f, p = self._out(self.n_lin)
        _check(self.L, self.L.ep_get_linpoint(self.ctx, p), self.ctx)
        return f

    def set_linpoint(self, f) -> None:
        k, p = self._in(f, self.n_lin)
        _check(self.L, self.L.ep_set_linpoint(self.ctx, p), self.ctx)

    def set_gmm(self, comps) -> None:
        """Per-star distance / log-extinction mixtures, (S, K, 6) rows
        (w, m_l, m_b, C_ll, C_lb, C_bb), for the GMM likelihood."""
        shape = tuple(comps.shape) if hasattr(comps, "shape") else np.asarray(comps).shape
        K = int(np.prod(shape)) // (6 * self.S) if self.S else 1
        k, p = self._in(comps, self.S * K * 6)
        _check(self.L, self.L.ep_set_gmm(self.ctx, K, p), self.ctx)

    def theta(self):
        """Posterior mean (5) and covariance (5 x 5) of phi = ln theta."""
        (m, pm), (c, pc) = self._out(N_THETA), self._out((N_THETA, N_THETA))
        _check(self.L, self.L.ep_theta(self.ctx, pm, pc), self.ctx)
        return m, c

    def pitc_setup(self, star_block, inducing, node_block) -> None:
        """PITC sub-catalogues (star_block: S ints 0..K-1), inducing node ids
        (R), and the sub-catalogue each node's prediction conditions on
        (node_block: N ints)."""
        sb = np.asarray(star_block.cpu() if hasattr(star_block, "cpu") else star_block)
        K = int(sb.max()) + 1 if sb.size else 0
        R = int(np.prod(np.shape(inducing)))
        keep = [self._in(a, n, np.int32) for a, n in ((star_block, self.S), (inducing, R), (node_block, self.N))]
        _check(self.L, self.L.ep_pitc_setup(self.ctx, K, keep[0][1], R, keep[1][1], keep[2][1]), self.ctx)
        self.n_inducing = R

    def pitc_sweep(self, damping: float = 1.0) -> float:
        """One parallel pass over the sub-catalogues; returns ln p(a~) under PITC."""
        lz = ctypes.c_double(0.0)
        _check(self.L, self.L.ep_pitc_sweep(self.ctx, float(damping), ctypes.byref(lz)), self.ctx)
        return lz.value

    def pitc_inducing(self):
        """Mean (R) and covariance (R x R) of q(u)."""
        (m, pm), (c, pc) = self._out(self.n_inducing), self._out((self.n_inducing, self.n_inducing))
        _check(self.L, self.L.ep_pitc_inducing(self.ctx, pm, pc), self.ctx)
        return m, c

    def pitc_theta(self):
        """Mean (5) and covariance (5 x 5) of phi = ln theta under q(u, Theta)."""
        (m, pm), (c, pc) = self._out(N_THETA), self._out((N_THETA, N_THETA))
        _check(self.L, self.L.ep_pitc_theta(self.ctx, pm, pc), self.ctx)
        return m, c

    def pitc_info(self) -> dict:
        st = ep_pitc_stats()
        _check(self.L, self.L.ep_pitc_info(self.ctx, ctypes.byref(st)), self.ctx)
        return {k: getattr(st, k) for k, _ in ep_pitc_stats._fields_}

    def pitc_predict(self):
        """PIC predictive mean and variance of f at every node."""
        (m, pm), (v, pv) = self._out(self.N), self._out(self.N)
        _check(self.L, self.L.ep_pitc_predict(self.ctx, pm, pv), self.ctx)
        return m, v

    def star_state(self) -> dict:
        keys = ("lnA", "cav_mu", "cav_var", "lnZ", "tilted_mean", "tilted_var")
        outs = [self._out(self.S) for _ in keys]
        _check(self.L, self.L.ep_star_state(self.ctx, *[p for _, p in outs]), self.ctx)
        return dict(zip(keys, [a for a, _ in outs]))

    def load_surrogate(self, weights) -> None:
        k, p = self._in(weights, MLP_NPARAM, np.float32)
        _check(self.L, self.L.ep_mlp_load(self.ctx, p), self.ctx)

    def ordering(self):
        perm, p = self._out(self.N, np.int32)
        _check(self.L, self.L.ep_ordering(self.ctx, p), self.ctx)
        return perm

    def density_moments(self):
        (m, pm), (v, pv) = self._out(self.N), self._out(self.N)
        _check(self.L, self.L.ep_density_moments(self.ctx, pm, pv), self.ctx)
        return m, v

    def extinction_map(self, z=None):
        """Exact posterior mean of A to every node; with z (K x N standard
        normals, K >= 2, consumed in elimination order) also the sample
        variance over the K posterior draws."""
        mean, pm = self._out(self.N)
        if z is None:
            _check(self.L, self.L.ep_extinction_map(self.ctx, 0, None, pm, None), self.ctx)
            return mean
        K = int(np.prod(tuple(z.shape))) // self.N if hasattr(z, "shape") else np.asarray(z).size // self.N
        kz, pz = self._in(z, K * self.N)
        var, pv = self._out(self.N)
        _check(self.L, self.L.ep_extinction_map(self.ctx, K, pz, pm, pv), self.ctx)
        return mean, var

    def point_predict(self, xyz2):
        n = (int(np.prod(tuple(xyz2.shape))) if hasattr(xyz2, "shape") else np.asarray(xyz2).size) // 6
        kx, px = self._in(xyz2, 6 * n)
        out, po = self._out((n, 5))
        _check(self.L, self.L.ep_point_predict(self.ctx, n, px, po), self.ctx)
        return out

    def structure(self) -> dict:
        st = ep_structure_stats()
        _check(self.L, self.L.ep_structure(self.ctx, ctypes.byref(st)), self.ctx)
        return {k: getattr(st, k) for k, _ in ep_structure_stats._fields_}

    def close(self) -> None:
        if getattr(self, "ctx", None):
            ep_free(self.ctx, lib=self.L)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

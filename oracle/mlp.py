"""Plain FP64 reference of the tilted-moment surrogate (test infrastructure only).

The surrogate maps one star's tilted problem (cavity mean mu_c and variance
v_c of a_n = ln A_n, observed extinction A and its 1-sigma noise s) to the
tilted moments (ln Z, mean, variance) of Sec. 4.1 / App. A.2.

Baseline: the likelihood N(A | e^a, s^2) linearised in a around
a0 = ln max(A, s) is N(a; a0 + (A - e^a0)/e^a0, (s/e^a0)^2); its product with
the cavity gives a Gaussian (m0, v0) and a normaliser Z0.  The network
predicts corrections to that baseline:
    y1 = (mean - m0) / sqrt(v0),  y2 = ln(var / v0),  y3 = ln Z - ln Z0.
Features: (mu_c, ln v_c, A e^{-mu_c}, ln(s e^{-mu_c})), standardised.
Network: 4 -> 128 -> 128 -> 128 -> 3, SiLU, mean squared error on the
standardised targets.

Parameter blob (float32, this order): W1 (4x128, row-major in x W), b1,
W2 (128x128), b2, W3 (128x128), b3, W4 (128x3), b4, then the input mean and
std (4 + 4) and the target mean and std (3 + 3).
"""
from __future__ import annotations

import math

import numpy as np

H = 128
SHAPES = [("W1", (4, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("W4", (H, 3)), ("b4", (3,)), ("xm", (4,)), ("xs", (4,)), ("ym", (3,)), ("ys", (3,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)
NTRAIN = sum(int(np.prod(s)) for n, s in SHAPES if n[0] in "Wb")


def unpack(blob: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(blob[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def baseline(mu, v, A, s):
    """Gaussian baseline (m0, v0, lnZ0) of the tilted distribution."""
    mu, v, A, s = (np.asarray(x, dtype=np.float64) for x in (mu, v, A, s))
    y0 = np.maximum(A, s)
    a0 = np.log(y0)
    ml = a0 + (A - y0) / y0            # mean of the linearised likelihood in a
    vl = (s / y0) ** 2                 # its variance
    v0 = 1.0 / (1.0 / v + 1.0 / vl)
    m0 = v0 * (mu / v + ml / vl)
    # Z0 = N(ml; mu, v + vl) times the Jacobian of A -> a at y0
    lnZ0 = -0.5 * np.log(2 * math.pi * (v + vl)) - 0.5 * (ml - mu) ** 2 / (v + vl) - np.log(y0)
    return m0, v0, lnZ0


def features(mu, v, A, s):
    mu, v, A, s = (np.asarray(x, dtype=np.float64) for x in (mu, v, A, s))
    return np.stack([mu, np.log(v), A * np.exp(-mu), np.log(s) - mu], axis=-1)


def targets(mu, v, A, s, lnZ, mean, var):
    m0, v0, lnZ0 = baseline(mu, v, A, s)
    return np.stack([(mean - m0) / np.sqrt(v0), np.log(var / v0), lnZ - lnZ0], axis=-1)


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    sg = 1.0 / (1.0 + np.exp(-x))
    return sg * (1.0 + x * (1.0 - sg))


def forward(p: dict, X: np.ndarray):
    """X: standardised features (n, 4).  Returns outputs (n, 3) and the
    cache of pre-activations for backprop."""
    z1 = X @ p["W1"] + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = silu(z2)
    z3 = h2 @ p["W3"] + p["b3"]
    h3 = silu(z3)
    out = h3 @ p["W4"] + p["b4"]
    return out, (X, z1, h1, z2, h2, z3, h3)


def loss_grad(p: dict, X: np.ndarray, Y: np.ndarray):
    """Mean over the batch of the squared error summed over the 3 outputs
    (Y standardised), and its gradient for every W and b."""
    n = X.shape[0]
    out, (X, z1, h1, z2, h2, z3, h3) = forward(p, X)
    d = out - Y
    loss = float(np.sum(d * d) / n)
    g = {}
    dout = 2.0 * d / n
    g["W4"] = h3.T @ dout
    g["b4"] = dout.sum(0)
    dz3 = (dout @ p["W4"].T) * dsilu(z3)
    g["W3"] = h2.T @ dz3
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"].T) * dsilu(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * dsilu(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g


def predict(blob: np.ndarray, mu, v, A, s):
    """Surrogate moments (lnZ, mean, var) in FP64."""
    p = unpack(blob)
    X = (features(mu, v, A, s) - p["xm"]) / p["xs"]
    out, _ = forward(p, X)
    y = out * p["ys"] + p["ym"]
    m0, v0, lnZ0 = baseline(mu, v, A, s)
    return lnZ0 + y[:, 2], m0 + np.sqrt(v0) * y[:, 0], v0 * np.exp(y[:, 1])


def gauss_hermite_check(mu, v, A, s, m, var, nodes: int = 8):
    """Moments of the tilted distribution by an n-node Gauss-Hermite rule
    centred at (m, sqrt(var)) (numpy's hermgauss)."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    sd = np.sqrt(var)[:, None]
    a = m[:, None] + math.sqrt(2.0) * sd * x[None, :]
    ell = (-(a - mu[:, None]) ** 2 / (2 * v[:, None]) - 0.5 * np.log(2 * math.pi * v[:, None])
           - (A[:, None] - np.exp(a)) ** 2 / (2 * s[:, None] ** 2) - 0.5 * np.log(2 * math.pi * s[:, None] ** 2))
    lg = ell + x[None, :] ** 2 + np.log(w)[None, :]
    mx = lg.max(1, keepdims=True)
    e = np.exp(lg - mx)
    Z = e.sum(1)
    mean = (e * a).sum(1) / Z
    varr = (e * (a - mean[:, None]) ** 2).sum(1) / Z
    lnZ = np.log(Z) + mx[:, 0] + np.log(math.sqrt(2.0) * sd[:, 0])
    return lnZ, mean, varr

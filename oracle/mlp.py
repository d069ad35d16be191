"""FP64 oracle of the retarded-delay surrogate network -- TEST INFRASTRUCTURE ONLY.

The model predicts the retarded look-back s = c (t - t_r) of a (target,
source) pair from 10 pair features as s_line exp(z), where s_line is the
look-back to a source coasting with its newest velocity (a closed form of
the features, straight_line_lookback) and z the network output:

    h1 = silu(W1 x + b1)     W1: 128 x 10
    h2 = silu(W2 h1 + b2)    W2: 128 x 128
    z  = W3 h2 + b3          W3: 1 x 128

It is trained on z against log(s / s_line) (mean squared error), i.e. on
the relative error of the delay; z = 0 is the straight-line guess.  Weights and inputs are rounded to bfloat16
(round to nearest even) before use, as the GPU kernels store them; all
arithmetic here is float64.

Features of the pair (target i at y_i, source j with history slots n, n-4):
    (y_i - w_{j,n}) / sigma_ref            3
    v_{j,n} / c                            3
    (w_{j,n} - w_{j,n-4}) / (c (T_n - T_{n-4}))   3
    log1p((t - T_n) / dt)                  1
The surrogate is not part of the paper; it only seeds the bracket search
and the exact search always decides the result.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
N_IN, N_HID = 10, 128
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (1, N_HID)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned
    as float64.  Goes through float32 first (the GPU stores float32 masters)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def silu(x):
    return x / (1.0 + np.exp(-x))


def silu_grad(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def forward(flat, X, round_bf16=True):
    """X: [batch, 10].  Returns z [batch] and the cache for backward."""
    p = unpack(bf16_round(flat) if round_bf16 else flat)
    Xr = bf16_round(X) if round_bf16 else np.asarray(X, dtype=np.float64)
    a1 = Xr @ p["W1"].T + p["b1"]
    h1 = silu(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = silu(a2)
    z = h2 @ p["W3"].T + p["b3"]
    return z[:, 0], (p, Xr, a1, h1, a2, h2)


def loss_and_grad(flat, X, y, round_bf16=True):
    """Mean squared error of z against y and its gradient with respect to
    the (unrounded) flat parameter vector (straight-through rounding)."""
    z, (p, Xr, a1, h1, a2, h2) = forward(flat, X, round_bf16)
    B = X.shape[0]
    r = z - y
    loss = float(np.mean(r * r))
    dz = (2.0 / B) * r[:, None]                 # [B, 1]
    g = {"W3": dz.T @ h2, "b3": dz.sum(0)}
    dh2 = dz @ p["W3"]                          # [B, 128]
    da2 = dh2 * silu_grad(a2)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * silu_grad(a1)
    g["W1"] = da1.T @ Xr
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def adam_step(flat, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; step counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1**step)
    vh = v / (1 - beta2**step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def features(y_i, w_n, v_n, w_n4, T_n, T_n4, t, dt, sigma_ref):
    """Pair features.  y_i, w_n, v_n, w_n4: [3, P] arrays; scalars otherwise.
    Returns [P, 10]."""
    rel = (y_i - w_n) / sigma_ref
    beta = v_n / C_LIGHT
    slope = (w_n - w_n4) / (C_LIGHT * (T_n - T_n4))
    lg = np.full((1, rel.shape[1]), np.log1p((t - T_n) / dt))
    return np.concatenate([rel, beta, slope, lg]).T


def straight_line_lookback(y_i, w_n, v_n):
    """Light distance s = c (t - t_r) from y_i back to a source that moved
    with constant velocity v_n and is at w_n at the present time t: with
    R = y_i - w_n and beta = v_n / c the source was at w_n - beta s, so
    |R + beta s| = s, i.e. (1 - beta^2) s^2 - 2 (R . beta) s - |R|^2 = 0;
    the positive root.  Arrays [3, P]; returns [P]."""
    R = y_i - w_n
    beta = v_n / C_LIGHT
    rb = np.sum(R * beta, axis=0)
    R2 = np.sum(R * R, axis=0)
    g2 = 1.0 - np.sum(beta * beta, axis=0)
    return (rb + np.sqrt(rb * rb + g2 * R2)) / g2


def normalised_delay(y_i, w_n, t, tr):
    """g = c (t - t_r) / |y_i - w_n|."""
    return C_LIGHT * (t - tr) / np.linalg.norm(y_i - w_n, axis=0)

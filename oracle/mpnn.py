"""Message-passing network used as a learned Poisson preconditioner
(oracle; test infrastructure only).

Not part of the paper: this is the benchmark spec's learned form.  The network
maps a residual r to a correction z, z = D^-1 r + s_d * y(r), where D^-1 is
the Jacobi scaling and y is a 3-layer message-passing network of width 32
over the cell-face graph (each cell's 4 face neighbours; a boundary face has
no neighbour):

    x_i   = [r_i / s_r, (D^-1 r)_i / s_d]            s_r, s_d = RMS of r, D^-1 r
    h0_i  = We x_i + be
    for l in 1..3:
        m_i  = 1/4 sum_{j face neighbour of i} h_j
        u_i  = relu(W1_l [h_i; m_i] + b1_l)
        h_i <- h_i + W2_l u_i + b2_l
    y_i   = wd . h3_i + bd

z is 1-homogeneous in r (s_r, s_d scale with r).  Two training losses:

  residual:  L = || r - K z(r) ||^2 / || r ||^2,
             dL/dz = -2 K^T (r - K z) / ||r||^2;
  energy:    L = (z^T K z - 2 z^T r) / (r^T D^-1 r),
             dL/dz = 2 (K_s z - r) / (r^T D^-1 r),   K_s = (K + K^T) / 2.

The energy functional is minimised by z = K_s^-1 r and equals
||z - K_s^-1 r||^2_{K_s} minus a constant, the norm conjugate gradients
minimise; it needs no solution vector.  The residual loss weights the error
by K^2, i.e. toward the rough end of the spectrum.

``forward(..., bf16_like_gpu=True)`` rounds to bfloat16 exactly where the GPU
kernels store or feed a matrix core: the weights, h after the encoder and
after every layer, and u.  The neighbour mean m is not rounded: the kernels
form it inside the matrix-core product (each neighbour row times W1's m-half
scaled by 1/4, FP32 accumulation), so it never exists as a bf16 value.  ``backward`` is the chain rule of the forward it is given:
exact for the FP64 forward (pinned by finite differences in the tests); for
the rounded forward it treats each rounding as the identity (straight-through)
and so multiplies by the rounded weights, the ones that forward used.
"""
from __future__ import annotations

import numpy as np

H = 32
LAYERS = 3


def init_params(seed=0, scale=0.1):
    """Parameter dict; the decoder starts at zero so z starts as D^-1 r."""
    rng = np.random.default_rng(seed)
    p = {"We": rng.normal(0, scale, (H, 2)), "be": np.zeros(H)}
    for l in range(LAYERS):
        p[f"W1_{l}"] = rng.normal(0, scale, (H, 2 * H))
        p[f"b1_{l}"] = np.zeros(H)
        p[f"W2_{l}"] = rng.normal(0, scale, (H, H))
        p[f"b2_{l}"] = np.zeros(H)
    p["wd"] = np.zeros(H)
    p["bd"] = np.zeros(1)
    return p


PARAM_ORDER = (["We", "be"] + [f"{k}_{l}" for l in range(LAYERS) for k in ("W1", "b1", "W2", "b2")]
               + ["wd", "bd"])


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k in PARAM_ORDER])


def unflatten(v, like):
    out, at = {}, 0
    for k in PARAM_ORDER:
        n = np.asarray(like[k]).size
        out[k] = np.asarray(v[at:at + n]).reshape(np.shape(like[k]))
        at += n
    return out


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    b = a32.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = ((b + 0x7FFF + lsb) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _neigh_mean(h, nbr):
    """1/4 sum over the (up to 4) face neighbours; nbr[i, k] < 0: none."""
    valid = nbr >= 0
    g = h[np.where(valid, nbr, 0)] * valid[..., None]
    return g.sum(axis=1) / 4.0


def _neigh_scatter(g, nbr, n):
    """Adjoint of _neigh_mean: out_j = 1/4 sum_{i : j face neighbour of i} g_i."""
    out = np.zeros((n, g.shape[1]))
    valid = nbr >= 0
    for k in range(nbr.shape[1]):
        idx = nbr[:, k][valid[:, k]]
        np.add.at(out, idx, g[valid[:, k]] / 4.0)
    return out


def scales(r, dinv):
    n = len(r)
    s_r = np.sqrt(np.dot(r, r) / n)
    dr = dinv * r
    s_d = np.sqrt(np.dot(dr, dr) / n)
    return s_r, s_d


def forward(p, r, dinv, nbr, bf16_like_gpu=False):
    """z(r) and the activations the backward needs."""
    q = (lambda a: bf16(a)) if bf16_like_gpu else (lambda a: np.asarray(a, np.float64))
    s_r, s_d = scales(r, dinv)
    x = np.stack([r / s_r, dinv * r / s_d], axis=1)
    h = q(x @ q(p["We"]).T + p["be"])
    cache = {"x": x, "h": [h], "a": [], "v": [], "u": [], "s_d": s_d, "s_r": s_r,
             "bf16": bool(bf16_like_gpu)}
    for l in range(LAYERS):
        m = _neigh_mean(h, nbr)
        a = np.concatenate([h, m], axis=1)
        v = a @ q(p[f"W1_{l}"]).T + p[f"b1_{l}"]
        u = q(np.maximum(v, 0.0))
        h = q(h + u @ q(p[f"W2_{l}"]).T + p[f"b2_{l}"])
        cache["a"].append(a)
        cache["v"].append(v)
        cache["u"].append(u)
        cache["h"].append(h)
    y = h @ p["wd"] + p["bd"][0]
    z = dinv * r + s_d * y
    return z, cache


def backward(p, cache, nbr, dz):
    """Parameter gradients of sum_i dz_i z_i (FP64 chain rule)."""
    g = {}
    n = len(dz)
    q = bf16 if cache.get("bf16") else (lambda a: np.asarray(a, np.float64))
    dy = cache["s_d"] * dz
    h3 = cache["h"][-1]
    g["wd"] = h3.T @ dy
    g["bd"] = np.array([dy.sum()])
    dh = np.outer(dy, p["wd"])
    for l in reversed(range(LAYERS)):
        a, v, u = cache["a"][l], cache["v"][l], cache["u"][l]
        g[f"W2_{l}"] = dh.T @ u
        g[f"b2_{l}"] = dh.sum(axis=0)
        du = (dh @ q(p[f"W2_{l}"])) * (v > 0)
        g[f"W1_{l}"] = du.T @ a
        g[f"b1_{l}"] = du.sum(axis=0)
        da = du @ q(p[f"W1_{l}"])
        dh = dh + da[:, :H] + _neigh_scatter(da[:, H:], nbr, n)
    g["We"] = dh.T @ cache["x"]
    g["be"] = dh.sum(axis=0)
    return g


def loss_and_grad(p, K, r, dinv, nbr, bf16_like_gpu=False, kind="residual"):
    """Loss of one sample r and its parameter gradient (FP64 arithmetic; with
    bf16_like_gpu the forward rounds as the GPU does)."""
    z, cache = forward(p, r, dinv, nbr, bf16_like_gpu)
    if kind == "residual":
        res = r - K @ z
        rr = np.dot(r, r)
        L = np.dot(res, res) / rr
        dz = -2.0 * (K.T @ res) / rr
    elif kind == "energy":
        rdr = np.dot(r, dinv * r)
        kz, ktz = K @ z, K.T @ z
        L = (np.dot(z, kz) - 2.0 * np.dot(z, r)) / rdr
        dz = (kz + ktz - 2.0 * r) / rdr
    else:
        raise ValueError(kind)
    return L, backward(p, cache, nbr, dz)


def face_neighbours(geo):
    """[Nc,4] cell across each face, -1 for a boundary face (from the oracle
    geometry)."""
    other = np.where(geo.csign > 0, geo.fR[geo.cfaces], geo.fL[geo.cfaces])
    return np.where(other < geo.nc, other, -1)

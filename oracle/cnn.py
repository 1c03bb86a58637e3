"""Oracle of the learned preconditioner (FP64, numpy; test infrastructure only).

A small residual 3-D CNN refines the filtered Landweber update u = alpha p * B r
(eq. 4's step): out = u + f(u), with f four 3^3 convolutions
1 -> 16 -> 32 -> 32 -> 1 channels, zero "same" padding, and erf-GELU after the
first three.  Training minimises the mean squared error against the true
error of the current iterate.  Everything here is the plain definition:
convolutions as sums over the 27 taps, gradients by the chain rule.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

__all__ = ["CHANNELS", "init_params", "conv3d", "conv3d_grad_input", "conv3d_grad_weight", "gelu", "gelu_grad",
           "forward", "backward", "mse", "adam_step"]

CHANNELS = (1, 16, 32, 32, 1)


def init_params(seed: int = 0, scale: float = 1.0):
    """He-style initialisation from PCG64; the last layer starts at zero so the
    network starts as the identity (out = u)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for li in range(4):
        ci, co = CHANNELS[li], CHANNELS[li + 1]
        std = scale * math.sqrt(2.0 / (27 * ci))
        W = rng.normal(0.0, std, size=(co, ci, 3, 3, 3))
        if li == 3:
            W[:] = 0.0
        params.append([W, np.zeros(co)])
    return params


def _shift(x, dz, dy, dx):
    """y[c, z, y, x] = x[c, z+dz, y+dy, x+dx], zero outside."""
    out = np.zeros_like(x)
    C, D, H, W = x.shape
    zs, ys, xs = slice(max(0, -dz), min(D, D - dz)), slice(max(0, -dy), min(H, H - dy)), slice(max(0, -dx), min(W, W - dx))
    zt, yt, xt = slice(max(0, dz), min(D, D + dz)), slice(max(0, dy), min(H, H + dy)), slice(max(0, dx), min(W, W + dx))
    out[:, zs, ys, xs] = x[:, zt, yt, xt]
    return out


def conv3d(x, W, b):
    """Cross-correlation with zero "same" padding (the convention of
    torch.nn.functional.conv3d): out[o, v] = b[o] + sum_{i, d} W[o, i, d] x[i, v + d - 1]."""
    Co = W.shape[0]
    out = np.zeros((Co,) + x.shape[1:]) + b[:, None, None, None]
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = _shift(x, kz - 1, ky - 1, kx - 1)
                out += np.tensordot(W[:, :, kz, ky, kx], xs, axes=(1, 0))
    return out


def conv3d_grad_input(g, W):
    """d/dx of sum(g * conv3d(x, W, b)): sum_{o, d} W[o, i, d] g[o, v - d + 1]."""
    Ci = W.shape[1]
    out = np.zeros((Ci,) + g.shape[1:])
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                gs = _shift(g, 1 - kz, 1 - ky, 1 - kx)
                out += np.tensordot(W[:, :, kz, ky, kx], gs, axes=(0, 0))
    return out


def conv3d_grad_weight(x, g):
    """d/dW of sum(g * conv3d(x, W, b)) and d/db."""
    Co, Ci = g.shape[0], x.shape[0]
    dW = np.zeros((Co, Ci, 3, 3, 3))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = _shift(x, kz - 1, ky - 1, kx - 1)
                dW[:, :, kz, ky, kx] = np.tensordot(g, xs, axes=([1, 2, 3], [1, 2, 3]))
    return dW, g.sum(axis=(1, 2, 3))


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(u, params):
    """u: (D, H, W).  Returns out = u + f(u) and the cache for backward."""
    h = u[None]
    cache = []
    for li, (W, b) in enumerate(params):
        z = conv3d(h, W, b)
        cache.append((h, z))
        h = gelu(z) if li < 3 else z
    return u + h[0], cache


def backward(cache, dout, params):
    """Gradients of sum(dout * out) with respect to every W, b (and u)."""
    g = dout[None]
    grads = [None] * 4
    du = dout.copy()
    for li in range(3, -1, -1):
        h, z = cache[li]
        if li < 3:
            g = g * gelu_grad(z)
        dW, db = conv3d_grad_weight(h, g)
        grads[li] = [dW, db]
        g = conv3d_grad_input(g, params[li][0])
    du += g[0]
    return grads, du


def mse(out, target):
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) in place; state holds (t, m, v)."""
    t = state.get("t", 0) + 1
    state["t"] = t
    if "m" not in state:
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    for li, layer in enumerate(params):
        for pi, p in enumerate(layer):
            gp = grads[li][pi]
            m = state["m"][li][pi]
            v = state["v"][li][pi]
            m *= b1
            m += (1 - b1) * gp
            v *= b2
            v += (1 - b2) * gp * gp
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            p -= lr * mh / (np.sqrt(vh) + eps)
    return params

"""The learned preconditioner's storage model, composed from the FP64 oracle's
layer functions (test helper; not part of the oracle).

The library keeps the network's master weights, the input u, the
pre-activations z and the accumulations in FP32, and stores in BF16 (round to
nearest even) exactly these values: the weights of the two 32-output layers
(layers 2 and 3), the activations h1, h2, h3 after each GELU, and the
back-propagated pre-activation gradients dz1, dz2, dz3.  Applying those
roundings between the oracle's own FP64 convolutions, GELU and gradient
functions gives a reference that differs from the GPU only by FP32
accumulation order and the occasional BF16 rounding flip, so the comparison
can be tight enough to catch a wrong tap or channel block in one kernel.
"""

from __future__ import annotations

import numpy as np

from oracle import cnn


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def bf16(x):
    """Round to FP32, then to BF16 (nearest even), back to float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def stored_weights(params):
    """The weights each layer computes with: FP32 master values, BF16 for
    layers 2 and 3."""
    out = []
    for li, (W, b) in enumerate(params):
        out.append([bf16(W) if li in (1, 2) else f32(W), f32(b)])
    return out


def forward(u, params):
    """out = u + f(u) under the storage model; returns (out, cache)."""
    P = stored_weights(params)
    u32 = f32(u)
    h = u32[None]
    cache = []
    for li, (W, b) in enumerate(P):
        z = cnn.conv3d(h, W, b)
        cache.append((h, z))
        h = bf16(cnn.gelu(z)) if li < 3 else z
    return u32 + h[0], cache


def backward(cache, dout, params):
    """Weight and bias gradients of sum(dout * out) under the storage model."""
    P = stored_weights(params)
    g = np.asarray(dout, dtype=np.float64)[None]
    grads = [None] * 4
    for li in range(3, -1, -1):
        h, z = cache[li]
        grads[li] = list(cnn.conv3d_grad_weight(h, g))
        if li > 0:
            hz = cache[li - 1][1]
            g = bf16(cnn.gelu_grad(hz) * cnn.conv3d_grad_input(g, P[li][0]))
    return grads

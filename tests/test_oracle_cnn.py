"""Pins of the CNN oracle (CPU): convolution against torch's conv3d (a
library routine), GELU against its closed form, network gradients against
central finite differences."""

import math

import numpy as np
import pytest
import torch

from oracle import cnn


def test_conv3d_matches_library(rng):
    x = rng.normal(size=(5, 6, 7, 8))
    W = rng.normal(size=(4, 5, 3, 3, 3))
    b = rng.normal(size=4)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x)[None], torch.from_numpy(W), torch.from_numpy(b),
                                     padding=1)[0].numpy()
    assert np.allclose(cnn.conv3d(x, W, b), ref, atol=1e-12)


def test_conv3d_adjoints(rng):
    x = rng.normal(size=(3, 5, 4, 6))
    W = rng.normal(size=(2, 3, 3, 3, 3))
    g = rng.normal(size=(2, 5, 4, 6))
    # <conv(x), g> = <x, conv^T(g)> and = <W, dW(x, g)>
    lhs = float((cnn.conv3d(x, W, np.zeros(2)) * g).sum())
    assert abs(lhs - float((x * cnn.conv3d_grad_input(g, W)).sum())) < 1e-10 * abs(lhs)
    dW, db = cnn.conv3d_grad_weight(x, g)
    assert abs(lhs - float((W * dW).sum())) < 1e-10 * abs(lhs)
    assert np.allclose(db, g.sum(axis=(1, 2, 3)))


def test_gelu_closed_form():
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    ref = [0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x]
    assert np.allclose(cnn.gelu(x), ref, atol=1e-15)
    eps = 1e-6
    assert np.allclose(cnn.gelu_grad(x), (cnn.gelu(x + eps) - cnn.gelu(x - eps)) / (2 * eps), atol=1e-8)


def test_network_gradients_central_differences(rng):
    params = cnn.init_params(seed=3, scale=1.0)
    params[3][0] = rng.normal(0, 0.05, size=params[3][0].shape)   # non-trivial last layer
    params[3][1] = rng.normal(0, 0.05, size=1)
    u = rng.normal(size=(5, 4, 6))
    target = rng.normal(size=u.shape)
    out, cache = cnn.forward(u, params)
    loss, dout = cnn.mse(out, target)
    grads, du = cnn.backward(cache, dout, params)
    eps = 1e-6
    for li, pi, idx in [(0, 0, (3, 0, 1, 2, 0)), (1, 0, (5, 7, 0, 1, 2)), (2, 0, (1, 2, 2, 0, 1)),
                        (3, 0, (0, 4, 1, 1, 1)), (1, 1, (6,)), (3, 1, (0,))]:
        p = params[li][pi]
        old = p[idx]
        p[idx] = old + eps
        lp = cnn.mse(cnn.forward(u, params)[0], target)[0]
        p[idx] = old - eps
        lm = cnn.mse(cnn.forward(u, params)[0], target)[0]
        p[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert grads[li][pi][idx] == pytest.approx(fd, rel=1e-5, abs=1e-10)
    idx = (2, 1, 3)
    old = u[idx]
    u[idx] = old + eps
    lp = cnn.mse(cnn.forward(u, params)[0], target)[0]
    u[idx] = old - eps
    lm = cnn.mse(cnn.forward(u, params)[0], target)[0]
    u[idx] = old
    assert du[idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5)


def test_identity_at_initialisation(rng):
    params = cnn.init_params(seed=0)
    u = rng.normal(size=(4, 4, 4))
    out, _ = cnn.forward(u, params)
    assert np.array_equal(out, u)


def test_adam_constant_gradient_closed_form(rng):
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step, so each Adam step moves a parameter by -lr g/(|g| + eps);
    a sign flip in either moment, a missing bias correction or a wrong power
    of beta breaks this."""
    params = [[rng.normal(size=(2, 3)), rng.normal(size=2)]]
    grads = [[rng.normal(size=(2, 3)) * 10.0 ** rng.integers(-3, 3, size=(2, 3)), rng.normal(size=2)]]
    p0 = [[p.copy() for p in layer] for layer in params]
    state = {}
    lr, eps = 3e-3, 1e-8
    for _ in range(5):
        cnn.adam_step(params, grads, state, lr=lr, eps=eps)
    for p, q, g in zip(params[0], p0[0], grads[0]):
        assert np.allclose(p, q - 5 * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    # a changing gradient: the second step from the moments written out
    params = [[np.array([1.0])]]
    state = {}
    cnn.adam_step(params, [[np.array([2.0])]], state, lr=0.1)
    cnn.adam_step(params, [[np.array([-1.0])]], state, lr=0.1)
    m = 0.9 * 0.1 * 2.0 + 0.1 * -1.0
    v = 0.999 * 0.001 * 4.0 + 0.001 * 1.0
    step2 = 0.1 * (m / (1 - 0.81)) / (math.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert abs(params[0][0][0] - (1.0 - 0.1 * 2.0 / (2.0 + 1e-8) - step2)) < 1e-12

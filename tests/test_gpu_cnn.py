"""Learned preconditioner network on the matrix cores against the FP64
oracle.  The GPU keeps BF16 weights for the two 32-output layers and BF16
activations between layers (FP32 accumulation), so results are compared at
the level those roundings allow: 2^-9 relative per stored value, compounded
over four layers."""

import numpy as np
import pytest

import paper_2103_10329_amd as mg
from gpu_common import rel_l2, say, to_dev, to_host
from oracle import cnn

pytestmark = pytest.mark.gpu


def _setup(shape=(16, 24, 32), seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = cnn.init_params(seed=seed)
    params[3][0] = rng.normal(0, 0.05, size=params[3][0].shape)
    params[3][1] = rng.normal(0, 0.05, size=1)
    for layer in params:
        layer[1] = rng.normal(0, 0.05, size=layer[1].shape)
    u = rng.normal(size=shape)
    target = u + 0.3 * rng.normal(size=shape)
    ctx = mg.Context(0)
    ctx.cnn_set_weights(mg.cnn_flatten(params))
    return ctx, params, u, target


def test_forward_matches_oracle():
    ctx, params, u, _ = _setup()
    out = to_host(ctx.cnn_forward(to_dev(u)))
    ref, _ = cnn.forward(u, params)
    e = rel_l2(out - u, ref - u)
    say("cnn forward: rel L2 of f(u)", e)
    assert e <= 2e-2


def test_gradients_match_oracle():
    ctx, params, u, target = _setup()
    g, loss = ctx.cnn_gradients(to_dev(u), to_dev(target))
    out, cache = cnn.forward(u, params)
    lref, dout = cnn.mse(out, target)
    grads, _ = cnn.backward(cache, dout, params)
    gref = mg.cnn_unflatten(mg.cnn_flatten(grads))
    gg = mg.cnn_unflatten(g)
    say("cnn loss", loss, lref)
    assert abs(loss - lref) / lref <= 1e-2
    for li in range(4):
        for pi in range(2):
            e = rel_l2(gg[li][pi], gref[li][pi])
            say("  layer", li + 1, "W" if pi == 0 else "b", "rel L2", e)
            assert e <= 5e-2


def test_adam_training_reduces_loss():
    ctx, params, u, target = _setup(shape=(16, 16, 32), seed=9)
    ut, tt = to_dev(u), to_dev(target)
    losses = [ctx.cnn_train_step(ut, tt, 3e-3) for _ in range(40)]
    say("cnn training loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    # the same 3 steps on the oracle, from the same start
    ctx2, params2, u2, t2 = _setup(shape=(16, 16, 32), seed=9)
    w0 = mg.cnn_flatten(params2).astype(np.float64)
    st = {}
    for _ in range(3):
        out, cache = cnn.forward(u2, params2)
        _, dout = cnn.mse(out, t2)
        gr, _ = cnn.backward(cache, dout, params2)
        cnn.adam_step(params2, gr, st, lr=3e-3)
    for _ in range(3):
        ctx2.cnn_train_step(to_dev(u2), to_dev(t2), 3e-3, want_loss=False)
    # Adam's first steps are close to lr * sign(g): compare the updates, whose
    # error reflects the BF16-level gradient differences (~2e-3 relative) on
    # components with small gradients
    dw = ctx2.cnn_get_weights().astype(np.float64) - w0
    dref = mg.cnn_flatten(params2).astype(np.float64) - w0
    e = rel_l2(dw, dref)
    say("Adam update after 3 steps vs oracle", e)
    assert e <= 5e-2

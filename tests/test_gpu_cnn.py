"""Learned preconditioner network on the matrix cores against the FP64
oracle.

Two references: the plain FP64 network (what the method computes), and the
same oracle layer functions with the library's documented BF16 storage
roundings applied between them (``cnn_storage``).  The second differs from
the GPU only by FP32 accumulation order and rare BF16 rounding flips, so the
forward output, every layer's weight and bias gradient and three Adam steps
are compared with it at bars a localized kernel error cannot hide under."""

import numpy as np
import pytest

import cnn_storage
import paper_2103_10329_amd as mg
from gpu_common import rel_l2, say, to_dev, to_host
from oracle import cnn

pytestmark = pytest.mark.gpu

# Bars against the storage-model reference.  What is left after the storage
# roundings is the BF16 rounding flips that FP32 accumulation order triggers
# (a value within FP32 error of a BF16 rounding boundary rounds the other way,
# one BF16 ulp, and the flip propagates through later layers): measured on
# MI355X forward 1.9e-4 (max 1.2e-3), and the same floor is reproduced on the
# CPU by evaluating the storage model's convolutions in FP32 (2.2e-4, max
# 1.1e-3).  The bars sit about 5x above that floor and at least 10x below the
# deviation of any localized kernel error planted in the storage model on the
# CPU (one tap of one 8-channel block: >= 4e-2; tests/test_cnn_storage.py).
FWD_L2, FWD_MAX = 1e-3, 6e-3
GRAD_L2 = 1e-3
# Adam: its first steps are about lr * sign(g), so a component whose gradient
# sits at the flip floor may take the opposite step (|dw| up to 2 lr per step).
# Measured on MI355X: 14 of 42849 components differ by more than 0.1 lr, the
# rest agree to 1.1e-3 of the update (L2).  Bars about 5x those.
ADAM_FLIPS, ADAM_REST_L2 = 64, 5e-3


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


def _max_rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def test_forward_matches_oracle():
    ctx, params, u, _ = _setup()
    out = to_host(ctx.cnn_forward(to_dev(u)))
    ref, _ = cnn.forward(u, params)
    e_plain = rel_l2(out - u, ref - u)
    sref, _ = cnn_storage.forward(u, params)
    u32 = cnn_storage.f32(u)
    e = rel_l2(out - u32, sref - u32)
    emax = _max_rel(out - u32, sref - u32)
    say("cnn forward f(u): rel L2 vs storage model %.3e (max %.3e), vs plain FP64 network %.3e" % (e, emax, e_plain))
    assert e <= FWD_L2 and emax <= FWD_MAX
    assert e_plain <= 2e-2


@pytest.fixture(scope="module")
def large_grid():
    """A ragged grid above 128^3 voxels (z not a multiple of the 4-z block, y
    not a multiple of 3) and its storage-model forward pass, shared by the
    two large-grid tests."""
    ctx, params, u, target = _setup(shape=(102, 136, 160), seed=7)
    sref, cache = cnn_storage.forward(u, params)
    return ctx, params, u, target, sref, cache


def test_forward_large_grid_marching_kernel(large_grid):
    """From 128^3 voxels up the two 32-output layers run on the persistent,
    weight-stationary kernels that march along y (and the activations use
    the branch-free GELU), against the same storage model."""
    ctx, params, u, _, sref, _ = large_grid
    out = to_host(ctx.cnn_forward(to_dev(u)))
    u32 = cnn_storage.f32(u)
    e = rel_l2(out - u32, sref - u32)
    emax = _max_rel(out - u32, sref - u32)
    say("cnn forward 160x136x102: rel L2 vs storage model %.3e (max %.3e)" % (e, emax))
    assert e <= FWD_L2 and emax <= FWD_MAX


def test_gradients_large_grid(large_grid):
    """The training forward pass on a large grid keeps every layer's FP32
    pre-activations besides the BF16 activations (the marching kernels'
    second output); the gradients built from them against the storage
    model's."""
    ctx, params, u, target, sref, cache = large_grid
    g, loss = ctx.cnn_gradients(to_dev(u), to_dev(target))
    gg = mg.cnn_unflatten(g)
    lref, dout = cnn.mse(sref, target)
    gref = cnn_storage.backward(cache, dout, params)
    say("cnn loss 160x136x102", loss, lref)
    assert abs(loss - lref) / lref <= 1e-5
    for li in range(4):
        for pi in range(2):
            e = rel_l2(gg[li][pi], gref[li][pi])
            say("  layer %d %s rel L2 %.3e" % (li + 1, "W" if pi == 0 else "b", e))
            assert e <= GRAD_L2, (li, pi, e)


def test_gradients_match_oracle():
    ctx, params, u, target = _setup()
    g, loss = ctx.cnn_gradients(to_dev(u), to_dev(target))
    gg = mg.cnn_unflatten(g)
    out, cache = cnn_storage.forward(u, params)
    lref, dout = cnn.mse(out, target)
    gref = cnn_storage.backward(cache, dout, params)
    say("cnn loss", loss, lref)
    assert abs(loss - lref) / lref <= 1e-5
    for li in range(4):
        for pi in range(2):
            e = rel_l2(gg[li][pi], gref[li][pi])
            emax = _max_rel(gg[li][pi], gref[li][pi])
            say("  layer %d %s rel L2 %.3e max %.3e" % (li + 1, "W" if pi == 0 else "b", e, emax))
            assert e <= GRAD_L2, (li, pi, e)


def test_backward_and_adam_entry_points():
    """The standalone backward (a caller-defined loss through its d loss /
    d out) and Adam step of the boundary: with dout = 2 (out - target) / n,
    the mean squared error's, mgct_cnn_backward returns mgct_cnn_gradients's
    gradients, and mgct_adam_step with them leaves the weights that
    mgct_cnn_train_step leaves."""
    import torch
    ctx, params, u, target = _setup()
    ud, td = to_dev(u), to_dev(target)
    g_ref, _ = ctx.cnn_gradients(ud, td)
    out = ctx.cnn_forward(ud)
    dout = 2.0 * (out - td) / float(u.size)
    g = ctx.cnn_backward(ud, dout)
    e = _max_rel(g, g_ref)
    say("cnn_backward vs cnn_gradients: max rel %.3e" % e)
    # torch's division rounds a few dout values differently from the library's
    # loss kernel (last bit); measured 7.4e-7, bar about 14x that
    assert e <= 1e-5
    lr = 3e-3
    ctx_a, _, _, _ = _setup()
    ga, _ = ctx_a.cnn_gradients(ud, td)
    ctx_a.adam_step(ga, lr)
    ctx_b, _, _, _ = _setup()
    ctx_b.cnn_train_step(ud, td, lr, want_loss=False)
    wa, wb = ctx_a.cnn_get_weights(), ctx_b.cnn_get_weights()
    assert np.array_equal(wa, wb)
    assert not np.array_equal(wa, mg.cnn_flatten(params).astype(np.float32))
    del torch


def test_adam_training_reduces_loss():
    ctx, params, u, target = _setup(shape=(16, 16, 32), seed=9)
    ut, tt = to_dev(u), to_dev(target)
    losses = [ctx.cnn_train_step(ut, tt, 3e-3) for _ in range(40)]
    say("cnn training loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.7 * losses[0]
    # the same 3 Adam steps under the storage model, from the same start
    ctx2, params2, u2, t2 = _setup(shape=(16, 16, 32), seed=9)
    w0 = mg.cnn_flatten(params2).astype(np.float64)
    st = {}
    for _ in range(3):
        out, cache = cnn_storage.forward(u2, params2)
        _, dout = cnn.mse(out, t2)
        gr = cnn_storage.backward(cache, dout, params2)
        cnn.adam_step(params2, gr, st, lr=3e-3)
    for _ in range(3):
        ctx2.cnn_train_step(to_dev(u2), to_dev(t2), 3e-3, want_loss=False)
    w = ctx2.cnn_get_weights().astype(np.float64)
    wref = mg.cnn_flatten(params2).astype(np.float64)
    du, duref = w - w0, wref - w0
    d = np.abs(du - duref)
    big = d > 0.1 * 3e-3
    e_rest = float(np.linalg.norm((du - duref)[~big]) / np.linalg.norm(duref[~big]))
    say("Adam after 3 steps vs storage model: weights rel L2 %.3e, updates %.3e; %d components beyond 0.1 lr, "
        "the rest %.3e" % (rel_l2(w, wref), rel_l2(du, duref), int(big.sum()), e_rest))
    assert int(big.sum()) <= ADAM_FLIPS and e_rest <= ADAM_REST_L2

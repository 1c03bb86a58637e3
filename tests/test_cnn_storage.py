"""CPU checks of the learned preconditioner's storage-model reference used by
the GPU parity tests: its BF16 rounding is the standard one, without the
roundings it is the oracle's network, its rounding floor (FP32 accumulation
order flipping BF16 roundings) sits well under the GPU bars, and a localized
kernel error planted in it deviates far above them."""

import copy

import numpy as np
import pytest
import torch

import cnn_storage as cs
from oracle import cnn
from test_gpu_cnn import FWD_L2, GRAD_L2


def _setup(shape=(8, 12, 16), seed=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = cnn.init_params(seed=seed)
    params[3][0] = rng.normal(0, 0.05, size=params[3][0].shape)
    params[3][1] = rng.normal(0, 0.05, size=1)
    for layer in params:
        layer[1] = rng.normal(0, 0.05, size=layer[1].shape)
    u = rng.normal(size=shape)
    return params, u, u + 0.3 * rng.normal(size=shape)


def _run(params, u, target):
    out, cache = cs.forward(u, params)
    _, dout = cnn.mse(out, target)
    return out, cs.backward(cache, dout, params)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.random.default_rng(1).normal(size=20000) * np.exp(np.random.default_rng(2).normal(size=20000) * 5)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    assert np.array_equal(cs.bf16(x), ref)
    # ties: 1 + 2^-8 lies half-way between 1 and 1 + 2^-7 and goes to the even one
    assert cs.bf16(np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8]))[0] == 1.0
    assert cs.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_without_roundings_it_is_the_oracle(monkeypatch):
    params, u, target = _setup()
    monkeypatch.setattr(cs, "bf16", lambda x: np.asarray(x, dtype=np.float64))
    monkeypatch.setattr(cs, "f32", lambda x: np.asarray(x, dtype=np.float64))
    out, grads = _run(params, u, target)
    ref, cache = cnn.forward(u, params)
    _, dout = cnn.mse(ref, target)
    gref, _ = cnn.backward(cache, dout, params)
    assert np.allclose(out, ref, rtol=0, atol=1e-13)
    for li in range(4):
        for pi in range(2):
            assert np.allclose(grads[li][pi], gref[li][pi], rtol=0, atol=1e-12 * np.abs(gref[li][pi]).max())


def _conv32(x, W, b):
    """The same convolution accumulated in FP32 (another summation order and
    precision, as on the GPU)."""
    x32, W32 = x.astype(np.float32), W.astype(np.float32)
    out = np.zeros((W.shape[0],) + x.shape[1:], np.float32) + b.astype(np.float32)[:, None, None, None]
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                out += np.tensordot(W32[:, :, kz, ky, kx], cnn._shift(x32, kz - 1, ky - 1, kx - 1),
                                    axes=(1, 0)).astype(np.float32)
    return out.astype(np.float64)


def test_rounding_floor_is_below_the_gpu_bars(monkeypatch):
    params, u, target = _setup()
    out, grads = _run(params, u, target)
    monkeypatch.setattr(cnn, "conv3d", _conv32)
    out32, grads32 = _run(params, u, target)
    u32 = cs.f32(u)
    ef = np.linalg.norm(out32 - out) / np.linalg.norm(out - u32)
    eg = max(np.linalg.norm(grads32[li][0] - grads[li][0]) / np.linalg.norm(grads[li][0]) for li in range(4))
    assert ef <= FWD_L2 / 2 and eg <= GRAD_L2 / 2, (ef, eg)


@pytest.mark.parametrize("plant", ["l1_tap", "l2_block_centre", "l2_block_corner", "l3_out_block", "l3_z_swap",
                                   "l4_block", "l2_bias_block"])
def test_localized_kernel_error_exceeds_the_bars(plant):
    params, u, target = _setup()
    out, grads = _run(params, u, target)
    p = copy.deepcopy(params)
    if plant == "l1_tap":
        p[0][0][:, 0, 1, 1, 0] = 0
    elif plant == "l2_block_centre":
        p[1][0][:, 0:8, 1, 1, 1] = 0
    elif plant == "l2_block_corner":
        p[1][0][:, 8:16, 0, 0, 0] = 0
    elif plant == "l3_out_block":
        p[2][0][8:16, :, 0, 2, 1] = 0
    elif plant == "l3_z_swap":
        W = p[2][0]
        W[:, :, 0, 1, 1], W[:, :, 2, 1, 1] = W[:, :, 2, 1, 1].copy(), W[:, :, 0, 1, 1].copy()
    elif plant == "l4_block":
        p[3][0][0, 0:8, 1, 1, 1] = 0
    elif plant == "l2_bias_block":
        p[1][1][0:8] = 0
    out2, grads2 = _run(p, u, target)
    u32 = cs.f32(u)
    ef = np.linalg.norm(out2 - out) / np.linalg.norm(out - u32)
    eg = max(np.linalg.norm(grads2[li][0] - grads[li][0]) / np.linalg.norm(grads[li][0]) for li in range(4))
    assert ef >= 10 * FWD_L2 or eg >= 10 * GRAD_L2, (ef, eg)

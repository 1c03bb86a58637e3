"""Reduced-precision storage (BF16 volume, FP16 detector stacks, FP32
accumulation) against the FP64 oracle.

Two errors are measured per result: against the oracle run on the values the
GPU actually stored (what the kernels compute, so FP32 parity applies up to
the output's own rounding) and against the oracle run on the original FP64
inputs (the end-to-end cost of the reduced storage).  Bounds, from the
arithmetic: BF16 keeps 8 significant bits (relative rounding <= 2^-9 = 2e-3
per value), FP16 11 bits (<= 2^-12 = 2.4e-4); a projection or back-projection
averages hundreds of independently rounded values, so the relative L2 error
of a result is well below the per-value bound except for the rounding of the
output itself.
"""

import json
import os

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
import synth
from gpu_common import context, rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _bf16_round(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


def _f16_round(x):
    return np.asarray(x, np.float16).astype(np.float64)


def test_project_bf16_volume_f16_stack():
    import torch
    g = workload("c1").level(1)   # 64^3, 360 x 96^2
    d = synth.make_dataset("c1", truth=True)
    mu = oracle.restrict_volume(d["mu"])
    ctx = context(g)
    vb = to_dev(mu, torch.bfloat16)
    out = to_host(ctx.project(vb, out_dtype=torch.float16))
    ref_stored = oracle.project(g, _bf16_round(mu))
    ref_exact = oracle.project(g, mu)
    e_s, e_x = rel_l2(out, ref_stored), rel_l2(out, ref_exact)
    say("A bf16->f16: vs stored", e_s, "vs exact", e_x)
    assert e_s <= 2.5e-4          # FP16 rounding of the output
    assert e_x <= 2e-3


def test_backproject_f16_stack_bf16_volume():
    import torch
    g = workload("c1").level(1)
    rng = np.random.Generator(np.random.PCG64(21))
    y = rng.random(g.stack_shape)
    ctx = context(g)
    yt = to_dev(y, torch.float16)
    out32 = to_host(ctx.backproject(yt))
    out16 = to_host(ctx.backproject(yt, out_dtype=torch.bfloat16))
    ref_stored = oracle.backproject(g, _f16_round(y))
    ref_exact = oracle.backproject(g, y)
    e1, e2, e3 = rel_l2(out32, ref_stored), rel_l2(out32, ref_exact), rel_l2(out16, ref_exact)
    say("At f16 data: f32 out vs stored", e1, "vs exact", e2, "; bf16 out vs exact", e3)
    # the transposed, ray-scaled copy of an F16 stack is itself F16: each
    # scaled value is rounded once more (2^-11 relative, random), which
    # leaves about 1e-5 on the FP32 sums; BF16 output adds its own 2^-9
    assert e1 <= 3e-5 and e2 <= 5e-5 and e3 <= 3e-3


def test_mixed_sirt_c0():
    g = workload("c0")
    d = synth.make_dataset("c0")
    ctx = context(g)
    ctx.set_precision("bfloat16", "float16")
    alpha = 1.0 / oracle.power_iteration(g, None, iters=30, seed=0)
    mu = np.zeros(g.vol_shape)
    vol = to_dev(mu)
    b = to_dev(d["b"])
    for _ in range(10):
        mu, r = oracle.landweber_step(g, mu, d["b"], alpha, None)
        rg = ctx.landweber_step(vol, b, alpha)
    e = rel_l2(to_host(vol), mu)
    say("mixed SIRT x10 vs FP64 oracle", e, "residual", abs(rg - r) / r)
    # measured on MI355X: 1.0e-4 (volume); bars about 5x that
    assert e <= 5e-4 and abs(rg - r) / r <= 5e-4


def test_crop_resolve_mixed_vs_fp64_oracle():
    """The 512^3 workload's error check: its central 64^3 box, all 1440 views
    on a 96^2 detector, 4 grids, 2 PMG iterations, radial filter; GPU in mixed
    storage and in FP32 against the FP64 oracle with the same steps."""
    path = os.path.join(HERE, "golden", "alphas.json")
    al = json.load(open(path)).get("c2_crop") if os.path.exists(path) else None
    if al is None:
        pytest.skip("tests/golden/alphas.json has no c2_crop steps (run tests/golden/make_golden.py)")
    alphas = al["radial_ramp"]
    d = synth.crop_dataset("c2", n=64, nu=96)
    g = oracle.Geom(64, 64, 64, d["h"], (0, 0, 0), 96, 96, d["views"])
    t, r = oracle.radial_table(64)
    say("crop re-solve: oracle")
    ref, hist_ref = oracle.multigrid(g, np.zeros(g.vol_shape), d["b"], 4, 2, oracle.filter_radial(t, r), alphas)
    ctx = context(g)
    b = to_dev(d["b"])
    res = {}
    for mode in ("fp32", "mixed"):
        if mode == "mixed":
            ctx.set_precision("bfloat16", "float16")
        vol = to_dev(np.zeros(g.vol_shape))
        hist = ctx.multigrid_solve(vol, b, 4, 2, mg.filter_radial(t, r), alphas=alphas)
        res[mode] = (rel_l2(to_host(vol), ref), float(np.max(np.abs(hist - hist_ref) / hist_ref)))
    say("crop re-solve rel L2 vs FP64 oracle: fp32 %.3e (hist %.3e), mixed %.3e (hist %.3e)"
        % (res["fp32"] + res["mixed"]))
    assert res["fp32"][0] <= 1e-5 and res["fp32"][1] <= 1e-5
    # measured on MI355X: mixed 1.0e-4 (volume); bars about 5x that
    assert res["mixed"][0] <= 5e-4 and res["mixed"][1] <= 5e-4

"""The LDS-staged forward projector against the oracle and against the
gather projector: both evaluate the same Joseph sums with the same FP64
set-up, 32.32 fixed-point z stepping and FP32 blend order, so every output is
bit-identical; every shape of the projector parity cases (ragged tiles,
single views at 0 and 45 degrees (columns of both ray axes in one tile), fine
and coarse detectors whose windows do not fit the staging buffer (the
direct path), flipped and few rows), the fused residual and norm epilogues of
a Landweber step, BF16 copies, and sampled rays at 512^3 x 1440."""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import context, rel_l2, say, to_dev, to_host, workload
from test_gpu_projector import CASES, TOL

pytestmark = pytest.mark.gpu


def _coarse_detector_geom():
    # pixels 3 voxels apart at the axis: a block's 8 columns span more in-plane
    # rows than the staging buffer holds, so its chunks read the copy directly
    views = synth.trajectory(10, 4, 4.0)
    return oracle.Geom(48, 44, 40, 0.7, (0.0, 0.0, 0.0), 24, 20, views)


STAGED_CASES = dict(CASES)
STAGED_CASES["coarse_detector"] = _coarse_detector_geom


@pytest.mark.parametrize("case", list(STAGED_CASES))
def test_staged_projector_matches_oracle_and_gather(case):
    g = STAGED_CASES[case]()
    rng = np.random.Generator(np.random.PCG64(17))
    x = rng.random(g.vol_shape)
    ctx = context(g)
    xd = to_dev(x)
    ctx.set_projector("staged")
    a = to_host(ctx.project(xd))
    ctx.set_projector("gather")
    b = to_host(ctx.project(xd))
    err = rel_l2(a, oracle.project(g, x))
    say("staged projector", case, g.vol_shape, g.stack_shape, "rel L2 %.3e" % err, "identical", np.array_equal(a, b))
    assert err <= TOL
    assert np.array_equal(a, b)


@pytest.mark.parametrize("vt", ["float32", "bfloat16"])
def test_staged_landweber_epilogues_identical(vt):
    """Residual epilogue (transposed, scaled residual) and norm epilogue of a
    Landweber step: the same volume and the same residual norm (FP64 sums of
    the same per-ray values, grouped differently: 1e-12)."""
    import torch
    g = workload("c1").level(1)
    ctx = context(g)
    ctx.set_precision(vt, "float32")
    rng = np.random.Generator(np.random.PCG64(18))
    b = to_dev(oracle.project(g, rng.random(g.vol_shape)))
    alpha = ctx.estimate_step(None, iters=20)
    out = {}
    for variant in ("staged", "gather"):
        ctx.set_projector(variant)
        ctx.set_divergence(1.05)  # a new chain: each variant starts from zero
        v = torch.zeros(g.vol_shape, device="cuda")
        r = [ctx.landweber_step(v, b, alpha) for _ in range(3)]
        out[variant] = (to_host(v), r)
    say("staged Landweber", vt, "volumes identical", np.array_equal(out["staged"][0], out["gather"][0]),
        "residuals", out["staged"][1], out["gather"][1])
    assert np.array_equal(out["staged"][0], out["gather"][0])
    for p, q in zip(out["staged"][1], out["gather"][1]):
        assert abs(p - q) <= 1e-12 * q


def test_staged_bf16_copy_identical():
    import torch
    g = workload("c1").level(1)
    ctx = context(g)
    x = torch.rand(g.vol_shape, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    xb = x.to(torch.bfloat16)
    ctx.set_projector("staged")
    a = to_host(ctx.project(xb, out_dtype=torch.float16))
    ctx.set_projector("gather")
    b = to_host(ctx.project(xb, out_dtype=torch.float16))
    assert np.array_equal(a, b)


def test_staged_full_size_512_sampled():
    """512^3 x 1440 views of 768^2 in FP32 (the automatic choice there):
    sampled rays against the oracle, and the plain sum against the gather
    projector's."""
    import torch
    g = workload("c2")
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(19))
    x = rng.random(g.vol_shape, dtype=np.float32)
    xd = torch.from_numpy(x).cuda()
    ctx.set_projector("auto")
    a = ctx.project(xd)
    rays = np.stack([rng.integers(0, g.n_views, 2000), rng.integers(0, g.nu, 2000), rng.integers(0, g.nv, 2000)], 1)
    got = a.cpu().numpy()[rays[:, 0], rays[:, 2], rays[:, 1]].astype(np.float64)
    e = rel_l2(got, oracle.project_rays(g, x.astype(np.float64), rays))
    ctx.set_projector("gather")
    b = ctx.project(xd)
    same = bool(torch.equal(a, b))
    say("512^3 staged: sampled rays rel L2 %.3e, identical to gather: %s" % (e, same))
    assert e <= TOL and same

"""Parity at the full sizes of the large workloads, on outputs the oracle can
compute one by one: sampled rays of A and sampled voxels of A^T, the adjoint
identity of the GPU pair over the whole arrays, and (tilted geometry) the
per-view geometry derivative on a subset of views.

  * 512^3 volume, 1440 views of 768^2, BF16 volume and FP16 stack storage
    (the mixed-precision layout used at that size);
  * 256^3 volume, 720 views of 384^2 with a source offset and a detector tilt
    (the general-geometry kernels).
"""

import numpy as np
import pytest

import oracle
import synth
from gpu_common import context, rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu


def _samples(rng, g, n_rays=2000, n_vox=150):
    rays = np.stack([rng.integers(0, g.n_views, n_rays), rng.integers(0, g.nu, n_rays),
                     rng.integers(0, g.nv, n_rays)], 1)
    vox = np.stack([rng.integers(0, g.nx, n_vox), rng.integers(0, g.ny, n_vox),
                    rng.integers(0, g.nz, n_vox)], 1)
    return rays, vox


def test_full_size_512_mixed_precision_sampled():
    import torch
    g = workload("c2")
    say("512^3 mixed sampled parity", g.vol_shape, g.stack_shape)
    rng = np.random.Generator(np.random.PCG64(12))
    ctx = context(g)
    # BF16 volume: the oracle takes the stored (rounded) values
    xb = torch.from_numpy(rng.random(g.vol_shape, dtype=np.float32)).to(torch.bfloat16)
    x = xb.float().numpy().astype(np.float64)
    Ax = ctx.project(xb.cuda(), out_dtype=torch.float16)
    rays, vox = _samples(rng, g)
    ref_r = oracle.project_rays(g, x, rays)
    Ax_h = Ax.cpu()
    got_r = Ax_h[rays[:, 0], rays[:, 2], rays[:, 1]].double().numpy()
    e1 = rel_l2(got_r, ref_r)
    del x
    # FP16 stack in, FP32 volume out: the oracle takes the stored values
    yh = torch.from_numpy(rng.random(g.stack_shape, dtype=np.float32)).to(torch.float16)
    Aty = ctx.backproject(yh.cuda())
    y = yh.numpy().astype(np.float64)
    ref_v = oracle.backproject_voxels(g, y, vox)
    del y
    Aty_h = to_host(Aty)
    got_v = Aty_h[vox[:, 2], vox[:, 1], vox[:, 0]]
    e2 = rel_l2(got_v, ref_v)
    # adjoint identity <A x, y> = <x, A^T y> on the GPU pair, in FP64 on the
    # host; the FP16 rounding of A x enters once (<= 2^-11 relative per value)
    dot1 = float(torch.dot(Ax_h.double().reshape(-1), yh.double().reshape(-1)))
    dot2 = float(torch.dot(xb.double().reshape(-1), torch.from_numpy(Aty_h).reshape(-1)))
    e3 = abs(dot1 - dot2) / abs(dot2)
    # per ray: FP16 round-to-nearest moves a value by at most 2^-11 of itself;
    # the FP32 accumulation adds about 1e-6
    worst = float(np.max(np.abs(got_r - ref_r) / np.maximum(np.abs(ref_r), 1e-30)))
    say("  rays rel L2", e1, "worst ray", worst, " voxels rel L2", e2, " adjoint", e3)
    assert worst <= 2.0 ** -11 + 1e-5
    assert e2 <= 1e-5
    # measured 1.5e-7 on MI355X (the FP16 roundings of A x average out)
    assert e3 <= 1e-6


def test_full_size_256_tilted_sampled_and_geometry_gradient():
    import torch
    g0 = workload("c3")
    views = synth.perturb_geometry(g0.views, g0.h, 0.7, -0.6, 0.4)
    g = oracle.Geom(g0.nx, g0.ny, g0.nz, g0.h, g0.origin, g0.nu, g0.nv, views)
    say("256^3 tilted sampled parity", g.vol_shape, g.stack_shape)
    rng = np.random.Generator(np.random.PCG64(13))
    ctx = context(g)
    ph = synth.random_phantom(synth.CONFIGS["c3"], 1003)
    x = synth.voxelize(ph, g.nx, g.h, ss=2)
    xt = to_dev(x)
    Ax = to_host(ctx.project(xt))
    rays, vox = _samples(rng, g)
    e1 = rel_l2(Ax[rays[:, 0], rays[:, 2], rays[:, 1]], oracle.project_rays(g, x, rays))
    y = rng.random(g.stack_shape, dtype=np.float32).astype(np.float64)
    yt = to_dev(y)
    Aty = to_host(ctx.backproject(yt))
    e2 = rel_l2(Aty[vox[:, 2], vox[:, 1], vox[:, 0]], oracle.backproject_voxels(g, y, vox))
    dot1 = float(np.vdot(Ax, y))
    dot2 = float(np.vdot(x, Aty))
    e3 = abs(dot1 - dot2) / (np.linalg.norm(Ax) * np.linalg.norm(y))
    say("  rays rel L2", e1, " voxels rel L2", e2, " adjoint", e3)
    assert e1 <= 1e-5 and e2 <= 1e-5 and e3 <= 1e-6
    # geometry derivative: each view's 12 values depend only on that view, so
    # the oracle runs on a subset of views with the matching cotangent rows
    cot = rng.normal(size=g.stack_shape).astype(np.float32)
    got = ctx.project_geom_grad(xt, to_dev(cot))
    idx = np.sort(rng.choice(g.n_views, 6, replace=False))
    ref = oracle.project_geom_grad(g.subset(idx), x, cot[idx].astype(np.float64))
    e4 = rel_l2(got[idx], ref)
    say("  geometry gradient (6 views) rel L2", e4)
    # FP32 samples (tap differences of the bilinear derivative) summed over a
    # few hundred planes per ray, then over 147456 rays weighted by a random
    # cotangent, which cancels most of the sum: measured 5.0e-5 on MI355X
    # (5.5e-8 on the 32^3 crop, tests/test_gpu_geometry.py, bar 1e-5)
    assert e4 <= 2.5e-4


def test_paper_shaped_volume_with_wide_copies():
    """640 x 640 x 2304 FP32 volume (the paper's volume shape, nx = ny != nz),
    760^2 detector, every 10th view of the 3600-view helix: the projector's
    pair copies (7.7 GB) exceed 4 GiB, so this runs the 64-bit-address
    variant; sampled rays and voxels against the oracle, adjoint identity."""
    import torch
    cfg = synth.PAPER_SHAPED
    nx, nz = cfg.n, synth.PAPER_SHAPED_NZ
    views = synth.helix_trajectory(cfg.n_views, cfg.pixel)[::10]
    g = oracle.Geom(nx, nx, nz, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views)
    say("paper-shaped sampled parity", g.vol_shape, g.stack_shape)
    rng = np.random.Generator(np.random.PCG64(14))
    ctx = context(g)
    xt = torch.from_numpy(rng.random(g.vol_shape, dtype=np.float32)).cuda()
    Ax = ctx.project(xt)
    torch.cuda.synchronize()
    rays, vox = _samples(rng, g, 1000, 100)
    x = xt.cpu().numpy().astype(np.float64)
    ref_r = oracle.project_rays(g, x, rays)
    del x
    Ax_h = Ax.cpu()
    del Ax
    got_r = Ax_h[rays[:, 0], rays[:, 2], rays[:, 1]].double().numpy()
    e1 = rel_l2(got_r, ref_r)
    yt = torch.from_numpy(rng.random(g.stack_shape, dtype=np.float32)).cuda()
    Aty = ctx.backproject(yt).cpu()
    y = yt.cpu().numpy().astype(np.float64)
    ref_v = oracle.backproject_voxels(g, y, vox)
    del y
    got_v = Aty.numpy()[vox[:, 2], vox[:, 1], vox[:, 0]].astype(np.float64)
    e2 = rel_l2(got_v, ref_v)
    dot1 = float(torch.dot(Ax_h.double().reshape(-1), yt.cpu().double().reshape(-1)))
    dot2 = float(torch.dot(xt.cpu().double().reshape(-1), Aty.double().reshape(-1)))
    e3 = abs(dot1 - dot2) / abs(dot2)
    say("  rays rel L2", e1, " voxels rel L2", e2, " adjoint", e3)
    assert e1 <= 1e-5 and e2 <= 1e-5 and e3 <= 1e-6


def test_paper_shaped_volume_ops_sampled():
    """Bilateral filter and soft threshold on the 640 x 640 x 2304 volume
    (943 M voxels, more than the capped grid has threads, so the grid-stride
    loops take several turns): sampled voxels, corners and the last voxel
    against the oracle run on their 3^3 neighbourhoods, which hold every
    input of the filter at that voxel (neighbours outside the grid are
    outside the crop as well)."""
    import torch
    cfg = synth.PAPER_SHAPED
    nx, nz = cfg.n, synth.PAPER_SHAPED_NZ
    views = synth.helix_trajectory(cfg.n_views, cfg.pixel)[::100]
    g = oracle.Geom(nx, nx, nz, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views)
    say("paper-shaped volume ops sampled parity", g.vol_shape)
    rng = np.random.Generator(np.random.PCG64(15))
    ctx = context(g)
    x = rng.random(g.vol_shape, dtype=np.float32) * 0.2
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    ctx.bilateral(xt, out, 1.0, 0.05)
    got = out.cpu().numpy()
    idx = np.stack([rng.integers(0, nz, 300), rng.integers(0, nx, 300), rng.integers(0, nx, 300)], 1)
    idx = np.concatenate([idx, [[nz - 1, nx - 1, nx - 1], [0, 0, 0], [nz - 1, 0, nx - 1], [0, nx - 1, 0]]])
    ref, gv = np.empty(len(idx)), np.empty(len(idx))
    for k, (z, y, xx) in enumerate(idx):
        z0, y0, x0 = max(z - 1, 0), max(y - 1, 0), max(xx - 1, 0)
        crop = x[z0:z + 2, y0:y + 2, x0:xx + 2].astype(np.float64)
        ref[k] = oracle.bilateral(crop, 1.0, 0.05)[z - z0, y - y0, xx - x0]
        gv[k] = got[z, y, xx]
    e1 = rel_l2(gv, ref)
    del got, out
    ctx.soft_threshold(xt, 0.1)
    got = xt.cpu().numpy()
    sel = (idx[:, 0], idx[:, 1], idx[:, 2])
    e2 = rel_l2(got[sel].astype(np.float64), oracle.soft_threshold(x[sel].astype(np.float64), 0.1))
    say("  bilateral rel L2", e1, " soft threshold rel L2", e2)
    assert e1 <= 1e-5 and e2 <= 1e-5

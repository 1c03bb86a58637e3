"""General (tilted-detector) geometry and the geometry derivative on the GPU
against the FP64 oracle."""

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
import synth
from gpu_common import context, rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu


def _tilted(n=32, nu=48, n_views=64, p=(0.6, -0.4, 0.5)):
    g = workload("c0", n=n, nu=nu, nv=nu, n_views=n_views)
    views = synth.perturb_geometry(g.views, g.h, *p)
    return oracle.Geom(g.nx, g.ny, g.nz, g.h, g.origin, g.nu, g.nv, views), g.views


def test_tilted_projector_and_transpose():
    g, _ = _tilted()
    rng = np.random.Generator(np.random.PCG64(31))
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    ctx = context(g)
    Ax = to_host(ctx.project(to_dev(x)))
    Aty = to_host(ctx.backproject(to_dev(y)))
    e1 = rel_l2(Ax, oracle.project(g, x))
    e2 = rel_l2(Aty, oracle.backproject(g, y))
    adj = abs(np.vdot(Ax, y) - np.vdot(x, Aty)) / (np.linalg.norm(Ax) * np.linalg.norm(y))
    say("tilted: A", e1, "A^T", e2, "adjoint", adj)
    assert e1 <= 1e-5 and e2 <= 1e-5 and adj <= 1e-6


def test_geometry_gradient_matches_oracle():
    g, views0 = _tilted(n=32, nu=48, n_views=24)
    rng = np.random.Generator(np.random.PCG64(32))
    x = synth.voxelize(synth.random_phantom(synth.CONFIGS["c0"], 1000), 32, g.h)
    cot = rng.normal(size=g.stack_shape)
    ref = oracle.project_geom_grad(g, x, cot)
    ctx = context(g)
    got = ctx.project_geom_grad(to_dev(x), to_dev(cot))
    e = rel_l2(got, ref)
    say("geometry gradient rel L2", e)
    assert e <= 1e-5
    p = ctx_p = (0.6, -0.4, 0.5)
    gp = mg.geometry_param_grad(views0, got, g.h, *p)
    gp_ref = oracle.geometry_param_grad(views0, ref, g.h, *ctx_p)
    assert np.allclose(gp, gp_ref, rtol=1e-5, atol=1e-8 * np.abs(gp_ref).max())


def test_parameter_gradient_central_differences_on_gpu():
    """d/d(dx, dz, tilt) of 0.5||A(p) x - b||^2 from the kernels against central
    differences with step 1e-3 of the GPU-evaluated objective (FP32 data, FP64
    norms): agreement 1e-2 relative, as the difference crosses interpolation
    kinks."""
    import torch
    g0 = workload("c0", n=32, nu=48, nv=48, n_views=48)
    x = synth.voxelize(synth.random_phantom(synth.CONFIGS["c0"], 1000), 32, g0.h)
    p_true = np.array([0.5, -0.7, 0.4])
    gt = oracle.Geom(32, 32, 32, g0.h, g0.origin, 48, 48, synth.perturb_geometry(g0.views, g0.h, *p_true))
    b = oracle.project(gt, x)
    p = np.array([0.2, -0.3, 0.1])
    ctx = mg.Context(0)
    xt, bt = to_dev(x), to_dev(b)

    def setp(q):
        v = synth.perturb_geometry(g0.views, g0.h, *q)
        ctx.set_geometry(32, 32, 32, g0.h, g0.origin, 48, 48, v)

    def f(q):
        setp(q)
        r = ctx.project(xt) - bt
        return 0.5 * float(torch.sum(r.double() ** 2).item())

    setp(p)
    r = ctx.project(xt) - bt
    grad = mg.geometry_param_grad(g0.views, ctx.project_geom_grad(xt, r.contiguous()), g0.h, *p)
    fd = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1e-3
        fd[k] = (f(p + e) - f(p - e)) / 2e-3
    say("param grad", grad, "fd", fd)
    assert np.allclose(grad, fd, rtol=1e-2, atol=1e-3 * np.abs(fd).max())


def _awkward(kind):
    """32^3 geometries off the usual path of the general kernels: a 25 degree
    detector tilt (columns near the diagonal need both plane families), a
    detector pitched by 0.5 rad about its column axis (rows no longer along
    z), and a source 26 units from the axis with the detector cutting through
    the volume (samples end at the pixel, inside the grid)."""
    g = workload("c0", n=32, nu=48, nv=48, n_views=40)
    vw = g.views.copy()
    if kind == "tilt25":
        vw = synth.perturb_geometry(vw, g.h, 0.3, 0.2, 25.0)
    elif kind == "pitched":
        for r in vw:
            vv = r[9:12].copy()
            lv = np.linalg.norm(vv)
            nrm = np.cross(r[6:9] / np.linalg.norm(r[6:9]), vv / lv)
            r[9:12] = lv * (np.cos(0.5) * vv / lv + np.sin(0.5) * nrm)
    else:  # detector inside the volume
        s = vw[:, 0:3].copy()
        rad = np.linalg.norm(s[:, :2], axis=1, keepdims=True)
        vw[:, 0:2] = s[:, :2] / rad * 26.0
        vw[:, 3:5] = s[:, :2] / rad * 5.0
        vw[:, 6:9] *= 0.5
        vw[:, 9:12] *= 0.15
    return oracle.Geom(g.nx, g.ny, g.nz, g.h, g.origin, g.nu, g.nv, vw)


@pytest.mark.parametrize("kind", ["tilt25", "pitched", "detector_inside"])
def test_awkward_general_geometries(kind):
    g = _awkward(kind)
    say("awkward geometry", kind)
    rng = np.random.Generator(np.random.PCG64(33))
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    ctx = context(g)
    Ax = to_host(ctx.project(to_dev(x)))
    Aty = to_host(ctx.backproject(to_dev(y)))
    e1 = rel_l2(Ax, oracle.project(g, x))
    ref = oracle.backproject(g, y)
    e2 = rel_l2(Aty, ref)
    worst = float(np.max(np.abs(Aty - ref)) / np.max(np.abs(ref)))
    adj = abs(np.vdot(Ax, y) - np.vdot(x, Aty)) / (np.linalg.norm(Ax) * np.linalg.norm(y))
    say("  A", e1, "A^T", e2, "worst voxel / max", worst, "adjoint", adj)
    assert e1 <= 1e-5 and e2 <= 1e-5 and worst <= 1e-5 and adj <= 1e-6

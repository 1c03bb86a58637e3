"""Joint geometry estimation (the paper's Sec. 1 motivation): gradients of
0.5||A(p) mu - b||^2 with respect to a source offset (dx, dz) and a detector
tilt flow from the hand-written adjoint kernels through torch.autograd, and
Adam on p interleaved with reconstruction steps recovers a hidden
misalignment."""

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
import synth
from gpu_common import rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu


def test_autograd_volume_and_geometry_gradients():
    import torch
    from paper_2103_10329_amd.autograd import project
    g = workload("c0", n=32, nu=48, nv=48, n_views=24)
    views = synth.perturb_geometry(g.views, g.h, 0.3, -0.2, 0.3)
    g = oracle.Geom(32, 32, 32, g.h, g.origin, 48, 48, views)
    rng = np.random.Generator(np.random.PCG64(41))
    x = rng.random(g.vol_shape)
    b = rng.random(g.stack_shape)
    ctx = mg.Context(0)
    ctx.set_geometry(32, 32, 32, g.h, g.origin, 48, 48, views)
    xt = to_dev(x).requires_grad_(True)
    vt = torch.from_numpy(views.copy()).requires_grad_(True)
    r = project(xt, vt, ctx) - to_dev(b)
    loss = 0.5 * (r.double() ** 2).sum()
    loss.backward()
    rr = oracle.project(g, x) - b
    e_vol = rel_l2(to_host(xt.grad), oracle.backproject(g, rr))
    e_geo = rel_l2(vt.grad.numpy(), oracle.project_geom_grad(g, x, rr))
    say("autograd: volume grad", e_vol, "geometry grad", e_geo)
    assert e_vol <= 1e-5 and e_geo <= 1e-5


def test_joint_estimation_recovers_misalignment():
    import torch
    cfg = synth.CONFIGS["c3"]
    n, nu, V = 64, 96, 180
    g0 = workload("c3", n=n, nu=nu, nv=nu, n_views=V)
    rng = np.random.Generator(np.random.PCG64(3003))
    p_true = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-0.5, 0.5)])
    ph = synth.random_phantom(cfg, 1003)
    b = synth.add_noise(synth.line_integrals(ph, synth.perturb_geometry(g0.views, g0.h, *p_true), nu, nu),
                        cfg, 2003)
    bt = to_dev(b)
    ctx = mg.Context(0)
    t, rm = oracle.radial_table(n)
    filt = mg.filter_radial(t, rm)
    p = np.zeros(3)
    m1, m2 = np.zeros(3), np.zeros(3)
    lr, beta1, beta2 = 0.08, 0.9, 0.999
    vol = torch.zeros((n, n, n), device="cuda")
    err0 = np.abs(p - p_true)
    for it in range(1, 26):
        views = synth.perturb_geometry(g0.views, g0.h, *p)
        ctx.set_geometry(n, n, n, g0.h, (0, 0, 0), nu, nu, views)
        vol.zero_()
        ctx.multigrid_solve(vol, bt, 2, 2, filt, power_iters=20, want_hist=False)
        r = (ctx.project(vol) - bt).contiguous()
        gp = mg.geometry_param_grad(g0.views, ctx.project_geom_grad(vol, r), g0.h, *p)
        m1 = beta1 * m1 + (1 - beta1) * gp
        m2 = beta2 * m2 + (1 - beta2) * gp * gp
        p = p - lr * (m1 / (1 - beta1 ** it)) / (np.sqrt(m2 / (1 - beta2 ** it)) + 1e-12)
    err = np.abs(p - p_true)
    say("joint estimation: hidden", p_true, "estimated", p, "error", err, "initial", err0)
    # dx (source along the detector columns) and the detector tilt are
    # identifiable; dz moves the source along z with the detector fixed, which
    # for this trajectory is nearly equivalent to a z-translation of the object
    # (absorbed by the reconstruction), so it is reported, not required
    assert err[0] <= 0.5 * err0[0] + 0.05 and err[2] <= 0.5 * err0[2] + 0.02

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


def _identifiability(ctx, views0, n, h, nu, mu, p0, iters=25, step=0.05):
    """How much of each geometry parameter's effect on the data survives when
    the volume is re-solved: J_i = d(A(p) mu)/dp_i by central differences, R_i
    = J_i minus its least-squares fit by A x (CGLS, `iters` iterations).
    Returns diag(R^T R) / diag(J^T J) and the eigenvalues of R^T R scaled by
    diag(J^T J) (the reduced Gauss-Newton matrix of the joint problem)."""
    import torch
    from synth import perturb_geometry
    J = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = step
        ctx.set_geometry(n, n, n, h, (0, 0, 0), nu, nu, perturb_geometry(views0, h, *(p0 + e)))
        jp = ctx.project(mu).double()
        ctx.set_geometry(n, n, n, h, (0, 0, 0), nu, nu, perturb_geometry(views0, h, *(p0 - e)))
        jm = ctx.project(mu).double()
        J.append(((jp - jm) / (2 * step)).reshape(-1))
    ctx.set_geometry(n, n, n, h, (0, 0, 0), nu, nu, perturb_geometry(views0, h, *p0))
    shp = ctx.shapes(0)[1]
    R = []
    for i in range(3):
        bvec = J[i]
        x = torch.zeros((n, n, n), device="cuda", dtype=torch.float64)
        r = bvec.clone()
        sv = ctx.backproject(r.float().reshape(shp)).double()
        pd = sv.clone()
        gam = float((sv * sv).sum())
        for _ in range(iters):
            q = ctx.project(pd.float()).double().reshape(-1)
            al = gam / float((q * q).sum())
            x += al * pd
            r -= al * q
            sv = ctx.backproject(r.float().reshape(shp)).double()
            gn = float((sv * sv).sum())
            pd = sv + (gn / gam) * pd
            gam = gn
        R.append(r)
    Jm = torch.stack(J, 1)
    Rm = torch.stack(R, 1)
    Hf = (Jm.T @ Jm).cpu().numpy()
    Hr = (Rm.T @ Rm).cpu().numpy()
    d = np.sqrt(np.diag(Hf))
    return np.diag(Hr) / np.diag(Hf), np.linalg.eigvalsh(Hr / np.outer(d, d))


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
    # dx (source along the detector columns) and the detector tilt converge
    assert err[0] <= 0.5 * err0[0] + 0.05 and err[2] <= 0.5 * err0[2] + 0.02
    # dz moves the source along z with the detector fixed: apart from the
    # depth-dependent magnification that is a z-translation of the object,
    # which the re-solved volume absorbs.  The reduced Gauss-Newton matrix
    # shows it: the fraction of each parameter's data signature that no
    # volume change can reproduce (measured with the oracle at 32^3: dx 0.93,
    # dz 0.085, tilt 0.90; smallest normalised eigenvalue 0.085, eigenvector
    # along dz).  dz is required to be at least 4x less identifiable than dx
    # and the tilt, and its estimate to stay inside the prior range widened
    # by one voxel (Adam's normalised steps random-walk a flat direction).
    mu_t = to_dev(synth.voxelize(ph, n, g0.h, ss=2))
    ratio, eig = _identifiability(ctx, g0.views, n, g0.h, nu, mu_t, p_true)
    say("identifiability with the volume re-solved (dx, dz, tilt):", ratio, "eigenvalues", eig)
    assert ratio[1] <= 0.25 * min(ratio[0], ratio[2])
    assert abs(p[1]) <= 2.0


def test_joint_estimation_full_size():
    """256^3, 720 views of 384^2 (the full geometry-estimation workload):
    data from the device phantom generators under a hidden misalignment,
    Poisson noise, then Adam on (dx, dz, tilt) alternating with one warm-started
    iteration of Algorithm 1 (3 grids, radial filter; step sizes from the
    unperturbed geometry) per geometry update, 24 updates (the step lowered
    after 12).  dx and the tilt move toward the hidden values.  A tilted detector takes the general-geometry kernels."""
    import time
    import torch
    from paper_2103_10329_amd.learned import poisson_data
    cfg = synth.CONFIGS["c3"]
    n, nu, V = cfg.n, cfg.nu, cfg.n_views
    views0 = synth.trajectory(V, cfg.z_levels, cfg.pixel)
    rng = np.random.Generator(np.random.PCG64(3003))
    p_true = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(-0.5, 0.5)])
    ph = synth.random_phantom(cfg, 1003)
    ctx_true = mg.Context(0)
    ctx_true.set_geometry(n, n, n, cfg.h, (0, 0, 0), nu, nu, synth.perturb_geometry(views0, cfg.h, *p_true))
    gen = torch.Generator(device="cuda").manual_seed(2003)
    b = poisson_data(ctx_true.synth_line_integrals(ph), cfg.noise_level, gen)
    ctx_true.close()
    ctx = mg.Context(0)
    ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), nu, nu, views0)
    t, rm = oracle.radial_table(n)
    filt = mg.filter_radial(t, rm)
    alphas = [ctx.estimate_step(filt, level=lv, iters=20) for lv in range(2)]
    vol = torch.zeros((n, n, n), device="cuda")
    ctx.multigrid_solve(vol, b, 3, 2, filt, alphas=alphas, want_hist=False)
    say("joint estimation 256^3: data and first reconstruction ready")
    p = np.zeros(3)
    m1, m2 = np.zeros(3), np.zeros(3)
    lr, beta1, beta2 = 0.12, 0.9, 0.999
    err0 = np.abs(p - p_true)
    t0 = time.time()
    for it in range(1, 25):
        if it == 13:
            lr = 0.04
        if it > 1:
            ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), nu, nu, synth.perturb_geometry(views0, cfg.h, *p))
            ctx.multigrid_solve(vol, b, 3, 1, filt, alphas=alphas, want_hist=False)
        r = (ctx.project(vol) - b).contiguous()
        gp = mg.geometry_param_grad(views0, ctx.project_geom_grad(vol, r), cfg.h, *p)
        m1 = beta1 * m1 + (1 - beta1) * gp
        m2 = beta2 * m2 + (1 - beta2) * gp * gp
        p = p - lr * (m1 / (1 - beta1 ** it)) / (np.sqrt(m2 / (1 - beta2 ** it)) + 1e-12)
        say("  step", it, "p", p, "%.1fs" % (time.time() - t0))
    err = np.abs(p - p_true)
    say("joint estimation 256^3: hidden", p_true, "estimated", p, "error", err, "initial", err0)
    assert err[0] <= 0.5 * err0[0] + 0.05 and err[2] <= 0.5 * err0[2] + 0.02
    # dz: weakly identifiable, as at 64^3 (see the test above)
    ratio, eig = _identifiability(ctx, views0, n, cfg.h, nu, ctx.synth_voxelize(ph, ss=2), p_true)
    say("identifiability at 256^3 (dx, dz, tilt):", ratio, "eigenvalues", eig)
    assert ratio[1] <= 0.25 * min(ratio[0], ratio[2])
    assert abs(p[1]) <= 2.0

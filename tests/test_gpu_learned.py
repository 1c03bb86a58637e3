"""Learned preconditioner inside Algorithm 1: device phantom generators
against the CPU generator, the residual judge and fallback, and a short
training run on solver-generated pairs compared with the plain filter."""

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
import synth
from gpu_common import rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu


def _ctx(g):
    ctx = mg.Context(0)
    ctx.set_geometry(g.nx, g.ny, g.nz, g.h, g.origin, g.nu, g.nv, g.views)
    return ctx


def test_device_phantom_generators_match_cpu():
    g = workload("c0")
    cfg = synth.CONFIGS["c1"]
    ph = synth.random_phantom(cfg, 1001)
    ctx = _ctx(g)
    b = to_host(ctx.synth_line_integrals(ph))
    mu = to_host(ctx.synth_voxelize(ph, ss=4))
    e1 = rel_l2(b, synth.line_integrals(ph, g.views, g.nu, g.nv))
    e2 = rel_l2(mu, synth.voxelize(ph, 32, g.h, ss=4))
    say("device line integrals", e1, "voxelize", e2)
    assert e1 <= 1e-6 and e2 <= 1e-6


def _problem(n=64, nu=96, n_views=120, seed=1001):
    g = workload("c1", n=n, nu=nu, nv=nu, n_views=n_views)
    cfg = synth.CONFIGS["c1"]
    ph = synth.random_phantom(cfg, seed)
    b = synth.add_noise(synth.line_integrals(ph, g.views, g.nu, g.nv), cfg, seed + 1000)
    t, r = oracle.radial_table(n)
    return g, b, mg.filter_radial(t, r), synth.voxelize(ph, n, g.h, ss=4)


def test_identity_network_and_fallback():
    import torch
    from paper_2103_10329_amd.learned import he_init
    g, b, filt, _ = _problem()
    ctx = _ctx(g)
    bt = to_dev(b)
    alphas = [ctx.estimate_step(filt, level=lv, iters=30) for lv in range(2)]
    plain = torch.zeros(g.vol_shape, device="cuda")
    ctx.multigrid_solve(plain, bt, 3, 2, filt, alphas=alphas, want_hist=False)
    # identity network (zero last layer): u + f(u) = u, so accepted or not the
    # iterate equals the plain one up to the rounding of mu + alpha*p (the plain
    # step fuses it into one FMA)
    ctx.cnn_set_weights(mg.cnn_flatten(he_init(0)))
    ctx.learned_stats()
    v = torch.zeros(g.vol_shape, device="cuda")
    ctx.multigrid_solve(v, bt, 3, 2, filt, alphas=alphas, want_hist=False, learned=True)
    acc, rej = ctx.learned_stats()
    e = rel_l2(to_host(v), to_host(plain))
    say("identity network vs plain", e, "accepted", acc, "rejected", rej)
    assert e <= 1e-5 and acc + rej == 2
    # adversarial network: every step must fall back to the plain update
    p = he_init(1)
    p[3][0] = np.random.Generator(np.random.PCG64(5)).normal(0, 50.0, size=p[3][0].shape)
    ctx.cnn_set_weights(mg.cnn_flatten(p))
    v = torch.zeros(g.vol_shape, device="cuda")
    ctx.multigrid_solve(v, bt, 3, 2, filt, alphas=alphas, want_hist=False, learned=True)
    acc, rej = ctx.learned_stats()
    say("adversarial network: accepted", acc, "rejected", rej)
    e = rel_l2(to_host(v), to_host(plain))
    assert rej == 2 and acc == 0 and e <= 1e-5


def test_short_training_gains_over_plain_filter():
    """Pairs from 48 phantoms (2 iterations each) at 64^3 / 120 views,
    600 Adam steps on 32^3 crops; on 3 held-out phantoms the learned
    iteration's image error after 2 iterations is below the plain one's."""
    import torch
    from paper_2103_10329_amd import learned as L
    n, nu, V = 64, 96, 120
    g = workload("c1", n=n, nu=nu, nv=nu, n_views=V)
    ctx = _ctx(g)
    t, r = oracle.radial_table(n)
    filt = mg.filter_radial(t, r)
    alphas = [ctx.estimate_step(filt, level=lv, iters=30) for lv in range(2)]
    # the workload's phantom distribution on the small grid
    store = L.PairStore((n, n, n), 96)
    import synth.geometry as sg
    small = sg.ScanConfig("c1s", n, nu, nu, V, 8, 60, (0.01, 0.3), "poisson", 1e4, levels=3)
    L.generate_pairs(ctx, small, range(20000, 20048), 3, filt, alphas, store, log=None)
    sigma = float(1.0 / store.e[: store.n].float().std().item())
    ctx.cnn_set_weights(mg.cnn_flatten(L.he_init(0)))
    losses = L.train(ctx, store, 600, 2e-3, 32, sigma, seed=1, log=None)
    ctx.cnn_set_weights(L.fold_scale(ctx.cnn_get_weights(), sigma))
    say("training loss", losses[0][1], "->", losses[-1][1])
    gains = []
    for seed in (30000, 30001, 30002):
        ph = synth.random_phantom(small, seed)
        truth = ctx.synth_voxelize(ph, ss=4)
        gen = torch.Generator(device="cuda").manual_seed(seed)
        b = L.poisson_data(ctx.synth_line_integrals(ph), small.noise_level, gen)
        errs = []
        for learned in (False, True):
            v = torch.zeros((n, n, n), device="cuda")
            ctx.multigrid_solve(v, b, 3, 2, filt, alphas=alphas, want_hist=False, learned=learned)
            errs.append(float(torch.linalg.vector_norm(v - truth) / torch.linalg.vector_norm(truth)))
        gains.append(errs)
    acc, rej = ctx.learned_stats()
    say("held-out image error plain vs learned", gains, "accepted", acc, "rejected", rej)
    assert np.mean([e[1] for e in gains]) < np.mean([e[0] for e in gains])


def _masked_err(v, truth, mask):
    import torch
    t = truth[mask].double()
    return float(torch.linalg.vector_norm(v[mask].double() - t) / torch.linalg.vector_norm(t))


def test_trained_weights_gain_at_128():
    """The shipped weights (trained on 900 phantoms of the 128^3 / 360-view
    distribution) on 4 phantoms outside the training seeds: masked image
    error after 2 iterations below the plain method's on every one."""
    import torch
    from paper_2103_10329_amd import learned as L
    cfg = synth.CONFIGS["c4"]
    ctx = L.make_context(cfg, synth.trajectory(cfg.n_views, cfg.z_levels, cfg.pixel))
    t, r = mg.ramp_table(cfg.n)
    filt = mg.filter_radial(t, r)
    alphas = [ctx.estimate_step(filt, level=lv, iters=30) for lv in range(cfg.levels - 1)]
    ctx.cnn_set_weights(L.load_weights())
    rows, acc, rej = L.evaluate(ctx, cfg, range(40000, 40004), cfg.levels, filt, alphas)
    say("shipped weights at 128^3: (seed, plain, learned)", rows, "accepted", acc, "rejected", rej)
    assert all(lr < pl for _, pl, lr in rows)


def test_trained_weights_at_512_mixed_precision():
    """The same weights run inside Algorithm 1 at 512^3 with 1440 views of
    768^2 (4 grids, BF16 volume copy and FP16 stacks): the residual judge keeps
    the learned iteration no worse in residual than the plain one; image
    errors and wall times are reported."""
    import time
    import torch
    from paper_2103_10329_amd import learned as L
    cfg = synth.CONFIGS["c2"]
    n = cfg.n
    ctx = L.make_context(cfg, synth.trajectory(cfg.n_views, cfg.z_levels, cfg.pixel))
    ctx.set_precision("bfloat16", "float16")
    ph = synth.random_phantom(cfg, 1002)
    truth = ctx.synth_voxelize(ph, ss=2)
    gen = torch.Generator(device="cuda").manual_seed(2002)
    b = L.poisson_data(ctx.synth_line_integrals(ph), cfg.noise_level, gen).half()
    t, r = mg.ramp_table(n)
    filt = mg.filter_radial(t, r)
    alphas = [ctx.estimate_step(filt, level=lv, iters=20) for lv in range(cfg.levels - 1)]
    ctx.cnn_set_weights(L.load_weights())
    mask = torch.from_numpy(synth.evaluation_mask(n, cfg.h)).cuda()
    bf = b.float()
    out = {}
    for learned in (False, True):
        v = torch.zeros((n, n, n), device="cuda")
        ctx.learned_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.multigrid_solve(v, b, cfg.levels, 2, filt, alphas=alphas, want_hist=False, learned=learned)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res = float(torch.linalg.vector_norm((bf - ctx.project(v)).double()) / torch.linalg.vector_norm(bf.double()))
        out[learned] = (res, _masked_err(v, truth, mask), dt, ctx.learned_stats())
        del v
    say("512^3 (rel residual, masked error, seconds, (accepted, rejected)) plain", out[False], "learned", out[True])
    assert out[True][0] <= out[False][0] * 1.01


def test_judge_over_view_subset():
    """On a scan of 720 views (256^3, 384^2 detector) the judge compares the
    residual before and after the network's refinement over every second view
    (the staged projector's view-subset order; the value before the update
    summed from the Landweber projection's block partials).  With two grids
    and no coarse passes one iteration is one fine-grid step from the given
    volume, so both values can be formed independently: full projections of
    mu and of mu + f(u) (u captured from the solve, f the network), squared
    residuals summed in FP64 over the even views.  The kept iterate follows
    r1 < r0."""
    import torch
    from paper_2103_10329_amd import learned as L
    cfg = synth.CONFIGS["c3"]
    n = cfg.n
    ctx = L.make_context(cfg, synth.trajectory(cfg.n_views, cfg.z_levels, cfg.pixel))
    ph = synth.random_phantom(cfg, 1031)
    gen = torch.Generator(device="cuda").manual_seed(2031)
    b = L.poisson_data(ctx.synth_line_integrals(ph), cfg.noise_level, gen)
    mu0 = 0.5 * ctx.synth_voxelize(ph, ss=1)
    t, r = mg.ramp_table(n)
    filt = mg.filter_radial(t, r)
    alpha = ctx.estimate_step(filt, level=0, iters=20)
    ctx.cnn_set_weights(L.load_weights())
    u = torch.empty_like(mu0)
    v = mu0.clone()
    ctx.learned_stats()
    ctx.multigrid_solve(v, b, 2, 1, filt, alphas=[alpha], coarse_passes=0, want_hist=False, learned=True,
                        capture_update=u)
    acc, rej = ctx.learned_stats()
    r0, r1, k = ctx.learned_judge()
    even = torch.arange(cfg.n_views, device="cuda") % 2 == 0
    ref0 = float(((b - ctx.project(mu0)).double() ** 2)[even].sum())
    ref1 = float(((b - ctx.project(mu0 + ctx.cnn_forward(u))).double() ** 2)[even].sum())
    say("judge over every %d-th view: r0 %.9e (ref %.9e), r1 %.9e (ref %.9e), kept %d rejected %d"
        % (k, r0, ref0, r1, ref1, acc, rej))
    assert k == 2
    assert abs(r0 - ref0) <= 1e-9 * ref0 and abs(r1 - ref1) <= 1e-9 * ref1
    assert (acc, rej) == ((1, 0) if r1 < r0 else (0, 1))

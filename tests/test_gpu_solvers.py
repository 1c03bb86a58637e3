"""GPU parity of the iterations (step-size estimate, Landweber/SIRT,
preconditioned Landweber, OS-EMTR, Algorithm 1) against the FP64 oracle run
with identical parameters, plus properties at the full 128^3 size."""

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


def _c0():
    d = synth.make_dataset("c0")
    return workload("c0"), d


@pytest.mark.parametrize("kind", ["identity", "stencil27", "radial"])
def test_estimate_step(kind):
    g, _ = _c0()
    ctx = context(g)
    if kind == "identity":
        fo, fg = None, None
    elif kind == "stencil27":
        fo, fg = oracle.filter_stencil27(), mg.filter_eq5()
    else:
        t, r = oracle.radial_table(g.nx)
        fo, fg = oracle.filter_radial(t, r), mg.filter_radial(t, r)
    say("estimate_step", kind)
    a_ref = 1.0 / oracle.power_iteration(g, fo, iters=30, seed=0)
    a = ctx.estimate_step(fg, iters=30, seed=0)
    say("  alpha", a, a_ref)
    assert abs(a - a_ref) / a_ref <= 1e-5


def test_sirt_20_iterations_c0():
    g, d = _c0()
    ctx = context(g)
    alpha = 1.0 / oracle.power_iteration(g, None, iters=30, seed=0)
    mu = np.zeros(g.vol_shape)
    vol = to_dev(mu)
    b = to_dev(d["b"])
    res_o, res_g = [], []
    for _ in range(20):
        mu, r = oracle.landweber_step(g, mu, d["b"], alpha, None)
        res_o.append(r)
        res_g.append(ctx.landweber_step(vol, b, alpha))
    err = rel_l2(to_host(vol), mu)
    herr = np.max(np.abs(np.array(res_g) - res_o) / np.array(res_o))
    say("SIRT c0 rel L2", err, "residual history", herr)
    assert err <= 1e-5 and herr <= 1e-5
    assert all(res_o[i + 1] < res_o[i] for i in range(19))


@pytest.mark.parametrize("kind", ["stencil27", "radial"])
def test_preconditioned_landweber_c0(kind):
    g, d = _c0()
    ctx = context(g)
    if kind == "stencil27":
        fo, fg = oracle.filter_stencil27(), mg.filter_eq5()
    else:
        t, r = oracle.radial_table(g.nx)
        fo, fg = oracle.filter_radial(t, r), mg.filter_radial(t, r)
    alpha = 1.0 / oracle.power_iteration(g, fo, iters=30, seed=0)
    mu = np.zeros(g.vol_shape)
    vol = to_dev(mu)
    b = to_dev(d["b"])
    for _ in range(5):
        mu, r = oracle.landweber_step(g, mu, d["b"], alpha, fo)
        rg = ctx.landweber_step(vol, b, alpha, fg)
        assert abs(rg - r) / r <= 1e-5
    err = rel_l2(to_host(vol), mu)
    say("PL", kind, "rel L2", err)
    assert err <= 1e-5


def test_landweber_f16_data():
    import torch
    g, d = _c0()
    ctx = context(g)
    alpha = 1.0 / oracle.power_iteration(g, None, iters=30, seed=0)
    b16 = d["b"].astype(np.float16)
    mu, r = oracle.landweber_step(g, np.zeros(g.vol_shape), b16.astype(np.float64), alpha, None)
    vol = to_dev(np.zeros(g.vol_shape))
    rg = ctx.landweber_step(vol, torch.from_numpy(b16).cuda(), alpha)
    assert rel_l2(to_host(vol), mu) <= 1e-5 and abs(rg - r) / r <= 1e-5


def test_osemtr_coarse_grid():
    g = workload("c1").level(2)  # 32^3, 360 x 48^2
    d = synth.make_dataset("c1", truth=False)
    b = oracle.restrict_stack(oracle.restrict_stack(d["b"]))
    mu0 = np.zeros(g.vol_shape)
    say("osemtr 32^3 x 360")
    ref = oracle.osemtr(g, mu0, b, M=8, passes=2)
    ctx = context(g)
    vol = to_dev(mu0)
    ctx.osemtr(vol, to_dev(b), subsets=8, passes=2)
    err = rel_l2(to_host(vol), ref)
    say("  rel L2", err)
    assert err <= 1e-5


@pytest.mark.parametrize("case", ["64cube", "ragged"])
def test_osemtr_deep_grids(case):
    """OS-EMTR on grids deeper than 32 (the plane-blocked back-projector with
    two outputs): 64^3 x 360 views of 96^2 (one pass of 8 subsets), and a
    ragged 37 x 29 x 70 grid with a 53 x 71 detector (row blocks with tails,
    z range split in two)."""
    if case == "64cube":
        g = workload("c1").level(1)
        d = synth.make_dataset("c1", truth=False)
        b = oracle.restrict_stack(d["b"])
        M, passes = 8, 1
    else:
        views = synth.trajectory(48, 4, 72.0 / 53)
        views[:, 9:12] = np.array([0.0, 0.0, 0.45])
        g = oracle.Geom(37, 29, 70, 0.45, (0.3, -0.2, 0.1), 53, 71, views)
        ph = synth.random_phantom(synth.CONFIGS["c0"], 1000)
        b = 0.25 * synth.line_integrals(ph, g.views, g.nu, g.nv)  # line integrals up to about 3
        M, passes = 4, 2
    mu0 = np.zeros(g.vol_shape)
    say("osemtr", case, g.vol_shape, g.stack_shape)
    ref = oracle.osemtr(g, mu0, b, M=M, passes=passes)
    ctx = context(g)
    vol = to_dev(mu0)
    ctx.osemtr(vol, to_dev(b), subsets=M, passes=passes)
    err = rel_l2(to_host(vol), ref)
    say("  rel L2", err)
    assert err <= 1e-5


def _mg_case(n, nu, n_views, levels, n_outer, lam, bil, kind="radial"):
    g = workload("c1", n=n, nu=nu, nv=nu, n_views=n_views)
    ph = synth.random_phantom(synth.CONFIGS["c1"], 1001)
    b = synth.add_noise(synth.line_integrals(ph, g.views, g.nu, g.nv), synth.CONFIGS["c1"], 2001)
    if kind == "radial":
        t, r = oracle.radial_table(n)
        fo, fg = oracle.filter_radial(t, r), mg.filter_radial(t, r)
    else:
        fo, fg = oracle.filter_stencil27(), mg.filter_eq5()
    alphas = [1.0 / oracle.power_iteration(g.level(lv), fo, iters=30, seed=0) for lv in range(max(levels - 1, 1))]
    return g, b, fo, fg, alphas


@pytest.mark.parametrize("preset", ["parity", "paper", "stencil", "one_level"])
def test_multigrid_small(preset):
    levels, n_outer, lam, bil, kind = {
        "parity": (3, 2, 0.0, None, "radial"),
        "paper": (3, 2, 1e-3, (1.0, 0.05), "radial"),
        "stencil": (2, 1, 0.0, None, "stencil"),
        "one_level": (1, 2, 1e-3, (1.0, 0.05), "radial"),
    }[preset]
    g, b, fo, fg, alphas = _mg_case(32, 48, 64, levels, n_outer, lam, bil, kind)
    say("multigrid", preset)
    ref, hist_ref = oracle.multigrid(g, np.zeros(g.vol_shape), b, levels, n_outer, fo, alphas, lam=lam,
                                     bilateral_on=bil is not None, sigma_s=(bil or (1, 1))[0],
                                     sigma_r=(bil or (1, 1))[1], coarse_M=8, coarse_passes=2)
    ctx = context(g)
    vol = to_dev(np.zeros(g.vol_shape))
    hist = ctx.multigrid_solve(vol, to_dev(b), levels, n_outer, fg, alphas=alphas, lam=lam, bilateral=bil)
    err = rel_l2(to_host(vol), ref)
    herr = np.max(np.abs(hist - hist_ref) / hist_ref)
    say("  rel L2", err, "hist", herr)
    assert err <= 1e-5 and herr <= 1e-5


def test_multigrid_64_three_levels():
    g, b, fo, fg, alphas = _mg_case(64, 96, 120, 3, 1, 0.0, None)
    say("multigrid 64^3 x 120 views")
    ref, hist_ref = oracle.multigrid(g, np.zeros(g.vol_shape), b, 3, 1, fo, alphas)
    ctx = context(g)
    vol = to_dev(np.zeros(g.vol_shape))
    hist = ctx.multigrid_solve(vol, to_dev(b), 3, 1, fg, alphas=alphas)
    err = rel_l2(to_host(vol), ref)
    say("  rel L2", err)
    assert err <= 1e-5 and np.max(np.abs(hist - hist_ref) / hist_ref) <= 1e-5


def test_multigrid_full_c1_properties():
    """128^3, 360 views of 192^2, 3 levels, radial filter: the residual of
    every grid falls between the two outer iterations, two iterations give
    the same volume as one plus one (resume), and repeat runs are identical."""
    import torch
    d = synth.make_dataset("c1", truth=True)
    g = workload("c1")
    ctx = context(g)
    t, r = oracle.radial_table(g.nx)
    fg = mg.filter_radial(t, r)
    path = os.path.join(HERE, "golden", "alphas.json")
    alphas = json.load(open(path))["c1"]["radial_ramp"] if os.path.exists(path) else None
    b = to_dev(d["b"])
    v2 = torch.zeros(g.vol_shape, device="cuda")
    hist = ctx.multigrid_solve(v2, b, 3, 2, fg, alphas=alphas)
    say("c1 history", hist)
    assert np.all(hist[1] < hist[0])
    v11 = torch.zeros(g.vol_shape, device="cuda")
    ctx.multigrid_solve(v11, b, 3, 1, fg, alphas=alphas)
    ctx.multigrid_solve(v11, b, 3, 1, fg, alphas=alphas)
    assert torch.equal(v2, v11)
    # image error against the ground truth decreases
    mu = d["mu"]
    e = rel_l2(to_host(v2), mu)
    say("c1 rel error vs phantom after 2 PMG iterations", e)
    assert e < 0.6

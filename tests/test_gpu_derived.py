"""Preconditioners derived from the scan's own point-spread function: the
transfer function of A^T A, its shell averages and the inverse filter on the
GPU against the FP64 oracle, and the derived filters inside Algorithm 1 next
to the ramp filter."""

import math

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
import synth
from gpu_common import context, rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu


def _ambiguous_shells(shape, n_table, rho_max, rel=4e-7):
    """Lower shell index of every frequency whose shell coordinate
    t = rho/rho_max (n_table - 1) lies within rel*(t+1) of a half-way point
    t = i + 1/2 (FP32 evaluation of rho may round it to either side)."""
    k = [np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n) / n for n in shape]
    kz, ky, kx = np.meshgrid(*k, indexing="ij")
    t = 2 * np.sqrt(kx ** 2 + ky ** 2 + kz ** 2) / rho_max * (n_table - 1)
    near = np.abs((t - 0.5) - np.round(t - 0.5)) <= rel * (t + 1.0)
    return np.round(t[near] - 0.5).astype(np.int64)


def test_transfer_function_and_filter_match_oracle():
    g = workload("c1").level(1)   # 64^3, 360 views of 96^2
    ctx = context(g)
    T_gpu = ctx.psf_spectrum()
    T_or = oracle.psf_spectrum(g)
    e_T = rel_l2(to_host(T_gpu), T_or)
    n_table, rho_max = 257, math.sqrt(3.0)
    prof, cnt = ctx.radial_profile(T_gpu, n_table=n_table, rho_max=rho_max)
    prof_or, cnt_or = oracle.radial_profile(T_or, n_table, rho_max)
    # The library places rho in FP32, the oracle in FP64: a frequency whose
    # shell coordinate lies within FP32 rounding of a half-way point may fall
    # in either neighbouring shell.  Enumerate those frequencies; counts may
    # differ only by them, and shell means are compared on the other shells.
    amb_lo = _ambiguous_shells(g.vol_shape, n_table, rho_max)
    d = cnt.astype(np.int64) - cnt_or.astype(np.int64)
    allowed = np.zeros(n_table, dtype=np.int64)
    np.add.at(allowed, amb_lo, 1)
    np.add.at(allowed, np.minimum(amb_lo + 1, n_table - 1), 1)
    assert np.all(np.abs(d) <= allowed), np.nonzero(np.abs(d) > allowed)
    assert cnt.sum() == cnt_or.sum() or len(amb_lo) > 0
    touched = np.zeros(n_table, dtype=bool)
    touched[amb_lo] = True
    touched[np.minimum(amb_lo + 1, n_table - 1)] = True
    m = (cnt > 0) & (cnt_or > 0) & ~touched
    say("shell ambiguity: %d frequencies within FP32 rounding of a shell boundary" % len(amb_lo))
    e_p = rel_l2(prof[m], prof_or[m])
    H_gpu = to_host(ctx.transfer_from_spectrum(T_gpu, 1e-2))
    H_or = oracle.transfer_from_spectrum(T_or, 1e-2)
    e_H = rel_l2(H_gpu, H_or)
    # the TRANSFER filter itself, with the oracle's H on both sides
    rng = np.random.Generator(np.random.PCG64(51))
    x = rng.normal(size=g.vol_shape)
    Hd = to_dev(H_or)
    y = to_host(ctx.precondition(to_dev(x), mg.filter_transfer([Hd])))
    e_f = rel_l2(y, oracle.transfer_filter(x, H_or))
    say("T rel L2", e_T, "profile", e_p, "H", e_H, "filter", e_f, "T[0]", T_or.flat[0])
    assert e_T <= 1e-5 and e_p <= 1e-5 and e_H <= 1e-5 and e_f <= 1e-5


def test_derived_filters_in_algorithm1():
    """c1 (128^3, 360 views, Poisson data): 2 iterations of Algorithm 1 with
    the ramp filter, with 1/T-bar(rho) from the measured shell averages, and
    with the anisotropic 1/max(T(k), 0.03 T(0)) of each grid.  All converge;
    the anisotropic filter reaches a clearly lower residual and image error
    than the ramp (measured 0.056 vs 0.097 and 0.175 vs 0.266)."""
    import torch
    g = workload("c1")
    ctx = context(g)
    d = synth.make_dataset("c1", truth=True)
    b = to_dev(d["b"])
    truth = to_dev(d["mu"])
    mask = torch.from_numpy(synth.evaluation_mask(128, g.h)).cuda()
    n_table, rho_max = 1025, math.sqrt(3.0)
    Ts = [ctx.psf_spectrum(level=lv) for lv in range(2)]
    prof, cnt = ctx.radial_profile(Ts[0], n_table=n_table, rho_max=rho_max)
    ok = cnt > 0
    rho = np.linspace(0, rho_max, n_table)
    tbar = np.interp(rho, rho[ok], prof[ok])
    derived_radial = mg.filter_radial((1.0 / np.maximum(tbar, 1e-2 * tbar[0])).astype(np.float32), rho_max)
    derived_transfer = ctx.derived_filter(2)   # floor 0.03 T[0]
    t, r = mg.ramp_table(128)
    filters = {"ramp": mg.filter_radial(t, r), "derived radial": derived_radial,
               "derived transfer": derived_transfer}
    bn = float(torch.linalg.vector_norm(b.double()))
    out = {}
    for name, f in filters.items():
        alphas = [ctx.estimate_step(f, level=lv, iters=30) for lv in range(2)]
        v = torch.zeros((128,) * 3, device="cuda")
        res = []
        for _ in range(2):
            ctx.multigrid_solve(v, b, 3, 1, f, alphas=alphas, want_hist=False)
            res.append(float(torch.linalg.vector_norm((b - ctx.project(v)).double())) / bn)
        t_ = truth[mask].double()
        err = float(torch.linalg.vector_norm(v[mask].double() - t_) / torch.linalg.vector_norm(t_))
        out[name] = (res, err)
    say("2 iterations (relative residuals, masked image error):", out)
    for name, (res, err) in out.items():
        assert res[1] < res[0] < 1.0 and err < 1.0, name
    assert out["derived transfer"][0][1] < 0.8 * out["ramp"][0][1]
    assert out["derived transfer"][1] < 0.8 * out["ramp"][1]

"""GPU parity of the preconditioners, grid transfers and regularisers
against the FP64 oracle (relative L2 <= 1e-5)."""

import math

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg
from gpu_common import context, rel_l2, say, to_dev, to_host, workload

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _geom(nx, ny, nz):
    """c0's views around a grid of the given shape, voxel at most 0.5 and the
    box at most 32 units long (the source stays outside)."""
    g = workload("c0")
    return oracle.Geom(nx, ny, nz, min(0.5, 32.0 / max(nx, ny, nz)), (0, 0, 0), g.nu, g.nv, g.views)


@pytest.mark.parametrize("shape", [(32, 32, 32), (70, 29, 37), (8, 8, 8), (3, 4, 5)])
def test_stencil27_eq5(shape):
    nz, ny, nx = shape
    g = _geom(nx, ny, nz)
    ctx = context(g)
    x = np.random.Generator(np.random.PCG64(1)).random(shape)
    say("stencil27", shape)
    out = to_host(ctx.precondition(to_dev(x), mg.filter_eq5()))
    assert rel_l2(out, oracle.stencil27(x)) <= TOL
    # in place
    t = to_dev(x)
    ctx.precondition(t, mg.filter_eq5(), out=t)
    assert rel_l2(to_host(t), oracle.stencil27(x)) <= TOL


def test_stencil27_arbitrary_taps():
    g = _geom(16, 12, 10)
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(2))
    taps = rng.normal(size=(3, 3, 3))
    x = rng.random(g.vol_shape)
    out = to_host(ctx.precondition(to_dev(x), mg.filter_stencil27(taps)))
    assert rel_l2(out, oracle.stencil27(x, taps)) <= TOL


# Line lengths per stage path of the in-LDS FFT: radix 2 only (<= 64 points),
# one radix-2 stage then radix 4 (128, 512), radix 4 only (256, 1024); each
# length appears on every axis somewhere, 256^3 and 512^3 are the filtered
# grids of the 256^3 and 512^3 workloads.
@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 64, 64), (128, 128, 128), (16, 32, 64), (64, 8, 2),
                                   (256, 256, 256), (512, 16, 32), (16, 512, 32), (16, 32, 512),
                                   (4, 8, 1024), (8, 1024, 4), (1024, 4, 8), (256, 32, 128)])
def test_radial_filter(shape):
    nz, ny, nx = shape
    g = _geom(nx, ny, nz)
    ctx = context(g)
    x = np.random.Generator(np.random.PCG64(3)).random(shape)
    table, rho_max = oracle.radial_table(max(shape))
    say("radial", shape)
    out = to_host(ctx.precondition(to_dev(x), mg.filter_radial(table, rho_max)))
    ref = oracle.radial_filter(x, table, rho_max)
    err = rel_l2(out, ref)
    say("  rel L2", err)
    assert err <= TOL


def test_radial_filter_rejects_non_power_of_two():
    g = _geom(30, 32, 32)
    ctx = context(g)
    table, rho_max = oracle.radial_table(32)
    with pytest.raises(mg.MgctError) as e:
        ctx.precondition(to_dev(np.zeros(g.vol_shape)), mg.filter_radial(table, rho_max))
    assert e.value.code == mg.MGCT_ERR_NOT_IMPLEMENTED


def test_identity_filter_is_copy():
    g = _geom(8, 8, 8)
    ctx = context(g)
    x = np.random.Generator(np.random.PCG64(4)).random(g.vol_shape)
    out = to_host(ctx.precondition(to_dev(x), mg.filter_identity()))
    assert np.array_equal(out, x.astype(np.float32))


def test_grid_transfers():
    g = workload("c1").level(1)  # 64^3, 360 x 96^2
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(5))
    import torch
    x = rng.random(g.vol_shape)
    c = torch.empty((32, 32, 32), device="cuda")
    ctx.restrict_volume(to_dev(x), c, level=0)
    assert rel_l2(to_host(c), oracle.restrict_volume(x)) <= TOL
    b = rng.random(g.stack_shape)
    cb = torch.empty((g.n_views, g.nv // 2, g.nu // 2), device="cuda")
    ctx.restrict_stack(to_dev(b), cb, level=0)
    assert rel_l2(to_host(cb), oracle.restrict_stack(b)) <= TOL
    cn, co, f = rng.random((32, 32, 32)), rng.random((32, 32, 32)), rng.random(g.vol_shape)
    ft = to_dev(f)
    ctx.prolong_add(to_dev(cn), to_dev(co), ft, level=0)
    assert rel_l2(to_host(ft), f + oracle.prolongate(cn - co)) <= TOL


def test_soft_threshold_and_bilateral():
    g = _geom(37, 29, 20)
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(6))
    x = rng.normal(size=g.vol_shape) * 0.1
    t = to_dev(x)
    ctx.soft_threshold(t, 0.05)
    assert rel_l2(to_host(t), oracle.soft_threshold(x, 0.05)) <= TOL
    import torch
    y = rng.random(g.vol_shape) * 0.2
    out = torch.empty(g.vol_shape, device="cuda")
    ctx.bilateral(to_dev(y), out, 1.0, 0.05)
    assert rel_l2(to_host(out), oracle.bilateral(y, 1.0, 0.05)) <= TOL
    with pytest.raises(mg.MgctError):
        ctx.bilateral(out, out, 1.0, 0.05)


def test_transfer_filter_radix4_only_lines():
    """TRANSFER kind (a per-frequency H(k)) on 256^3: every axis takes the
    radix-4-only stage path."""
    shape = (256, 256, 256)
    g = _geom(256, 256, 256)
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(7))
    x = rng.normal(size=shape)
    H = 0.2 + rng.random(shape)
    say("transfer", shape)
    y = to_host(ctx.precondition(to_dev(x), mg.filter_transfer([to_dev(H)])))
    err = rel_l2(y, oracle.transfer_filter(x, H))
    say("  rel L2", err)
    assert err <= TOL

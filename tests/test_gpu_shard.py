"""View sharding rehearsed on one GPU.  A K-GPU run would give each GPU every
K-th view (round robin, so that each share covers the whole angular range):
A over a share must return exactly the rows of A over all views, since each
ray's sum depends on its own view only, and the back-projections of the
shares must add up to the back-projection of the whole stack, since Aᵀ is a
sum over views (Sec. 2.1, eq. 2: the gradient step back-projects every
view's residual), the sum exchange a multi-GPU step would make.  Only the
order of the floating-point sums differs there.  The full Aᵀ is pinned to
the oracle; both projector kernels are covered."""

import numpy as np
import pytest

import oracle
from gpu_common import context, rel_l2, say, to_dev, to_host, workload
from test_gpu_projector import TOL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("proj", ["gather", "staged"])
@pytest.mark.parametrize("k", [3, 4])
def test_view_shares_compose(proj, k):
    g = workload("c1", n=64, nu=96, nv=96, n_views=120)
    rng = np.random.Generator(np.random.PCG64(23))
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    xd, yd = to_dev(x), to_dev(y)
    full = context(g)
    full.set_projector(proj)
    a_full = to_host(full.project(xd))
    b_full = to_host(full.backproject(yd))
    full.close()
    err_full = rel_l2(b_full, oracle.backproject(g, y))
    assert err_full <= TOL
    acc = np.zeros_like(b_full)
    identical = True
    for r in range(k):
        gs = oracle.Geom(g.nx, g.ny, g.nz, g.h, g.origin, g.nu, g.nv, g.views[r::k])
        c = context(gs)
        c.set_projector(proj)
        identical &= bool(np.array_equal(to_host(c.project(xd)), a_full[r::k]))
        acc += to_host(c.backproject(to_dev(y[r::k])))
        c.close()
    err = rel_l2(acc, b_full)
    say("view shares", proj, "K", k, "A rows identical", identical, "sum of share A^T vs A^T %.2e" % err,
        "A^T vs oracle %.2e" % err_full)
    assert identical
    # the shares regroup the FP32 group sums of 16 views: rounding only (a
    # dropped or doubled view would be off by about 1/120)
    assert err <= 1e-6

"""Kernel timing (instrumentation of the C ABI): the selection masks decide
which launches are bracketed by events; the recorded durations are positive
and the counts match the calls."""

import numpy as np
import pytest

import paper_2103_10329_amd as mg
from gpu_common import context, workload

pytestmark = pytest.mark.gpu


def test_timing_records_only_the_selected_operations_and_grids():
    import torch
    g = workload("c0", n=32, nu=48, nv=48, n_views=16)
    ctx = context(g)
    rng = np.random.Generator(np.random.PCG64(11))
    vol = torch.from_numpy(rng.random(g.vol_shape, dtype=np.float32)).cuda()
    st = torch.empty(g.level(0).stack_shape, device="cuda")
    st1 = torch.from_numpy(rng.random(g.level(1).stack_shape, dtype=np.float32)).cuda()
    out1 = torch.empty(g.level(1).vol_shape, device="cuda")

    def run():
        ctx.project(vol, out=st)
        ctx.backproject(st, out=vol)
        ctx.backproject(st1, out=out1, level=1)
        torch.cuda.synchronize()

    ctx.kernel_timing(True, ops=(mg.MGCT_OP_BACKPROJECT,), levels=(0,))
    run()
    ctx.kernel_timing(False)
    assert ctx.kernel_time(mg.MGCT_OP_PROJECT, 0)[1] == 0
    assert ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 1)[1] == 0
    ms, n = ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)
    assert n == 1 and ms > 0.0
    # everything again (enabling clears the records)
    ctx.kernel_timing(True)
    run()
    run()
    ctx.kernel_timing(False)
    assert ctx.kernel_time(mg.MGCT_OP_PROJECT, 0)[1] == 2
    assert ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)[1] == 2
    assert ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 1)[1] == 2
    assert ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, -1)[1] == 4
    ctx.close()

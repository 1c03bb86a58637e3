"""Error behaviour of the C ABI on a GPU: every rejected call returns the
documented status (and leaves the context usable), none faults."""


import numpy as np
import pytest

import paper_2103_10329_amd as mg
import synth
from gpu_common import context, workload

pytestmark = pytest.mark.gpu


def _code(fn):
    with pytest.raises(mg.MgctError) as e:
        fn()
    return e.value.code


def _ptr(t):
    return t.data_ptr()


def test_calls_before_geometry_and_bad_arguments():
    import torch
    ctx = mg.Context(0)
    x = torch.zeros((8, 8, 8), device="cuda")
    y = torch.zeros((4, 8, 8), device="cuda")
    assert mg.mgct_project(ctx.handle, 0, _ptr(x), mg.MGCT_F32, _ptr(y), mg.MGCT_F32, None) == \
        mg.MGCT_ERR_NO_GEOMETRY
    g = workload("c0", n=32, nu=48, nv=48, n_views=16)
    ctx.set_geometry(32, 32, 32, g.h, g.origin, 48, 48, g.views)
    vol = torch.zeros((32, 32, 32), device="cuda")
    st = torch.zeros((16, 48, 48), device="cuda")
    # null pointers, bad dtypes, levels beyond the hierarchy
    assert mg.mgct_project(ctx.handle, 0, None, mg.MGCT_F32, _ptr(st), mg.MGCT_F32, None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_project(ctx.handle, 0, _ptr(vol), 7, _ptr(st), mg.MGCT_F32, None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_project(ctx.handle, 9, _ptr(vol), mg.MGCT_F32, _ptr(st), mg.MGCT_F32, None) != mg.MGCT_OK
    assert mg.mgct_landweber_step(ctx.handle, 0, _ptr(vol), _ptr(st), mg.MGCT_F32, float("nan"), None, None,
                                  None) == mg.MGCT_ERR_INVALID_ARG
    # timing controls: a null context is rejected
    assert mg.mgct_kernel_timing_select(None, 1, 1) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_kernel_timing(None, 1) == mg.MGCT_ERR_INVALID_ARG
    # the context still works
    ctx.project(vol, out=st)
    torch.cuda.synchronize()
    assert float(st.abs().sum()) == 0.0


def test_geometry_rejections():
    ctx = mg.Context(0)
    g = workload("c0")
    # source inside the volume box
    v = g.views.copy()
    v[:, 0:3] = 0.0
    assert _code(lambda: ctx.set_geometry(32, 32, 32, g.h, g.origin, 48, 48, v)) == mg.MGCT_ERR_UNSUPPORTED_GEOMETRY
    # a z-major ray: source far above the volume looking down
    v = g.views.copy()
    v[:, 0:3] = [0.0, 0.0, 100.0]
    v[:, 3:6] = [0.0, 0.0, -100.0]
    v[:, 6:9] = [1.5, 0.0, 0.0]
    v[:, 9:12] = [0.0, 1.5, 0.0]
    assert _code(lambda: ctx.set_geometry(32, 32, 32, g.h, g.origin, 48, 48, v)) == mg.MGCT_ERR_UNSUPPORTED_GEOMETRY
    # a valid geometry afterwards is accepted
    ctx.set_geometry(32, 32, 32, g.h, g.origin, 48, 48, g.views)


def test_size_and_filter_rejections():
    import torch
    g = workload("c0", n=32, nu=48, nv=48, n_views=16)
    ctx = context(g)
    vol = torch.zeros((32, 32, 32), device="cuda")
    b = torch.zeros((16, 48, 48), device="cuda")
    t, r = mg.ramp_table(32)
    # 6 grids need every edge divisible by 2^5: the 48-pixel detector is not
    assert _code(lambda: ctx.multigrid_solve(vol, b, 6, 1, mg.filter_radial(t, r), want_hist=False)) in (
        mg.MGCT_ERR_SIZE_NOT_DIVISIBLE, mg.MGCT_ERR_INVALID_ARG)
    # a TRANSFER filter without an array for the grid it is used on
    f = mg.filter_transfer([None])
    assert _code(lambda: ctx.precondition(vol, f)) == mg.MGCT_ERR_INVALID_ARG
    # H must not alias T
    T = ctx.psf_spectrum()
    assert _code(lambda: ctx.transfer_from_spectrum(T, 0.03, out=T)) == mg.MGCT_ERR_INVALID_ARG
    # the learned network needs weights and nx a multiple of 32
    u = torch.zeros((8, 8, 40), device="cuda")
    assert _code(lambda: ctx.cnn_forward(u)) == mg.MGCT_ERR_INVALID_ARG
    ctx.cnn_set_weights(np.zeros(mg.Context.CNN_PARAMS, np.float32))
    assert _code(lambda: ctx.cnn_forward(u)) == mg.MGCT_ERR_INVALID_ARG


def test_fourier_paths_need_power_of_two_edges():
    import torch
    views = synth.trajectory(16, 4, 72.0 / 48)
    ctx = mg.Context(0)
    ctx.set_geometry(48, 32, 32, 1.0, (0, 0, 0), 48, 48, views)
    x = torch.zeros((32, 32, 48), device="cuda")
    t, r = mg.ramp_table(32)
    assert _code(lambda: ctx.precondition(x, mg.filter_radial(t, r))) == mg.MGCT_ERR_NOT_IMPLEMENTED
    assert _code(lambda: ctx.psf_spectrum()) == mg.MGCT_ERR_NOT_IMPLEMENTED
    # the stencil filter (eq. 5) works on any size
    y = ctx.precondition(torch.ones_like(x), mg.filter_eq5())
    torch.cuda.synchronize()
    assert float(y.abs().max()) < 1e-5      # eq. 5's taps sum to zero

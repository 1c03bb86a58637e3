"""torch.autograd wrapper of the projector (argument marshalling only).

``project(vol, views, ctx)`` returns A(views) vol.  Its backward applies the
hand-written adjoints of libmgct: A^T (mgct_backproject) for the volume and
the geometry-derivative kernel (mgct_project_geom_grad) for the per-view
table (s, d, u, v).  Only the volume is kept for backward; nothing of the
projection stack is stored (the derivative kernel walks the rays again).
"""

from __future__ import annotations

import numpy as np
import torch

from . import Context


class _ProjectFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vol, views, mctx: Context, level: int):
        _sync_geometry(mctx, views)
        fctx.mctx = mctx
        fctx.level = level
        fctx.save_for_backward(vol)
        return mctx.project(vol.contiguous(), level=level)

    @staticmethod
    def backward(fctx, grad_out):
        (vol,) = fctx.saved_tensors
        mctx, level = fctx.mctx, fctx.level
        g = grad_out.contiguous().float()
        g_vol = g_views = None
        if fctx.needs_input_grad[0]:
            g_vol = mctx.backproject(g, level=level)
        if fctx.needs_input_grad[1]:
            dv = mctx.project_geom_grad(vol.contiguous().float(), g, level=level)
            g_views = torch.from_numpy(dv)
        return g_vol, g_views, None, None


def _sync_geometry(mctx: Context, views) -> None:
    v = views.detach().cpu().double().numpy() if isinstance(views, torch.Tensor) else np.asarray(views)
    cur = getattr(mctx, "_views_np", None)
    if cur is None or cur.shape != v.shape or not np.array_equal(cur, v):
        g = mctx.geom
        mctx.set_geometry(g["nx"], g["ny"], g["nz"], g["voxel"], g.get("origin", (0.0, 0.0, 0.0)),
                          g["nu"], g["nv"], v)
        mctx._views_np = v.copy()


def project(vol: torch.Tensor, views: torch.Tensor, mctx: Context, level: int = 0) -> torch.Tensor:
    """A(views) vol with gradients for vol (device) and views (CPU float64, (V, 12))."""
    return _ProjectFn.apply(vol, views, mctx, level)

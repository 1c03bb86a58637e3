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
        # the geometry this node projected with: backward restores it, so that
        # other projections between forward and backward cannot change it
        fctx.geom = dict(mctx.geom)
        fctx.views_np = mctx._views_np.copy()
        fctx.save_for_backward(vol)
        return mctx.project(vol.contiguous(), level=level)

    @staticmethod
    def backward(fctx, grad_out):
        (vol,) = fctx.saved_tensors
        mctx, level = fctx.mctx, fctx.level
        _sync_geometry(mctx, fctx.views_np, fctx.geom)
        g = grad_out.contiguous().float()
        g_vol = g_views = None
        if fctx.needs_input_grad[0]:
            g_vol = mctx.backproject(g, level=level)
        if fctx.needs_input_grad[1]:
            dv = mctx.project_geom_grad(vol.contiguous().float(), g, level=level)
            g_views = torch.from_numpy(dv)
        return g_vol, g_views, None, None


def _sync_geometry(mctx: Context, views, geom=None) -> None:
    """Make the context hold ``views`` (and the grid ``geom``, default: the
    context's current grid)."""
    v = views.detach().cpu().double().numpy() if isinstance(views, torch.Tensor) else np.asarray(views, dtype=np.float64)
    g = dict(mctx.geom) if geom is None else geom
    cur = getattr(mctx, "_views_np", None)
    same_grid = all(mctx.geom.get(k) == g.get(k) for k in ("nx", "ny", "nz", "voxel", "nu", "nv")) and \
        tuple(mctx.geom.get("origin", (0.0, 0.0, 0.0))) == tuple(g.get("origin", (0.0, 0.0, 0.0)))
    if cur is None or not same_grid or cur.shape != v.shape or not np.array_equal(cur, v):
        mctx.set_geometry(g["nx"], g["ny"], g["nz"], g["voxel"], g.get("origin", (0.0, 0.0, 0.0)),
                          g["nu"], g["nv"], v)
        mctx._views_np = v.copy()


def project(vol: torch.Tensor, views: torch.Tensor, mctx: Context, level: int = 0) -> torch.Tensor:
    """A(views) vol with gradients for vol (device) and views (CPU float64, (V, 12))."""
    return _ProjectFn.apply(vol, views, mctx, level)

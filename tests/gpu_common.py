"""Helpers shared by the GPU parity tests: build a library context and the
matching oracle geometry from one description, move arrays, compare."""

from __future__ import annotations

import sys

import numpy as np

import oracle
import synth


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def workload(name: str, n=None, nu=None, nv=None, n_views=None):
    """Geometry (oracle.Geom) of a named workload, optionally resized while
    keeping the physical field of view (voxel 32/n, pixel 72/nu)."""
    cfg = synth.CONFIGS[name]
    n = n or cfg.n
    nu = nu or cfg.nu
    nv = nv or cfg.nv
    n_views = n_views or cfg.n_views
    views = synth.trajectory(n_views, cfg.z_levels, 72.0 / nu)
    if nv != nu:
        views[:, 9:12] = np.array([0.0, 0.0, 72.0 / nu])
    return oracle.Geom(n, n, n, 32.0 / n, (0, 0, 0), nu, nv, views)


def context(geom: oracle.Geom):
    import paper_2103_10329_amd as mg
    ctx = mg.Context(0)
    ctx.set_geometry(geom.nx, geom.ny, geom.nz, geom.h, geom.origin, geom.nu, geom.nv, geom.views)
    return ctx


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32)))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)

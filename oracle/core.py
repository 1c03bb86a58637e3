"""Oracle geometry and projector bindings (FP64, test infrastructure only).

The projector / back-projector themselves are plain C (``joseph.c``), built
with gcc; this module only marshals numpy arrays into it.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

__all__ = [
    "Geom", "build", "project", "backproject", "project_rays", "backproject_voxels",
    "weight", "dense_matrix", "major_axis", "num_threads", "set_num_threads", "project_geom_grad",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "joseph.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP; no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int)
        ci, cd, cl = ctypes.c_int, ctypes.c_double, ctypes.c_long
        geo = [ci, ci, ci, cd, D, ci, ci]
        lib.oracle_project.argtypes = geo + [ci, D, D, D]
        lib.oracle_project.restype = None
        lib.oracle_backproject.argtypes = geo + [ci, D, D, D]
        lib.oracle_backproject.restype = None
        lib.oracle_project_rays.argtypes = geo + [D, D, cl, I, D]
        lib.oracle_project_rays.restype = None
        lib.oracle_backproject_voxels.argtypes = geo + [ci, D, D, cl, I, D]
        lib.oracle_backproject_voxels.restype = None
        lib.oracle_weight.argtypes = geo + [D, ci, ci, ci, ci, ci]
        lib.oracle_weight.restype = cd
        lib.oracle_dense_matrix.argtypes = geo + [ci, D, D]
        lib.oracle_dense_matrix.restype = None
        lib.oracle_project_geom_grad.argtypes = geo + [ci, D, D, D, D]
        lib.oracle_project_geom_grad.restype = None
        lib.oracle_major_axis.argtypes = [D]
        lib.oracle_major_axis.restype = ci
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ci
        lib.oracle_set_num_threads.argtypes = [ci]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


@dataclasses.dataclass
class Geom:
    """Volume grid plus per-view source/detector table (paper Sec. 2, eq. 1).

    Volume [nz][ny][nx], voxel size h, box centre ``origin``.  ``views`` is a
    (V, 12) float64 table of s, d, u, v per view; stacks are [V][nv][nu].
    """

    nx: int
    ny: int
    nz: int
    h: float
    origin: np.ndarray
    nu: int
    nv: int
    views: np.ndarray

    def __post_init__(self):
        self.origin = np.ascontiguousarray(np.asarray(self.origin, dtype=np.float64).reshape(3))
        self.views = np.ascontiguousarray(np.asarray(self.views, dtype=np.float64).reshape(-1, 12))

    @property
    def n_views(self) -> int:
        return self.views.shape[0]

    @property
    def vol_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def stack_shape(self):
        return (self.n_views, self.nv, self.nu)

    def subset(self, idx) -> "Geom":
        return Geom(self.nx, self.ny, self.nz, self.h, self.origin, self.nu, self.nv, self.views[idx])

    def level(self, g: int) -> "Geom":
        """Grid g of the multigrid hierarchy (Algorithm 1): every size halved
        g times, voxel size and pixel steps doubled g times, and the same
        source and detector-centre positions (the trajectory is shared by all
        grids)."""
        f = 2 ** g
        for n in (self.nx, self.ny, self.nz, self.nu, self.nv):
            if n % f:
                raise ValueError("size %d not divisible by %d" % (n, f))
        v = self.views.copy()
        v[:, 6:12] *= f
        return Geom(self.nx // f, self.ny // f, self.nz // f, self.h * f, self.origin,
                    self.nu // f, self.nv // f, v)

    def _args(self):
        return (self.nx, self.ny, self.nz, self.h, _dp(self.origin), self.nu, self.nv)


def project(geom: Geom, vol: np.ndarray) -> np.ndarray:
    """A mu for every ray (paper eq. 1's P, Joseph discretisation)."""
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    assert vol.shape == geom.vol_shape, (vol.shape, geom.vol_shape)
    out = np.zeros(geom.stack_shape)
    _load().oracle_project(*geom._args(), geom.n_views, _dp(geom.views), _dp(vol), _dp(out))
    return out


def backproject(geom: Geom, proj: np.ndarray) -> np.ndarray:
    """B y = A^T y (paper Sec. 2.1: B is the adjoint of P), ray-driven scatter."""
    proj = np.ascontiguousarray(proj, dtype=np.float64)
    assert proj.shape == geom.stack_shape, (proj.shape, geom.stack_shape)
    out = np.zeros(geom.vol_shape)
    _load().oracle_backproject(*geom._args(), geom.n_views, _dp(geom.views), _dp(proj), _dp(out))
    return out


def project_rays(geom: Geom, vol: np.ndarray, rays: np.ndarray) -> np.ndarray:
    """A mu for selected rays; ``rays`` is (n, 3) int (view, column a, row b)."""
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    rays = np.ascontiguousarray(rays, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(rays.shape[0])
    _load().oracle_project_rays(*geom._args(), _dp(geom.views), _dp(vol), rays.shape[0], _ip(rays), _dp(out))
    return out


def backproject_voxels(geom: Geom, proj: np.ndarray, voxels: np.ndarray) -> np.ndarray:
    """(A^T y) at selected voxels; ``voxels`` is (n, 3) int (i, j, k) = (x, y, z)."""
    proj = np.ascontiguousarray(proj, dtype=np.float64)
    vox = np.ascontiguousarray(voxels, dtype=np.int32).reshape(-1, 3)
    out = np.zeros(vox.shape[0])
    _load().oracle_backproject_voxels(*geom._args(), geom.n_views, _dp(geom.views), _dp(proj),
                                      vox.shape[0], _ip(vox), _dp(out))
    return out


def weight(geom: Geom, view: int, a: int, b: int, i: int, j: int, k: int) -> float:
    """System-matrix entry for voxel (i,j,k) and ray (view, a, b), from the
    hat-function definition with no index arithmetic."""
    v = np.ascontiguousarray(geom.views[view])
    return _load().oracle_weight(*geom._args(), _dp(v), a, b, i, j, k)


def dense_matrix(geom: Geom) -> np.ndarray:
    """Dense system matrix [ray][voxel] built entry by entry from ``weight``."""
    W = np.zeros((geom.n_views * geom.nv * geom.nu, geom.nx * geom.ny * geom.nz))
    _load().oracle_dense_matrix(*geom._args(), geom.n_views, _dp(geom.views), _dp(W))
    return W


def project_geom_grad(geom: Geom, vol: np.ndarray, g: np.ndarray) -> np.ndarray:
    """d/d(views) of sum(g * A(views) vol): (V, 12) in the order s, d, u, v
    (analytic derivative of the Joseph sums, major axes and plane sets held
    fixed)."""
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros((geom.n_views, 12))
    _load().oracle_project_geom_grad(*geom._args(), geom.n_views, _dp(geom.views), _dp(vol), _dp(g), _dp(out))
    return out


def major_axis(D) -> int:
    D = np.ascontiguousarray(np.asarray(D, dtype=np.float64).reshape(3))
    return _load().oracle_major_axis(_dp(D))


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    """Threads for the following oracle calls (timing only; A^T's partial
    volumes are summed in a different grouping, a rounding-level change)."""
    _load().oracle_set_num_threads(int(n))

"""Random ellipsoid/cube phantoms, their exact line integrals and noisy data.

All randomness comes from numpy's PCG64 with an explicit seed.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

from .geometry import CONFIGS, FOV, ScanConfig, trajectory

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "_synth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C generator with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_line_integrals.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, dp, ctypes.c_int, dp, dp]
        lib.synth_line_integrals.restype = None
        lib.synth_line_integrals_clipped.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_int,
                                                     ctypes.c_int, dp, ctypes.c_int, dp, dp, dp]
        lib.synth_line_integrals_clipped.restype = None
        lib.synth_voxelize.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                       ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp]
        lib.synth_voxelize.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclasses.dataclass
class Phantom:
    ellipsoids: np.ndarray  # (K, 16): centre, rotation (row-major), semi-axes, kappa
    boxes: np.ndarray       # (J, 7): lo, hi, kappa


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Rotation matrix from a uniformly distributed unit quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_phantom(cfg: ScanConfig, seed: int, fov: float = FOV, extent=None) -> Phantom:
    """Ellipsoids with centres in the inner 70% of the box, random rotations,
    semi-axes in ``cfg.semi_axis_range`` and attenuation in ``cfg.kappa``;
    plus axis-aligned cubes (side U[0.25, 1]) until ``cfg.cube_fraction`` of
    the box is covered in expectation.  The box is fov^3 centred at the
    origin, or extent = (ex, ey, ez) for a box of another shape (the
    semi-axis range is then taken as is)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ext = np.array((fov, fov, fov) if extent is None else extent, dtype=np.float64)
    K = cfg.n_ellipsoids
    ell = np.zeros((K, 16))
    lo, hi = cfg.semi_axis_range if extent is None else (2.0 * (10.0 / 60) ** (1 / 3), 8.0 * (10.0 / 60) ** (1 / 3))
    for k in range(K):
        ell[k, 0:3] = rng.uniform(-0.35 * ext, 0.35 * ext)
        ell[k, 3:12] = _random_rotation(rng).reshape(-1)
        ell[k, 12:15] = rng.uniform(lo, hi, size=3)
        ell[k, 15] = rng.uniform(*cfg.kappa)
    boxes = np.zeros((0, 7))
    if cfg.cube_fraction > 0:
        mean_vol = (1.0 ** 4 - 0.25 ** 4) / (4 * 0.75)  # E[s^3], s ~ U[0.25, 1]
        J = int(round(cfg.cube_fraction * float(np.prod(ext)) / mean_vol))
        boxes = np.zeros((J, 7))
        side = rng.uniform(0.25, 1.0, size=J)
        cen = rng.uniform(-0.5 * ext, 0.5 * ext, size=(J, 3))
        boxes[:, 0:3] = cen - side[:, None] / 2
        boxes[:, 3:6] = cen + side[:, None] / 2
        boxes[:, 6] = rng.uniform(*cfg.kappa, size=J)
    return Phantom(np.ascontiguousarray(ell), np.ascontiguousarray(boxes))


def voxelize(ph: Phantom, n, h: float, origin=(0.0, 0.0, 0.0), ss: int = 4) -> np.ndarray:
    """Ground truth: the ss^3-supersampled voxel mean of the phantom, [z][y][x]."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    vol = np.zeros((nz, ny, nx))
    org = np.ascontiguousarray(np.asarray(origin, dtype=np.float64))
    e = np.ascontiguousarray(ph.ellipsoids, dtype=np.float64).reshape(-1, 16)
    b = np.ascontiguousarray(ph.boxes, dtype=np.float64).reshape(-1, 7)
    if e.shape[0] == 0:
        e = np.zeros((1, 16))
        ne = 0
    else:
        ne = e.shape[0]
    if b.shape[0] == 0:
        b = np.zeros((1, 7))
        nb = 0
    else:
        nb = b.shape[0]
    _load().synth_voxelize(nx, ny, nz, h, _ptr(org), ne, _ptr(e), nb, _ptr(b), ss, _ptr(vol))
    return vol


def line_integrals(ph: Phantom, views: np.ndarray, nu: int, nv: int) -> np.ndarray:
    """Exact line integrals of the phantom for every ray, shape (V, nv, nu)."""
    views = np.ascontiguousarray(views, dtype=np.float64)
    V = views.shape[0]
    out = np.zeros((V, nv, nu))
    e = np.ascontiguousarray(ph.ellipsoids, dtype=np.float64).reshape(-1, 16)
    b = np.ascontiguousarray(ph.boxes, dtype=np.float64).reshape(-1, 7)
    ne, nb = e.shape[0], b.shape[0]
    if ne == 0:
        e = np.zeros((1, 16))
    if nb == 0:
        b = np.zeros((1, 7))
    _load().synth_line_integrals(V, _ptr(views), nu, nv, ne, _ptr(e), nb, _ptr(b), _ptr(out))
    return out


def crop(ph: Phantom, lo, hi) -> Phantom:
    """Shapes whose bounding box meets the box [lo, hi] (the others cannot
    contribute to anything inside it)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    e = ph.ellipsoids
    r = e[:, 12:15].max(axis=1, keepdims=True)
    keep_e = np.all((e[:, 0:3] + r >= lo) & (e[:, 0:3] - r <= hi), axis=1)
    b = ph.boxes
    keep_b = np.all((b[:, 3:6] >= lo) & (b[:, 0:3] <= hi), axis=1) if b.shape[0] else np.zeros(0, bool)
    return Phantom(np.ascontiguousarray(e[keep_e]), np.ascontiguousarray(b[keep_b]))


def line_integrals_clipped(ph: Phantom, views: np.ndarray, nu: int, nv: int, lo, hi) -> np.ndarray:
    """Exact line integrals of the phantom intersected with the box [lo, hi]."""
    ph = crop(ph, lo, hi)
    views = np.ascontiguousarray(views, dtype=np.float64)
    V = views.shape[0]
    out = np.zeros((V, nv, nu))
    e = np.ascontiguousarray(ph.ellipsoids, dtype=np.float64).reshape(-1, 16)
    b = np.ascontiguousarray(ph.boxes, dtype=np.float64).reshape(-1, 7)
    ne, nb = e.shape[0], b.shape[0]
    if ne == 0:
        e = np.zeros((1, 16))
    if nb == 0:
        b = np.zeros((1, 7))
    clip = np.ascontiguousarray(np.concatenate([np.asarray(lo, float), np.asarray(hi, float)]))
    _load().synth_line_integrals_clipped(V, _ptr(views), nu, nv, ne, _ptr(e), nb, _ptr(b), _ptr(clip), _ptr(out))
    return out


def crop_dataset(name: str = "c2", n: int = 64, nu: int = 96, levels: int = 4):
    """The central n^3 fine-voxel box of a workload's phantom, seen through a
    nu x nu detector of the workload's pixel size with all of its views.
    Returns dict(views, h, n, nu, mu, b, b_true)."""
    cfg = CONFIGS[name]
    idx = int(name[1:])
    views = trajectory(cfg.n_views, cfg.z_levels, cfg.pixel)
    ph = random_phantom(cfg, 1000 + idx)
    half = 0.5 * n * cfg.h
    lo, hi = (-half,) * 3, (half,) * 3
    b_true = line_integrals_clipped(ph, views, nu, nu, lo, hi)
    b = add_noise(b_true, cfg, 3000 + idx)
    mu = voxelize(crop(ph, lo, hi), n, cfg.h, ss=4)
    return dict(views=views, h=cfg.h, n=n, nu=nu, mu=mu, b=b, b_true=b_true, levels=levels)


def add_noise(b_true: np.ndarray, cfg: ScanConfig, seed: int) -> np.ndarray:
    """Measured data b = ln(I0/I).  Gaussian: b + N(0, sigma^2).  Poisson:
    counts ~ Poisson(I0 exp(-b)), zero counts clamped to 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if cfg.noise == "gauss":
        return b_true + rng.normal(0.0, cfg.noise_level, size=b_true.shape)
    I0 = cfg.noise_level
    counts = rng.poisson(I0 * np.exp(-b_true)).astype(np.float64)
    return np.log(I0 / np.maximum(counts, 1.0))


def make_dataset(name: str, index: int | None = None, views: np.ndarray | None = None, ss: int = 4,
                 truth: bool = True):
    """Geometry, ground-truth volume and noisy data for a named workload.

    Seeds: phantom 1000 + index, noise 2000 + index (index defaults to the
    workload's number).  Returns a dict with keys cfg, views, h, mu, b, b_true.
    """
    cfg = CONFIGS[name]
    idx = int(name[1:]) if index is None else index
    if views is None:
        views = trajectory(cfg.n_views, cfg.z_levels, cfg.pixel)
    ph = random_phantom(cfg, 1000 + idx)
    b_true = line_integrals(ph, views, cfg.nu, cfg.nv)
    b = add_noise(b_true, cfg, 2000 + idx)
    mu = voxelize(ph, cfg.n, cfg.h, ss=ss) if truth else None
    return dict(cfg=cfg, views=views, h=cfg.h, mu=mu, b=b, b_true=b_true, phantom=ph)

"""Scan geometries for the synthetic workloads.

A scan is described by a per-view table of 12 float64 values:
``s`` (source position), ``d`` (detector centre), ``u`` (step between
adjacent detector columns) and ``v`` (step between adjacent detector rows).
Pixel (a, b) of a view is centred at ``d + (a-(nu-1)/2) u + (b-(nv-1)/2) v``.

The trajectory is a "space-filling"-style one (paper, Sec. 1 and Sec. 2): the
source angle advances by the golden ratio turn, and the source height steps
through a small lattice, so that views are spread near-isotropically over the
sphere of directions.  The source sits at radius 100 from the rotation axis and
the detector centre sits diametrically opposite at radius 100 (source to
detector 200), moving up and down with the source.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

GOLDEN_TURN = 0.618034
SOURCE_RADIUS = 100.0
SOURCE_DETECTOR = 200.0
FOV = 32.0  # physical edge length of the reconstruction box (all workloads)


@dataclasses.dataclass(frozen=True)
class ScanConfig:
    """One synthetic workload: sizes, physics and phantom recipe."""

    name: str
    n: int                 # volume edge in voxels (cube)
    nu: int                # detector columns
    nv: int                # detector rows
    n_views: int
    z_levels: int          # height-lattice levels of the trajectory
    n_ellipsoids: int
    kappa: tuple           # attenuation range of each ellipsoid
    noise: str             # "gauss" or "poisson"
    noise_level: float     # sigma for "gauss", I0 for "poisson"
    cube_fraction: float = 0.0
    levels: int = 1        # multigrid levels used with this workload

    @property
    def h(self) -> float:
        return FOV / self.n

    @property
    def pixel(self) -> float:
        # 72 physical units of detector for 1.5 * n pixels: the pixel at the
        # rotation axis (magnification 2) is 0.75 voxel in every workload.
        return 72.0 / self.nu

    @property
    def semi_axis_range(self) -> tuple:
        # 2..8 units for 10 ellipsoids; for K ellipsoids shrink by (10/K)^(1/3)
        # so that the filled fraction of the box stays about the same.
        k = (10.0 / self.n_ellipsoids) ** (1.0 / 3.0)
        return (2.0 * k, 8.0 * k)


CONFIGS = {
    # 32^3, 64 views of 48^2, 10 ellipsoids, SIRT.
    "c0": ScanConfig("c0", 32, 48, 48, 64, 4, 10, (0.05, 0.5), "gauss", 1e-3),
    # 128^3, 360 views of 192^2, 60 ellipsoids, Poisson I0=1e4, 3 levels.
    "c1": ScanConfig("c1", 128, 192, 192, 360, 8, 60, (0.01, 0.3), "poisson", 1e4, levels=3),
    # 512^3, 1440 views of 768^2, 400 ellipsoids + 5% cubes, I0=5e3, 4 levels.
    "c2": ScanConfig("c2", 512, 768, 768, 1440, 8, 400, (0.01, 0.3), "poisson", 5e3,
                     cube_fraction=0.05, levels=4),
    # 256^3, 720 views of 384^2, 60 ellipsoids (geometry estimation).
    "c3": ScanConfig("c3", 256, 384, 384, 720, 8, 60, (0.01, 0.3), "poisson", 1e4, levels=3),
    # learned-preconditioner training distribution (as c1).
    "c4": ScanConfig("c4", 128, 192, 192, 360, 8, 60, (0.01, 0.3), "poisson", 1e4, levels=3),
}


# Paper-shaped workload (the scan of Sec. 2: 3600 radiographs binned to 760^2
# and a 640 x 640 x 2304 volume of a tall sample): the same physical width as
# the workloads above (32 units, h = 0.05), height 115.2 units, 216 ellipsoids
# (60 per 32^3 units), Poisson I0 = 1e4, a golden-angle helix over source
# heights [-48, 48] (the detector covers 36 units of height at the axis, so the
# sample's ends are seen by fewer views than its middle).
PAPER_SHAPED = ScanConfig("paper", 640, 760, 760, 3600, 1, 216, (0.01, 0.3), "poisson", 1e4, levels=4)
PAPER_SHAPED_NZ = 2304
PAPER_SHAPED_Z_RANGE = (-48.0, 48.0)


def helix_trajectory(n_views: int, pixel: float, z_range=PAPER_SHAPED_Z_RANGE) -> np.ndarray:
    """Golden-angle azimuths with the source height rising linearly with the
    view index over z_range (a helix), shape (n_views, 12) float64."""
    views = trajectory(n_views, 2, pixel)
    z = np.linspace(z_range[0], z_range[1], n_views)
    views[:, 2] = z
    views[:, 5] = z
    return views


def trajectory(n_views: int, z_levels: int, pixel: float, z_range=(-8.0, 8.0)) -> np.ndarray:
    """Golden-angle + height-lattice trajectory, shape (n_views, 12) float64."""
    i = np.arange(n_views, dtype=np.float64)
    theta = np.mod(2.0 * math.pi * i * GOLDEN_TURN, 2.0 * math.pi)
    lo, hi = z_range
    z = lo + (hi - lo) * (np.arange(n_views) % z_levels) / (z_levels - 1)
    c, s = np.cos(theta), np.sin(theta)
    far = SOURCE_DETECTOR - SOURCE_RADIUS
    views = np.zeros((n_views, 12), dtype=np.float64)
    views[:, 0] = SOURCE_RADIUS * c
    views[:, 1] = SOURCE_RADIUS * s
    views[:, 2] = z
    views[:, 3] = -far * c
    views[:, 4] = -far * s
    views[:, 5] = z
    views[:, 6] = -pixel * s
    views[:, 7] = pixel * c
    views[:, 8] = 0.0
    views[:, 9] = 0.0
    views[:, 10] = 0.0
    views[:, 11] = pixel
    return views


def perturb_geometry(views: np.ndarray, h: float, dx: float, dz: float, tilt_deg: float) -> np.ndarray:
    """Apply a source offset and a detector in-plane tilt to every view.

    ``dx`` moves the source along the view's unit column direction and ``dz``
    along the rotation axis, both in voxels of size ``h``; ``tilt_deg`` rotates
    the column/row step vectors about the detector normal (lengths kept).
    """
    out = views.copy()
    u = views[:, 6:9]
    v = views[:, 9:12]
    lu = np.linalg.norm(u, axis=1, keepdims=True)
    lv = np.linalg.norm(v, axis=1, keepdims=True)
    uh = u / lu
    vh = v / lv
    out[:, 0:3] = views[:, 0:3] + dx * h * uh + dz * h * np.array([0.0, 0.0, 1.0])
    t = math.radians(tilt_deg)
    ct, st = math.cos(t), math.sin(t)
    out[:, 6:9] = lu * (ct * uh + st * vh)
    out[:, 9:12] = lv * (-st * uh + ct * vh)
    return out


def volume_axes(n: int, h: float, origin=(0.0, 0.0, 0.0)):
    """Voxel-centre coordinates along x, y, z for an n^3 box centred at origin."""
    c = (n - 1) / 2.0
    idx = np.arange(n, dtype=np.float64)
    return tuple(origin[k] + (idx - c) * h for k in range(3))


def evaluation_mask(n: int, h: float, radius: float = 0.9 * FOV / 2, half_height: float = 12.0) -> np.ndarray:
    """Boolean [z][y][x] mask of the region every view sees well: a cylinder
    about the rotation axis (radius 0.9 of the half field of view, |z| below
    12 units), used to score reconstructions against the phantom."""
    x, y, z = volume_axes(n, h)
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    return (np.abs(z)[:, None, None] <= half_height) & (r2 <= radius * radius)[None, :, :]


def masked_rel_error(vol, truth, mask) -> float:
    """||mask (vol - truth)|| / ||mask truth|| in FP64."""
    d = (np.asarray(vol, np.float64) - np.asarray(truth, np.float64))[mask]
    t = np.asarray(truth, np.float64)[mask]
    return float(np.linalg.norm(d) / max(np.linalg.norm(t), 1e-300))

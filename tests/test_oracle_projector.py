"""Pins of the FP64 oracle projector / back-projector (CPU only).

Each test ties the oracle to something outside itself: hand-computed
geometry, closed-form chord lengths, brute force from the definition,
invariants (symmetry, adjointness).
"""

import math

import numpy as np
import pytest

import oracle
import synth
from conftest import random_views


def _ray_geom(s, q, n=4, h=1.0):
    """One view with a 1x1 detector whose single pixel centre is q."""
    views = np.zeros((1, 12))
    views[0, 0:3] = s
    views[0, 3:6] = q
    views[0, 6:9] = (0.0, 1.0, 0.0)
    views[0, 9:12] = (0.0, 0.0, 1.0)
    return oracle.Geom(n, n, n, h, (0, 0, 0), 1, 1, views)


def test_pixel_centre_and_weight_by_hand():
    # 2x2 detector: pixel (0,0) is centred at d - u/2 - v/2 = (10, -0.5, -0.5).
    views = np.array([[-10, 0, 0, 10, 0, 0, 0, 1, 0, 0, 0, 1]], dtype=float)
    g = oracle.Geom(4, 4, 4, 1.0, (0, 0, 0), 2, 2, views)
    # Ray s=(-10,0,0) -> (10,-0.5,-0.5); D=(20,-0.5,-0.5), x-major.
    # Voxel-centre plane x=-0.5 (i=1): t=9.5/20, y=z=-0.2375; voxel (1,1,1)
    # is centred at (-0.5,-0.5,-0.5): in-plane offsets 0.2625 -> hat 0.7375.
    L = math.sqrt(400.5) / 20.0
    expect = L * 0.7375 * 0.7375
    assert oracle.weight(g, 0, 0, 0, 1, 1, 1) == pytest.approx(expect, rel=1e-14)
    vol = np.zeros(g.vol_shape)
    vol[1, 1, 1] = 1.0
    p = oracle.project(g, vol)
    assert p[0, 0, 0] == pytest.approx(expect, rel=1e-14)
    # pixel (1,1) at (10, 0.5, 0.5) passes on the other side: y=z=+0.2375,
    # offset 0.7375 from voxel (1,1,1) -> hat 0.2625.
    assert p[0, 1, 1] == pytest.approx(L * 0.2625 * 0.2625, rel=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("offset", [(0.0, 0.0), (0.3, -0.7), (1.25, 0.5)])
def test_axis_aligned_ray_through_ones(axis, offset):
    n, h = 8, 0.5
    s = np.zeros(3)
    q = np.zeros(3)
    others = [k for k in range(3) if k != axis]
    s[axis], q[axis] = -30.0, 30.0
    for k, o in zip(others, offset):
        s[k] = q[k] = o
    g = _ray_geom(s, q, n=n, h=h)
    p = oracle.project(g, np.ones(g.vol_shape))
    assert p[0, 0, 0] == pytest.approx(n * h, rel=1e-14)


def _random_small(rng, n=8, n_views=6, nu=5, nv=4, allow_z=True):
    views = random_views(rng, n_views, radius=15.0, det_dist=12.0, pixel=1.3, allow_z=allow_z)
    return oracle.Geom(n, n - 1, n + 1, 0.9, (0.2, -0.1, 0.3), nu, nv, views)


def test_dense_matrix_matches_indexed_projector(rng):
    g = _random_small(rng)
    W = oracle.dense_matrix(g)
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    Ax = oracle.project(g, x).reshape(-1)
    Aty = oracle.backproject(g, y).reshape(-1)
    assert np.abs(W @ x.reshape(-1) - Ax).max() <= 1e-13 * np.abs(Ax).max()
    assert np.abs(W.T @ y.reshape(-1) - Aty).max() <= 1e-13 * np.abs(Aty).max()
    # every major axis occurs in this random geometry
    axes = set()
    for v in range(g.n_views):
        for a in range(g.nu):
            for b in range(g.nv):
                q = g.views[v, 3:6] + (a - (g.nu - 1) / 2) * g.views[v, 6:9] + (b - (g.nv - 1) / 2) * g.views[v, 9:12]
                axes.add(oracle.major_axis(q - g.views[v, 0:3]))
    assert axes == {0, 1, 2}


def test_adjoint_identity(rng):
    cfg = synth.CONFIGS["c0"]
    views = synth.trajectory(cfg.n_views, cfg.z_levels, cfg.pixel)
    g = oracle.Geom(32, 32, 32, 1.0, (0, 0, 0), 48, 48, views)
    x = rng.normal(size=g.vol_shape)
    y = rng.normal(size=g.stack_shape)
    Ax = oracle.project(g, x)
    Aty = oracle.backproject(g, y)
    lhs, rhs = np.vdot(Ax, y), np.vdot(x, Aty)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_single_ray_and_single_voxel_paths_agree(rng):
    g = _random_small(rng, n=10, n_views=9, nu=7, nv=6, allow_z=True)
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    Ax = oracle.project(g, x)
    Aty = oracle.backproject(g, y)
    rays = np.stack([rng.integers(0, g.n_views, 50), rng.integers(0, g.nu, 50), rng.integers(0, g.nv, 50)], 1)
    pr = oracle.project_rays(g, x, rays)
    assert np.allclose(pr, Ax[rays[:, 0], rays[:, 2], rays[:, 1]], rtol=1e-14, atol=0)
    vox = np.stack([rng.integers(0, g.nx, 40), rng.integers(0, g.ny, 40), rng.integers(0, g.nz, 40)], 1)
    bv = oracle.backproject_voxels(g, y, vox)
    ref = Aty[vox[:, 2], vox[:, 1], vox[:, 0]]
    assert np.allclose(bv, ref, rtol=1e-12, atol=1e-12 * np.abs(Aty).max())


def test_rotation_by_90_degrees_about_z(rng):
    # Rotating geometry and volume together by +90 deg about z: (x,y) -> (-y,x).
    g = _random_small(rng, n=9, n_views=5, nu=6, nv=5, allow_z=False)
    g = oracle.Geom(9, 9, 7, 1.1, (0, 0, 0), 6, 5, g.views)
    x = rng.random(g.vol_shape)
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], dtype=float)
    v2 = g.views.copy()
    for k in range(4):
        v2[:, 3 * k:3 * k + 3] = g.views[:, 3 * k:3 * k + 3] @ R.T
    g2 = oracle.Geom(9, 9, 7, 1.1, (0, 0, 0), 6, 5, v2)
    # voxel (i,j) at (x_i, y_j) moves to (-y_j, x_i): new index (n-1-j, i)
    x2 = np.zeros_like(x)
    n = 9
    for j in range(n):
        for i in range(n):
            x2[:, i, n - 1 - j] = x[:, j, i]
    p1 = oracle.project(g, x)
    p2 = oracle.project(g2, x2)
    assert np.allclose(p1, p2, rtol=1e-12, atol=1e-12)


def _ball_phantom(radius, centre=(0.7, -0.4, 0.3), kappa=1.0):
    e = np.zeros((1, 16))
    e[0, 0:3] = centre
    e[0, 3:12] = np.eye(3).reshape(-1)
    e[0, 12:15] = radius
    e[0, 15] = kappa
    return synth.Phantom(e, np.zeros((0, 7)))


def _ellipsoid_phantom():
    e = np.zeros((1, 16))
    e[0, 0:3] = (1.1, -0.6, 0.4)
    t = 0.4
    R = np.array([[math.cos(t), -math.sin(t), 0], [math.sin(t), math.cos(t), 0], [0, 0, 1.0]])
    e[0, 3:12] = R.reshape(-1)
    e[0, 12:15] = (10.0, 6.0, 8.0)
    e[0, 15] = 1.0
    return synth.Phantom(e, np.zeros((0, 7)))


def _chord_error(ph, n, h, views, nu, nv):
    g = oracle.Geom(n, n, n, h, (0, 0, 0), nu, nv, views)
    vol = synth.voxelize(ph, n, h, ss=4)
    p = oracle.project(g, vol)
    exact = synth.line_integrals(ph, views, nu, nv)
    hit = exact > 0
    return np.linalg.norm((p - exact)[hit]) / np.linalg.norm(exact[hit])


@pytest.mark.parametrize("which", ["ball", "ellipsoid"])
def test_projection_converges_to_analytic_chords(which):
    # Radius 12 units; grid spacing h=1 (R = 12 voxels) and h=2.
    ph = _ball_phantom(12.0) if which == "ball" else _ellipsoid_phantom()
    views = synth.trajectory(12, 4, 1.5)
    e1 = _chord_error(ph, 32, 1.0, views, 48, 48)
    e2 = _chord_error(ph, 16, 2.0, synth.trajectory(12, 4, 3.0), 24, 24)
    # first-order convergence of the discretisation error (measured ~2.1x per
    # halving of h); the ellipsoid's smallest semi-axis is 6 voxels at h=1.
    assert e1 <= (0.02 if which == "ball" else 0.035)
    assert e2 / e1 >= 1.5


def test_analytic_chord_closed_form():
    # Synthetic data generator against 2 sqrt(R^2 - d^2) for a ball.
    R = 5.0
    ph = _ball_phantom(R, centre=(0.0, 0.0, 0.0))
    views = np.array([[-50, 0, 0, 50, 0, 0, 0, 0.7, 0, 0, 0, 0.9]], dtype=float)
    nu, nv = 13, 11
    out = synth.line_integrals(ph, views, nu, nv)
    for b in range(nv):
        for a in range(nu):
            q = np.array([50.0, (a - 6) * 0.7, (b - 5) * 0.9])
            s = np.array([-50.0, 0, 0])
            D = q - s
            dist = np.linalg.norm(np.cross(-s, D)) / np.linalg.norm(D)
            ref = 2 * math.sqrt(max(R * R - dist * dist, 0.0))
            assert out[0, b, a] == pytest.approx(ref, abs=1e-12)

"""Pins of the oracle's geometry gradient (CPU): central finite differences
of the Joseph sums, and of the (dx, dz, tilt) parametrisation."""

import numpy as np

import oracle
import synth
from conftest import random_views


def test_view_gradient_matches_central_differences(rng):
    views = random_views(rng, 3, radius=15.0, det_dist=12.0, pixel=1.1, allow_z=True)
    mk = lambda V: oracle.Geom(9, 8, 10, 0.9, (0.1, -0.2, 0.05), 6, 5, V)
    g = mk(views)
    x = rng.random(g.vol_shape)
    y = rng.random(g.stack_shape)
    G = oracle.project_geom_grad(g, x, y)
    f = lambda V: float((oracle.project(mk(V), x) * y).sum())
    eps = 1e-6
    fd = np.zeros_like(G)
    for v in range(3):
        for k in range(12):
            vp, vm = views.copy(), views.copy()
            vp[v, k] += eps
            vm[v, k] -= eps
            fd[v, k] = (f(vp) - f(vm)) / (2 * eps)
    assert np.linalg.norm(G - fd) <= 1e-6 * np.linalg.norm(G)


def test_parameter_gradient_matches_central_differences(rng):
    cfg = synth.CONFIGS["c0"]
    views0 = synth.trajectory(12, 4, cfg.pixel)
    h = 1.0
    x = rng.random((16, 16, 16))
    b = rng.random((12, 24, 24))
    p0 = np.array([0.3, -0.4, 0.2])

    def geom(p):
        return oracle.Geom(16, 16, 16, h, (0, 0, 0), 24, 24, synth.perturb_geometry(views0, h, *p))

    def f(p):
        r = oracle.project(geom(p), x) - b
        return 0.5 * float((r * r).sum())

    g = geom(p0)
    r = oracle.project(g, x) - b
    G = oracle.geometry_param_grad(views0, oracle.project_geom_grad(g, x, r), h, *p0)
    fd = np.zeros(3)
    # a small step keeps the difference from crossing the kinks of the
    # piecewise-bilinear interpolant (a crossing biases it by O(1) there)
    for k, eps in enumerate((1e-7, 1e-7, 1e-7)):
        pp, pm = p0.copy(), p0.copy()
        pp[k] += eps
        pm[k] -= eps
        fd[k] = (f(pp) - f(pm)) / (2 * eps)
    assert np.allclose(G, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())

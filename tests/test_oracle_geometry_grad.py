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


def test_source_height_offset_is_weakly_identifiable():
    """With the volume re-solved, how much of each geometry parameter's effect
    on the data (central differences of the oracle projector) no volume change
    can reproduce (CGLS fit by A x): a source offset along z with the detector
    fixed is, up to the depth-dependent magnification, a z-translation of the
    object, so most of its signature is absorbed; the offset along the
    detector columns and the detector tilt keep most of theirs."""
    n, V = 24, 60
    nu = 36
    h = 32.0 / n
    cfg = synth.CONFIGS["c3"]
    views0 = synth.trajectory(V, cfg.z_levels, 72.0 / nu)
    mu = synth.voxelize(synth.random_phantom(cfg, 1003), n, h, ss=2)

    def geom(p):
        return oracle.Geom(n, n, n, h, (0, 0, 0), nu, nu, synth.perturb_geometry(views0, h, *p))

    J = []
    for i in range(3):
        e = np.zeros(3)
        e[i] = 0.05
        J.append(((oracle.project(geom(e), mu) - oracle.project(geom(-e), mu)) / 0.1).ravel())
    g = geom(np.zeros(3))
    frac = []
    for i in range(3):
        b = J[i]
        r = b.copy()
        s = oracle.backproject(g, r.reshape(g.stack_shape)).ravel()
        p = s.copy()
        gam = s @ s
        for _ in range(25):
            q = oracle.project(g, p.reshape(g.vol_shape)).ravel()
            al = gam / (q @ q)
            r -= al * q
            s = oracle.backproject(g, r.reshape(g.stack_shape)).ravel()
            gn = s @ s
            p = s + (gn / gam) * p
            gam = gn
        frac.append((r @ r) / (b @ b))
    assert frac[1] <= 0.25 * min(frac[0], frac[2]), frac
    assert min(frac[0], frac[2]) >= 0.5, frac

"""Pins of the oracle's preconditioners, grid transfers, regularisers and
iterations (CPU only): closed forms, library routines, invariants and
reductions to textbook methods."""

import math

import numpy as np
import pytest
import scipy.ndimage

import oracle
from conftest import random_views


# ------------------------------------------------------------- eq. 5 stencil

def _eq5_response_closed_form(shape):
    nz, ny, nx = shape
    cz = np.cos(2 * np.pi * np.arange(nz) / nz)[:, None, None]
    cy = np.cos(2 * np.pi * np.arange(ny) / ny)[None, :, None]
    cx = np.cos(2 * np.pi * np.arange(nx) / nx)[None, None, :]
    return (64 - 8 * (cx + cy) - 32 * cx * cy - 2 * cz * (2 * cx + 2 * cy + 4 * cx * cy)) / 64.0


def test_eq5_taps_sum_to_zero_and_are_symmetric():
    t = oracle.STENCIL27_TAPS
    assert abs(t.sum()) < 1e-15               # zero response to a DC offset (paper Sec. 3)
    assert np.array_equal(t, t[::-1, ::-1, ::-1])
    assert np.array_equal(t, t.transpose(0, 2, 1))
    assert t[1, 1, 1] == 1.0 and t[1, 0, 0] == -8 / 64 and t[0, 1, 1] == 0.0


def test_eq5_response_matches_closed_form_and_fft_route(rng):
    shape = (8, 10, 12)
    delta = np.zeros(shape)
    delta[0, 0, 0] = 1.0
    resp = np.fft.fftn(oracle.stencil27(delta))
    assert np.abs(resp.imag).max() < 1e-14
    assert np.allclose(resp.real, _eq5_response_closed_form(shape), atol=1e-14)
    assert resp.real[0, 0, 0] == pytest.approx(0.0, abs=1e-15)
    assert resp.real[0, 0, 6] == pytest.approx(1.625)     # (pi, 0, 0)
    assert resp.real[4, 0, 0] == pytest.approx(0.5)       # (0, 0, pi) along z
    assert resp.real[4, 5, 6] == pytest.approx(0.75)      # (pi, pi, pi)
    assert resp.real.min() >= -1e-14
    x = rng.normal(size=shape)
    via_fft = np.real(np.fft.ifftn(np.fft.fftn(x) * _eq5_response_closed_form(shape)))
    assert np.allclose(oracle.stencil27(x), via_fft, atol=1e-12)


# ------------------------------------------------------------- radial filter

def _naive_dft3(x, inverse=False):
    out = x.astype(np.complex128)
    for ax in range(3):
        n = x.shape[ax]
        k = np.arange(n)
        sign = 1.0 if inverse else -1.0
        F = np.exp(sign * 2j * np.pi * np.outer(k, k) / n)
        if inverse:
            F /= n
        out = np.moveaxis(np.tensordot(F, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def test_radial_filter_against_naive_dft(rng):
    n = 8
    table, rho_max = oracle.radial_table(n, n_table=257)
    x = rng.normal(size=(n, n, n))
    # response by hand: rho = 2 |k/N| with signed k
    k = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n) / n
    rho = 2 * np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    H = np.interp(rho, np.linspace(0, rho_max, 257), table)
    ref = np.real(_naive_dft3(_naive_dft3(x) * H, inverse=True))
    out = oracle.radial_filter(x, table, rho_max)
    assert np.allclose(out, ref, atol=1e-12)
    # exact ramp values away from the floor: H = rho
    assert np.allclose(oracle.radial_response((n, n, n), table, rho_max)[0, 0, 3], 2 * 3 / 8, atol=1e-12)


def test_radial_filter_constant_and_delta(rng):
    n = 8
    table, rho_max = oracle.radial_table(n)
    c = 0.37
    out = oracle.radial_filter(np.full((n, n, n), c), table, rho_max)
    assert np.allclose(out, table[0] * c, atol=1e-14)      # DC gain H(0) = 2/N
    assert table[0] == pytest.approx(2.0 / n)
    delta = np.zeros((n, n, n))
    delta[0, 0, 0] = 1.0
    H = oracle.radial_response((n, n, n), table, rho_max)
    assert np.allclose(oracle.radial_filter(delta, table, rho_max), np.real(_naive_dft3(H, inverse=True)), atol=1e-13)


# ------------------------------------------------------------- grid transfer

def test_restrict_prolong_on_constants_and_linear_functions(rng):
    c = np.full((8, 6, 4), 2.5)
    assert np.allclose(oracle.restrict_volume(c), 2.5)
    assert np.allclose(oracle.prolongate(np.full((4, 3, 2), 2.5)), 2.5)
    # linear function of the cell centre is reproduced in the interior
    nz, ny, nx = 5, 6, 7
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = lambda z, y, x: 0.3 + 1.1 * x - 0.7 * y + 0.25 * z
    coarse = f(cz, cy, cx).astype(float)
    fine = oracle.prolongate(coarse)
    fz, fy, fx = np.meshgrid(np.arange(2 * nz), np.arange(2 * ny), np.arange(2 * nx), indexing="ij")
    expect = f((fz + 0.5) / 2 - 0.5, (fy + 0.5) / 2 - 0.5, (fx + 0.5) / 2 - 0.5)
    inner = (slice(1, -1),) * 3
    assert np.allclose(fine[inner], expect[inner], atol=1e-13)
    # restriction of the piecewise-constant injection is the identity
    x = rng.normal(size=(3, 4, 5))
    inj = np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)
    assert np.allclose(oracle.restrict_volume(inj), x, atol=1e-15)
    # stack restriction: 2x2 mean, by hand
    b = rng.normal(size=(2, 4, 6))
    rb = oracle.restrict_stack(b)
    assert rb[1, 1, 2] == pytest.approx((b[1, 2, 4] + b[1, 2, 5] + b[1, 3, 4] + b[1, 3, 5]) / 4)


def test_prolong_weights_by_hand():
    x = np.zeros((2, 2, 2))
    x[0, 0, 0] = 1.0
    p = oracle.prolongate(x)
    # fine (1,1,1) is at coarse coordinate 0.25 on every axis: weight (3/4)^3
    assert p[1, 1, 1] == pytest.approx(0.75 ** 3)
    assert p[0, 0, 0] == pytest.approx(1.0)        # clamped edge: 3/4 + 1/4 on voxel 0
    assert p[2, 1, 1] == pytest.approx(0.25 * 0.75 * 0.75)


# ------------------------------------------------------------- regularisers

def test_soft_threshold_closed_form(rng):
    x = np.array([-2.0, -0.5, -0.1, 0.0, 0.05, 0.3, 3.0])
    assert np.allclose(oracle.soft_threshold(x, 0.2), [-1.8, -0.3, 0.0, 0.0, 0.0, 0.1, 2.8])
    a, b = rng.normal(size=100), rng.normal(size=100)
    assert np.all(np.abs(oracle.soft_threshold(a, 0.3) - oracle.soft_threshold(b, 0.3)) <= np.abs(a - b) + 1e-15)


def test_bilateral_limits(rng):
    x = rng.random((6, 7, 5))
    # sigma_r -> infinity: normalised Gaussian blur over the in-grid 3^3 neighbourhood
    s = 0.8
    K = np.zeros((3, 3, 3))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                K[dz + 1, dy + 1, dx + 1] = math.exp(-(dx * dx + dy * dy + dz * dz) / (2 * s * s))
    blur = scipy.ndimage.correlate(x, K, mode="constant") / scipy.ndimage.correlate(np.ones_like(x), K, mode="constant")
    assert np.allclose(oracle.bilateral(x, s, 1e8), blur, atol=1e-12)
    # sigma_r -> 0: identity (distinct neighbour values get no weight)
    assert np.allclose(oracle.bilateral(x, s, 1e-6), x, atol=1e-12)
    # constant volume is a fixed point
    assert np.allclose(oracle.bilateral(np.full((4, 4, 4), 0.3), 1.0, 0.05), 0.3, atol=1e-15)


# ------------------------------------------------------------- iterations

def _tiny_problem(rng, n=6, n_views=10, nu=7, nv=7):
    views = random_views(rng, n_views, radius=14.0, det_dist=10.0, pixel=1.2, allow_z=False)
    return oracle.Geom(n, n, n, 1.0, (0, 0, 0), nu, nv, views)


def test_landweber_matches_svd_closed_form(rng):
    g = _tiny_problem(rng)
    W = oracle.dense_matrix(g)
    U, sig, Vt = np.linalg.svd(W, full_matrices=False)
    b = rng.random(g.stack_shape)
    alpha = 1.0 / sig[0] ** 2
    mu = np.zeros(g.vol_shape)
    for k in range(1, 6):
        mu, _ = oracle.landweber_step(g, mu, b, alpha, None)
        coef = np.where(sig > 1e-12 * sig[0], (1 - (1 - alpha * sig ** 2) ** k) / np.maximum(sig, 1e-300), 0.0)
        ref = Vt.T @ (coef * (U.T @ b.reshape(-1)))
        assert np.allclose(mu.reshape(-1), ref, atol=1e-10 * np.abs(ref).max())


def test_identity_preconditioner_reduces_eq4_to_eq2(rng):
    g = _tiny_problem(rng)
    mu0 = rng.random(g.vol_shape)
    b = rng.random(g.stack_shape)
    delta = np.zeros((3, 3, 3))
    delta[1, 1, 1] = 1.0
    m1, r1 = oracle.landweber_step(g, mu0, b, 0.01, oracle.filter_stencil27(delta))
    m2, r2 = oracle.landweber_step(g, mu0, b, 0.01, None)
    assert np.array_equal(m1, m2) and r1 == r2


@pytest.mark.parametrize("kind", ["identity", "stencil27", "radial"])
def test_monotone_residual_on_consistent_data(rng, kind):
    g = _tiny_problem(rng, n=8, n_views=16, nu=10, nv=10)
    truth = rng.random(g.vol_shape)
    b = oracle.project(g, truth)
    filt = {"identity": oracle.filter_identity(), "stencil27": oracle.filter_stencil27(),
            "radial": oracle.filter_radial(n=8)}[kind]
    lam = oracle.power_iteration(g, filt, iters=60)
    alpha = 1.0 / lam
    mu = np.zeros(g.vol_shape)
    res = []
    for _ in range(12):
        mu, r = oracle.landweber_step(g, mu, b, alpha, filt)
        res.append(r)
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))
    assert res[-1] < res[0]


def test_power_iteration_against_eigen_solver(rng):
    g = _tiny_problem(rng)
    W = oracle.dense_matrix(g)
    lam_ref = np.linalg.eigvalsh(W.T @ W).max()
    assert oracle.power_iteration(g, None, iters=400) == pytest.approx(lam_ref, rel=1e-6)
    # with eq. 5's kernel: eigenvalues of P W^T W (P the circulant matrix)
    n = g.nx * g.ny * g.nz
    P = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1
        P[:, i] = oracle.stencil27(e.reshape(g.vol_shape)).reshape(-1)
    lam_p = np.max(np.linalg.eigvals(P @ W.T @ W).real)
    assert oracle.power_iteration(g, oracle.filter_stencil27(), iters=600) == pytest.approx(lam_p, rel=1e-5)


def test_splitmix64_published_outputs():
    # SplitMix64 from state 0: 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f
    u = oracle.splitmix64_uniform(0, 3)
    top = [int(x * 2 ** 53) for x in u]
    assert top == [0xe220a8397b1dcdaf >> 11, 0x6e789e6aa1b965f4 >> 11, 0x06c45d188009454f >> 11]


def _one_voxel_one_ray(h=1.0):
    views = np.array([[-10.0, 0.1, 0.05, 10.0, 0.1, 0.05, 0, 1, 0, 0, 0, 1]])
    return oracle.Geom(1, 1, 1, h, (0, 0, 0), 1, 1, views)


def test_osemtr_one_voxel_is_newton():
    g = _one_voxel_one_ray(0.7)
    a = oracle.project(g, np.ones((1, 1, 1)))[0, 0, 0]
    mu_true = 1.3
    b = np.full((1, 1, 1), a * mu_true)
    y = math.exp(-a * mu_true)
    mu = 0.2
    errs = []
    for _ in range(6):
        new = oracle.osemtr(g, np.full((1, 1, 1), mu), b, M=1, passes=1)[0, 0, 0]
        newton = mu - (math.exp(-a * mu) - y) / (-a * math.exp(-a * mu))
        assert new == pytest.approx(newton, rel=1e-13)
        mu = new
        errs.append(abs(mu - mu_true))
    assert errs[-1] < 1e-12
    assert errs[2] < 10 * errs[1] ** 2 / mu_true          # quadratic convergence


def test_osemtr_fixed_point_and_full_batch(rng):
    g = _tiny_problem(rng, n=6, n_views=8)
    mu = rng.random(g.vol_shape) * 0.1
    b = oracle.project(g, mu)
    assert np.allclose(oracle.osemtr(g, mu, b, M=4, passes=1), mu, atol=1e-13)
    # M = 1 is one full-batch update of eq. 3, written out
    b2 = b + 0.01 * rng.random(b.shape)
    e = np.exp(-oracle.project(g, mu))
    pi = oracle.project(g, np.ones(g.vol_shape))
    num = oracle.backproject(g, e - np.exp(-b2))
    den = oracle.backproject(g, e * pi)
    ok = den > 1e-6 * den.max()
    ref = mu.copy()
    ref[ok] += num[ok] / den[ok]
    assert np.allclose(oracle.osemtr(g, mu, b2, M=1, passes=1), ref, atol=1e-14)


def test_multigrid_single_level_is_one_landweber_step(rng):
    g = _tiny_problem(rng, n=8, n_views=12, nu=8, nv=8)
    mu0 = rng.random(g.vol_shape)
    b = rng.random(g.stack_shape)
    f = oracle.filter_stencil27()
    m1, hist = oracle.multigrid(g, mu0, b, levels=1, n_outer=1, filt=f, alphas=[0.003])
    m2, r = oracle.landweber_step(g, mu0, b, 0.003, f)
    assert np.array_equal(m1, m2) and hist[0, 0] == r


def test_bilateral_hand_value():
    """1 x 1 x 3 volume (0, 0.1, 0.3), sigma_s = 0.8, sigma_r = 0.2.  Every
    neighbour is one voxel away, so its spatial weight is exp(-1/1.28) and its
    range weight exp(-delta^2/0.08):
      left end   (0 + 0.1 w1) / (1 + w1),             w1 = exp(-0.78125 - 0.125)
      middle     (0.1 + 0.3 w2) / (1 + w1 + w2),      w2 = exp(-0.78125 - 0.5)
      right end  (0.3 + 0.1 w2) / (1 + w2)
    evaluated by hand to 0.028776781576, 0.108999288453, 0.256532495791.
    A range term without its factor 2 would give 0.0987 in the middle, |delta|
    in place of delta^2 0.0952."""
    x = np.array([0.0, 0.1, 0.3]).reshape(1, 1, 3)
    out = oracle.bilateral(x, 0.8, 0.2).reshape(-1)
    assert out == pytest.approx([0.028776781576, 0.108999288453, 0.256532495791], abs=1e-11)
    # the same line along y and along z gives the same values (isotropic weights)
    assert np.allclose(oracle.bilateral(x.reshape(1, 3, 1), 0.8, 0.2).reshape(-1), out, atol=1e-15)
    assert np.allclose(oracle.bilateral(x.reshape(3, 1, 1), 0.8, 0.2).reshape(-1), out, atol=1e-15)


# ------------------------------------------------------------- Algorithm 1

def _mg_problem(rng, n=8, n_views=12, nu=8, nv=8):
    return _tiny_problem(rng, n=n, n_views=n_views, nu=nu, nv=nv)


def test_coarse_grid_centres_are_child_means(rng):
    """The coarse grid of Algorithm 1 keeps s and d and doubles h and the pixel
    steps: every coarse voxel centre is the mean of its 8 fine children and
    every coarse pixel centre the mean of its 2 x 2 fine pixels."""
    g = _mg_problem(rng)
    c = g.level(1)

    def vox(gg):
        i = (np.arange(gg.nx) - (gg.nx - 1) / 2) * gg.h + gg.origin[0]
        j = (np.arange(gg.ny) - (gg.ny - 1) / 2) * gg.h + gg.origin[1]
        k = (np.arange(gg.nz) - (gg.nz - 1) / 2) * gg.h + gg.origin[2]
        return i, j, k

    (fi, fj, fk), (ci, cj, ck) = vox(g), vox(c)
    assert np.allclose(ci, fi.reshape(-1, 2).mean(1), atol=1e-14)
    assert np.allclose(cj, fj.reshape(-1, 2).mean(1), atol=1e-14)
    assert np.allclose(ck, fk.reshape(-1, 2).mean(1), atol=1e-14)

    def pix(gg, v):
        s, d, u, w = gg.views[v, 0:3], gg.views[v, 3:6], gg.views[v, 6:9], gg.views[v, 9:12]
        a = np.arange(gg.nu) - (gg.nu - 1) / 2
        b = np.arange(gg.nv) - (gg.nv - 1) / 2
        return d + a[None, :, None] * u + b[:, None, None] * w, s

    for v in range(g.n_views):
        pf, sf = pix(g, v)
        pc, sc = pix(c, v)
        assert np.array_equal(sf, sc)
        mean = pf.reshape(g.nv // 2, 2, g.nu // 2, 2, 3).mean(axis=(1, 3))
        assert np.allclose(pc, mean, atol=1e-12)


def test_multigrid_without_coarse_change_is_one_fine_step(rng):
    """When the coarse grids leave the restricted volume unchanged (no OS-EMTR
    pass, and a zero step on the intermediate grid), Algorithm 1's correction
    mu += P(mu_c1 - mu_c0) adds exactly zero, so one iteration is exactly one
    grid-0 Landweber step followed by the regularisers.  Prolongating mu_c1
    instead of the coarse change, or restricting the wrong level's data,
    breaks it."""
    g = _mg_problem(rng)
    mu0 = rng.random(g.vol_shape)
    b = rng.random(g.stack_shape)
    f = oracle.filter_stencil27()
    # two grids, with both regularisers on
    m, hist = oracle.multigrid(g, mu0, b, levels=2, n_outer=1, filt=f, alphas=[0.004, 1.0], lam=0.01,
                               bilateral_on=True, sigma_s=0.9, sigma_r=0.3, coarse_passes=0)
    ref, r = oracle.landweber_step(g, mu0, b, 0.004, f)
    ref = oracle.bilateral(oracle.soft_threshold(ref, 0.01), 0.9, 0.3)
    assert np.array_equal(m, ref) and hist[0, 0] == r
    # the coarse residual is the restricted data against the restricted volume
    gc = g.level(1)
    assert hist[0, 1] == pytest.approx(np.linalg.norm(oracle.restrict_stack(b) - oracle.project(gc, oracle.restrict_volume(mu0))), rel=1e-14)
    # three grids, zero step on grid 1
    m3, hist3 = oracle.multigrid(g, mu0, b, levels=3, n_outer=1, filt=f, alphas=[0.004, 0.0, 1.0],
                                 coarse_passes=0)
    ref3, r3 = oracle.landweber_step(g, mu0, b, 0.004, f)
    assert np.array_equal(m3, ref3) and hist3[0, 0] == r3
    # the same with a non-zero coarse step does change the result
    m3b, _ = oracle.multigrid(g, mu0, b, levels=3, n_outer=1, filt=f, alphas=[0.004, 0.002, 1.0],
                              coarse_passes=0)
    assert np.linalg.norm(m3b - ref3) > 1e-6 * np.linalg.norm(ref3)


@pytest.mark.parametrize("levels", [2, 3])
def test_multigrid_injection_fixed_point(rng, levels):
    """mu = piecewise-constant injection of a coarsest-grid volume x_c, data
    b_0 = A_{L-1} x_c repeated over the 2^(L-1) x 2^(L-1) fine pixels of each
    coarsest pixel.  The restricted data on the coarsest grid are then
    exactly A_{L-1} x_c, the restricted volume exactly x_c, so the coarse
    OS-EMTR solve starts at its fixed point (eq. 3: e^{-A x} = I/I0) and, with
    a zero step on the finer grids, one iteration of Algorithm 1 returns mu
    unchanged.  The coarse residual it records is zero."""
    f = 2 ** (levels - 1)
    g = _mg_problem(rng, n=8, n_views=10, nu=8, nv=8)
    gc = g.level(levels - 1)
    xc = rng.random(gc.vol_shape) * 0.05
    mu = xc
    for _ in range(levels - 1):
        mu = np.repeat(np.repeat(np.repeat(mu, 2, 0), 2, 1), 2, 2)
    bc = oracle.project(gc, xc)
    b0 = np.repeat(np.repeat(bc, f, 1), f, 2)
    assert b0.shape == g.stack_shape
    out, hist = oracle.multigrid(g, mu, b0, levels=levels, n_outer=1, filt=oracle.filter_identity(),
                                 alphas=[0.0] * levels, coarse_M=2, coarse_passes=3)
    assert np.allclose(out, mu, rtol=0, atol=1e-13)
    assert hist[0, levels - 1] < 1e-13 * np.linalg.norm(bc)
    # a wrong coarse datum (the data not restricted, only subsampled) is not a fixed point
    b_bad = b0.copy()
    b_bad[:, 0::f, 0::f] += 0.01
    out_bad, _ = oracle.multigrid(g, mu, b_bad, levels=levels, n_outer=1, filt=oracle.filter_identity(),
                                  alphas=[0.0] * levels, coarse_M=2, coarse_passes=3)
    assert np.abs(out_bad - mu).max() > 1e-6

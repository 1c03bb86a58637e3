"""Pins of the oracle's derived-preconditioner functions (CPU): the transfer
function of A^T A against the dense system matrix built from the weight
definition, its two closed-form sums, and the shell averages on constants and
on rho itself."""

import math

import numpy as np

import oracle


def _geom():
    views = []
    for k in range(6):
        th = 2 * math.pi * k * 0.618034
        c, s = math.cos(th), math.sin(th)
        views.append([30 * c, 30 * s, 0.7 * (k % 2), -30 * c, -30 * s, 0.7 * (k % 2),
                      -1.6 * s, 1.6 * c, 0, 0, 0, 1.6])
    return oracle.Geom(8, 8, 8, 1.0, (0, 0, 0), 7, 6, np.array(views))


def test_psf_spectrum_equals_dense_matrix_column():
    g = _geom()
    A = oracle.dense_matrix(g)
    c = (g.nz // 2) * g.ny * g.nx + (g.ny // 2) * g.nx + g.nx // 2
    psf = (A.T @ A[:, c]).reshape(g.vol_shape)
    X = np.fft.fftn(psf)
    n = np.array([g.nz, g.ny, g.nx])
    k = np.indices(g.vol_shape)
    ph = 2 * np.pi * sum(k[a] * (n[a] // 2) / n[a] for a in range(3))
    ref = np.real(X * np.exp(1j * ph))
    T = oracle.psf_spectrum(g)
    assert np.allclose(T, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # inverse DFT at the impulse: sum_k T = N^3 psf[c] = N^3 ||A e_c||^2; DC = sum of the response
    assert abs(T.sum() - T.size * float(A[:, c] @ A[:, c])) < 1e-10 * T.size * float(A[:, c] @ A[:, c])
    assert abs(T.flat[0] - psf.sum()) < 1e-12 * psf.sum()


def test_transfer_from_spectrum_closed_form():
    T = np.array([4.0, 2.0, 0.01, -1.0])
    H = oracle.transfer_from_spectrum(T, 0.1)
    assert np.allclose(H, [0.25, 0.5, 1 / 0.4, 1 / 0.4])


def test_radial_profile_constants_and_rho():
    shape = (8, 16, 4)
    n_table, rho_max = 33, math.sqrt(3.0)
    prof, cnt = oracle.radial_profile(np.full(shape, 3.0), n_table, rho_max)
    assert cnt.sum() == np.prod(shape)
    assert np.allclose(prof[cnt > 0], 3.0) and np.all(np.isnan(prof[cnt == 0]))
    # T = rho (in FP64): each shell's mean lies within half a sample of the sample's rho
    k = [np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n) / n for n in shape]
    kz, ky, kx = np.meshgrid(*k, indexing="ij")
    rho = 2 * np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    prof, cnt = oracle.radial_profile(rho, n_table, rho_max)
    step = rho_max / (n_table - 1)
    centres = np.arange(n_table) * step
    assert np.all(np.abs(prof[cnt > 0] - centres[cnt > 0]) <= 0.5 * step + 1e-6)


def test_radial_profile_counts_by_enumeration():
    """Shell counts against a plain loop over every frequency with exact
    rational k/N: shell = nearest sample of [0, rho_max] to rho."""
    shape = (4, 8, 6)
    n_table, rho_max = 9, math.sqrt(3.0)
    prof, cnt = oracle.radial_profile(np.zeros(shape), n_table, rho_max)
    ref = np.zeros(n_table, dtype=int)
    for kz in range(shape[0]):
        for ky in range(shape[1]):
            for kx in range(shape[2]):
                f = [(k if k < n // 2 else k - n) / n for k, n in zip((kz, ky, kx), shape)]
                rho = 2 * math.sqrt(sum(q * q for q in f))
                best = min(range(n_table), key=lambda i: abs(i * rho_max / (n_table - 1) - rho))
                if abs(best * rho_max / (n_table - 1) - rho) <= 0.5 * rho_max / (n_table - 1):
                    ref[best] += 1
    assert np.array_equal(cnt, ref)

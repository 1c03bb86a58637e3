"""Oracle for everything around the projector (FP64, numpy; test infrastructure only).

Each function follows one passage of the paper (cited in its docstring).
Where the paper leaves a constant or an operator unstated, the reading used
is stated in the docstring.
"""

from __future__ import annotations

import math

import numpy as np

from .core import Geom, backproject, project

__all__ = [
    "STENCIL27_TAPS", "stencil27", "radial_table", "radial_response", "radial_filter",
    "precondition", "restrict_volume", "restrict_stack", "prolongate", "soft_threshold",
    "bilateral", "splitmix64_uniform", "power_iteration", "landweber_step", "osemtr",
    "multigrid", "filter_identity", "filter_stencil27", "filter_radial",
    "perturbation_jacobian", "geometry_param_grad",
    "psf_spectrum", "transfer_from_spectrum", "radial_profile", "transfer_filter",
]


# ---------------------------------------------------------------------------
# Preconditioners p (paper Sec. 3, eq. 4 and eq. 5)
# ---------------------------------------------------------------------------

def _eq5_taps() -> np.ndarray:
    """The empirically chosen 3^3 kernel of eq. 5, /64.  The three printed
    3x3 matrices are read as the z = -1, 0, +1 slices (z is the rotation
    axis), each indexed [y][x]; indices are [dz+1][dy+1][dx+1]."""
    outer = [[-1, -1, -1], [-1, 0, -1], [-1, -1, -1]]
    middle = [[-8, -4, -8], [-4, 64, -4], [-8, -4, -8]]
    return np.array([outer, middle, outer], dtype=np.float64) / 64.0


STENCIL27_TAPS = _eq5_taps()


def stencil27(x: np.ndarray, taps: np.ndarray = STENCIL27_TAPS) -> np.ndarray:
    """Circular 3-D convolution with a 3^3 kernel (eq. 4's p * g, eq. 5 taps):
    out[z,y,x] = sum_d taps[d] * x[(z,y,x) - d] with indices wrapped."""
    taps = np.asarray(taps, dtype=np.float64).reshape(3, 3, 3)
    out = np.zeros_like(x, dtype=np.float64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                w = taps[dz + 1, dy + 1, dx + 1]
                if w != 0.0:
                    out += w * np.roll(x, shift=(dz, dy, dx), axis=(0, 1, 2))
    return out


def radial_table(n: int, n_table: int = 4097, rho_max: float = math.sqrt(3.0)):
    """Default isotropic deconvolution profile H(rho) = max(rho, 2/n), sampled
    on n_table points in [0, rho_max].  Reading: the paper calls for an
    approximate deconvolution of the point-spread function of B P (Sec. 3)
    and gives no profile beyond eq. 5; for a complete, isotropic trajectory
    that PSF falls off as 1/|x|^2, whose inverse is a 3-D ramp.  The floor
    keeps a non-zero response at DC (the paper notes, Sec. 3, that eq. 5's
    zero DC response lets the grey levels drift)."""
    rho = np.linspace(0.0, rho_max, n_table)
    return np.maximum(rho, 2.0 / n), rho_max


def radial_response(shape, table: np.ndarray, rho_max: float) -> np.ndarray:
    """H on the DFT grid: rho = 2 sqrt(sum_a (k_a/N_a)^2) with signed
    frequencies k_a in [-N_a/2, N_a/2), H(rho) by linear interpolation of
    the uniformly sampled table (clamped beyond rho_max)."""
    nz, ny, nx = shape
    fz = np.fft.fftfreq(nz)[:, None, None]
    fy = np.fft.fftfreq(ny)[None, :, None]
    fx = np.fft.fftfreq(nx)[None, None, :]
    rho = 2.0 * np.sqrt(fz * fz + fy * fy + fx * fx)
    grid = np.linspace(0.0, rho_max, len(table))
    return np.interp(rho, grid, np.asarray(table, dtype=np.float64))


def radial_filter(x: np.ndarray, table: np.ndarray, rho_max: float) -> np.ndarray:
    """p * g as a circular convolution evaluated in Fourier space, with the
    3-D DFT sized to the volume: IDFT(DFT(g) H)."""
    H = radial_response(x.shape, table, rho_max)
    return np.real(np.fft.ifftn(np.fft.fftn(x) * H))


def filter_identity():
    return dict(kind="identity")


def filter_stencil27(taps=None):
    return dict(kind="stencil27", taps=STENCIL27_TAPS if taps is None else np.asarray(taps).reshape(3, 3, 3))


def filter_radial(table=None, rho_max=math.sqrt(3.0), n=None):
    if table is None:
        table, rho_max = radial_table(n)
    return dict(kind="radial", table=np.asarray(table, dtype=np.float64), rho_max=float(rho_max))


def precondition(x: np.ndarray, filt) -> np.ndarray:
    """Apply the preconditioner p of eq. 4 (identity gives plain SIRT, eq. 2)."""
    if filt is None or filt["kind"] == "identity":
        return np.array(x, dtype=np.float64)
    if filt["kind"] == "stencil27":
        return stencil27(x, filt["taps"])
    if filt["kind"] == "radial":
        return radial_filter(x, filt["table"], filt["rho_max"])
    raise ValueError(filt["kind"])


# ---------------------------------------------------------------------------
# Grid transfer (Algorithm 1: Restrict, Prolongate)
# ---------------------------------------------------------------------------

def restrict_volume(x: np.ndarray) -> np.ndarray:
    """Restrict of Algorithm 1 for the volume: mean of each 2x2x2 block.
    Reading: the operator is not stated; the block mean keeps the coarse
    voxel equal to the average attenuation it covers."""
    nz, ny, nx = x.shape
    return x.reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(1, 3, 5))


def restrict_stack(b: np.ndarray) -> np.ndarray:
    """Restrict of Algorithm 1 for the radiographs: mean of each 2x2 pixel
    block of the data b = ln(I0/I) (reading: the paper restricts I; the mean
    of b is used because b is linear in mu)."""
    V, nv, nu = b.shape
    return b.reshape(V, nv // 2, 2, nu // 2, 2).mean(axis=(2, 4))


def _prolong_axis(x: np.ndarray, axis: int) -> np.ndarray:
    nc = x.shape[axis]
    i = np.arange(2 * nc)
    c = (i + 0.5) / 2.0 - 0.5          # fine cell centre in coarse index units
    i0 = np.floor(c).astype(int)
    w = c - i0
    lo = np.clip(i0, 0, nc - 1)
    hi = np.clip(i0 + 1, 0, nc - 1)
    xl = np.take(x, lo, axis=axis)
    xh = np.take(x, hi, axis=axis)
    shape = [1] * x.ndim
    shape[axis] = 2 * nc
    w = w.reshape(shape)
    return (1.0 - w) * xl + w * xh


def prolongate(x: np.ndarray) -> np.ndarray:
    """Prolongate of Algorithm 1: cell-centred trilinear interpolation to the
    grid with twice the resolution (weights 3/4, 1/4; edges clamped).
    Reading: the operator is not stated."""
    out = x
    for ax in range(3):
        out = _prolong_axis(out, ax)
    return out


# ---------------------------------------------------------------------------
# Regularisers (Algorithm 1: SoftThreshold, BilateralFilter)
# ---------------------------------------------------------------------------

def soft_threshold(x: np.ndarray, lam: float) -> np.ndarray:
    """L1 regularisation by soft thresholding: sign(x) max(|x| - lam, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - lam, 0.0)


def bilateral(x: np.ndarray, sigma_s: float, sigma_r: float) -> np.ndarray:
    """Local regularisation by a bilateral filter over the 3^3 neighbourhood
    (neighbours outside the grid are left out): each output voxel is the
    weighted mean of its neighbours with weights
    exp(-|d|^2 / (2 sigma_s^2)) exp(-(x_n - x)^2 / (2 sigma_r^2)).
    Reading: the neighbourhood and both sigmas are not stated."""
    nz, ny, nx = x.shape
    pad = np.pad(x, 1, mode="constant")
    inside = np.pad(np.ones_like(x), 1, mode="constant")
    num = np.zeros_like(x)
    den = np.zeros_like(x)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                sl = (slice(1 + dz, 1 + dz + nz), slice(1 + dy, 1 + dy + ny), slice(1 + dx, 1 + dx + nx))
                xn = pad[sl]
                m = inside[sl]
                w = m * math.exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * sigma_s ** 2)) \
                    * np.exp(-((xn - x) ** 2) / (2.0 * sigma_r ** 2))
                num += w * xn
                den += w
    return num / den


# ---------------------------------------------------------------------------
# Step size (power iteration) and the iterations
# ---------------------------------------------------------------------------

_M64 = (1 << 64) - 1


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """n uniforms in [0,1): output k is SplitMix64 (Steele, Lea & Flood 2014)
    at state seed + (k+1) * 0x9E3779B97F4A7C15, top 53 bits / 2^53."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def power_iteration(geom: Geom, filt, iters: int = 30, seed: int = 0, x0=None) -> float:
    """Largest eigenvalue of x -> p * A^T A x by power iteration from a
    SplitMix64-uniform start vector (normalised), returning ||M x_{k}|| with
    ||x_k|| = 1 after ``iters`` products.  The step of eq. 2 / eq. 4 is
    alpha = omega / lambda (reading: the paper's "detector width in pixels"
    heuristic depends on its projector's scaling, so alpha is taken from the
    spectrum instead; omega = 1 keeps alpha < 2 / lambda_max)."""
    n = geom.nx * geom.ny * geom.nz
    x = splitmix64_uniform(seed, n).reshape(geom.vol_shape) if x0 is None else np.array(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = precondition(backproject(geom, project(geom, x)), filt)
        lam = float(np.linalg.norm(y))
        if lam == 0.0:
            return 0.0
        x = y / lam
    return lam


def landweber_step(geom: Geom, mu: np.ndarray, b: np.ndarray, alpha: float, filt=None):
    """One (preconditioned) Landweber iteration, eq. 2 (filt identity / None,
    i.e. SIRT) or eq. 4: mu + alpha p * B(b - P mu).  Returns the new volume
    and ||b - P mu|| of the input volume."""
    r = b - project(geom, mu)
    g = precondition(backproject(geom, r), filt)
    return mu + alpha * g, float(np.linalg.norm(r))


def osemtr(geom: Geom, mu: np.ndarray, b: np.ndarray, M: int = 8, passes: int = 2,
           rel_floor: float = 1e-6, pi=None):
    """Ordered-subset EM for transmission tomography, eq. 3.  Views are split
    into M interleaved subsets (view i in subset i mod M); for each subset:
    mu += B_m{exp(-P_m mu) - I/I0} / B_m{exp(-P_m mu) (P_m 1)}, where
    I/I0 = exp(-b) and P 1 (the projected length of the support) uses the
    whole grid as support.  Voxels whose denominator is not above
    rel_floor * max(denominator) are left unchanged.  One pass visits every
    subset once (the paper's "single full-resolution iteration")."""
    mu = np.array(mu, dtype=np.float64)
    if pi is None:
        pi = project(geom, np.ones(geom.vol_shape))
    y = np.exp(-b)
    for _ in range(passes):
        for m in range(M):
            idx = np.arange(m, geom.n_views, M)
            gm = geom.subset(idx)
            e = np.exp(-project(gm, mu))
            num = backproject(gm, e - y[idx])
            den = backproject(gm, e * pi[idx])
            ok = den > rel_floor * den.max()
            mu[ok] += num[ok] / den[ok]
    return mu


def multigrid(geom: Geom, mu: np.ndarray, b: np.ndarray, levels: int, n_outer: int, filt,
              alphas, lam: float = 0.0, bilateral_on: bool = False, sigma_s: float = 1.0,
              sigma_r: float = 0.05, coarse_M: int = 8, coarse_passes: int = 2, filters=None):
    """Algorithm 1 (recursive multigrid), ``n_outer`` full iterations from mu.

    MG(mu, g):  restrict mu (and, once, the data) to grid g+1; solve there by
    MG(., g+1) or, on the coarsest grid L-1, by OS-EMTR; add the prolongated
    coarse change mu_c(new) - mu_c(old); one preconditioned Landweber step
    (eq. 4) with step alphas[g]; soft threshold (lam); bilateral filter.
    Reading: the coarse problem is the full restricted problem (the paper
    restricts both mu and I), and the preconditioner on grid g is ``filt``
    re-sized to that grid (``filters[g]`` overrides).  With levels == 1 an
    iteration is just the Landweber step and the regularisers.

    Returns (mu, hist) with hist[n][g] = ||b_g - A_g mu|| at grid g's
    Landweber step (g < L-1) and, for g = L-1, the coarse residual before
    OS-EMTR.
    """
    L = int(levels)
    geoms = [geom.level(g) for g in range(L)]
    data = [np.asarray(b, dtype=np.float64)]
    for g in range(1, L):
        data.append(restrict_stack(data[-1]))
    flts = filters if filters is not None else [filt] * L
    hist = np.zeros((n_outer, L))

    def regularise(x):
        if lam > 0.0:
            x = soft_threshold(x, lam)
        if bilateral_on:
            x = bilateral(x, sigma_s, sigma_r)
        return x

    def mg(x, g, n):
        if g + 1 < L:
            xc0 = restrict_volume(x)
            if g + 1 < L - 1:
                xc1 = mg(xc0.copy(), g + 1, n)
            else:
                hist[n, L - 1] = np.linalg.norm(data[L - 1] - project(geoms[L - 1], xc0))
                xc1 = osemtr(geoms[L - 1], xc0, data[L - 1], coarse_M, coarse_passes)
            x = x + prolongate(xc1 - xc0)
        x, rn = landweber_step(geoms[g], x, data[g], alphas[g], flts[g])
        hist[n, g] = rn
        return regularise(x)

    x = np.array(mu, dtype=np.float64)
    for n in range(n_outer):
        x = mg(x, 0, n)
    return x, hist


# ---------------------------------------------------------------------------
# Joint geometry estimation (paper Sec. 1: model parameters such as drift
# estimated jointly with the image)
# ---------------------------------------------------------------------------

def perturbation_jacobian(views0: np.ndarray, h: float, dx: float, dz: float, tilt_deg: float) -> np.ndarray:
    """d(views)/d(dx, dz, tilt) for the perturbation model: the source moves
    by dx*h along the view's unit column direction and dz*h along z; the
    column and row steps rotate by tilt (degrees) about the detector normal,
    keeping their lengths.  Returns (V, 12, 3)."""
    V = views0.shape[0]
    J = np.zeros((V, 12, 3))
    u0, v0 = views0[:, 6:9], views0[:, 9:12]
    lu = np.linalg.norm(u0, axis=1, keepdims=True)
    lv = np.linalg.norm(v0, axis=1, keepdims=True)
    uh, vh = u0 / lu, v0 / lv
    J[:, 0:3, 0] = h * uh
    J[:, 2, 1] = h
    t = math.radians(tilt_deg)
    c, s = math.cos(t), math.sin(t)
    k = math.pi / 180.0
    J[:, 6:9, 2] = k * lu * (-s * uh + c * vh)
    J[:, 9:12, 2] = k * lv * (-c * uh - s * vh)
    return J


def geometry_param_grad(views0, dviews, h, dx, dz, tilt_deg) -> np.ndarray:
    """Chain rule: gradient with respect to (dx, dz, tilt) from the per-view
    gradient with respect to (s, d, u, v)."""
    J = perturbation_jacobian(np.asarray(views0, dtype=np.float64), h, dx, dz, tilt_deg)
    return np.einsum("vk,vkp->p", np.asarray(dviews, dtype=np.float64), J)


# ---------------------------------------------------------------------------
# Preconditioners derived from the scan (Sec. 3 leaves more rigorously derived
# kernels to later work; these measure the one the scan implies).

def psf_spectrum(geom: Geom) -> np.ndarray:
    """Transfer function of A^T A: the real part of the 3-D DFT of
    A^T A applied to a unit impulse at voxel (nx/2, ny/2, nz/2), multiplied by
    exp(+2 pi i k.c/n) to move the impulse to the origin (shift theorem).  The
    real part is the transfer function of the even part of that response.
    [kz][ky][kx] in DFT order.  parity pinned: the dense matrix's column,
    sum_k T = N^3 ||A e_c||^2 and T[0] = sum of the response."""
    c = (geom.nx // 2, geom.ny // 2, geom.nz // 2)
    delta = np.zeros(geom.vol_shape)
    delta[c[2], c[1], c[0]] = 1.0
    psf = backproject(geom, project(geom, delta))
    X = np.fft.fftn(psf)
    kz, ky, kx = np.meshgrid(np.arange(geom.nz), np.arange(geom.ny), np.arange(geom.nx), indexing="ij")
    phase = 2.0 * np.pi * (kx * c[0] / geom.nx + ky * c[1] / geom.ny + kz * c[2] / geom.nz)
    return np.real(X * np.exp(1j * phase))


def transfer_from_spectrum(T: np.ndarray, floor_rel: float) -> np.ndarray:
    """H = 1 / max(T, floor_rel * T[0]) (T[0] = the DC gain)."""
    return 1.0 / np.maximum(T, floor_rel * T.flat[0])


def radial_profile(T: np.ndarray, n_table: int, rho_max: float):
    """Mean of T over each shell of frequencies: the frequency with signed
    indices k_a in [-N_a/2, N_a/2) has rho = 2 sqrt(sum_a (k_a/N_a)^2) (the
    radial coordinate of the Fourier filter, Sec. 3's approximate
    deconvolution) and belongs to the shell of the nearest of n_table
    uniform samples of [0, rho_max], i.e. floor(rho / rho_max (n_table-1)
    + 1/2); frequencies beyond the last sample are left out.  rho and the
    shell index are evaluated in FP64 from that definition.  Returns (means
    with NaN for empty shells, counts).  parity pinned: shell means of
    constants and of rho itself, counts against a brute-force enumeration."""
    nz, ny, nx = T.shape
    def signed(n):
        k = np.arange(n)
        return np.where(k < n // 2, k, k - n).astype(np.float64) / float(n)
    fz, fy, fx = np.meshgrid(signed(nz), signed(ny), signed(nx), indexing="ij")
    rho = 2.0 * np.sqrt(fx * fx + fy * fy + fz * fz)
    b = np.floor(rho / float(rho_max) * (n_table - 1) + 0.5).astype(np.int64)
    keep = b < n_table
    sums = np.bincount(b[keep], weights=T[keep].astype(np.float64), minlength=n_table)
    cnt = np.bincount(b[keep], minlength=n_table)
    with np.errstate(invalid="ignore", divide="ignore"):
        prof = np.where(cnt > 0, sums / np.maximum(cnt, 1), np.nan)
    return prof, cnt


def transfer_filter(x: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Circular convolution with transfer function H (DFT order): real part
    of IDFT(DFT(x) H)."""
    return np.real(np.fft.ifftn(np.fft.fftn(x) * H))

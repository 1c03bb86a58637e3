"""Python binding of libmgct (the C ABI declared in include/mgct.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of libmgct.so.  The raw entry points are exposed under their C
names (``mgct_project`` ...); ``Context`` wraps them for torch tensors that
live on the GPU.  Importing this package does not need a GPU; loading the
library does, and fails loudly if it has not been built.
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmgct.so")

MGCT_OK = 0
MGCT_ERR_INVALID_ARG = -1
MGCT_ERR_UNSUPPORTED_GEOMETRY = -2
MGCT_ERR_SIZE_NOT_DIVISIBLE = -3
MGCT_ERR_OOM = -4
MGCT_ERR_HIP = -5
MGCT_ERR_DIVERGED = -6
MGCT_ERR_NOT_IMPLEMENTED = -7
MGCT_ERR_NO_GEOMETRY = -8
MGCT_ERR_TOO_LARGE = -9

MGCT_F32, MGCT_F16, MGCT_BF16 = 0, 1, 2
MGCT_FILTER_IDENTITY, MGCT_FILTER_STENCIL27, MGCT_FILTER_RADIAL, MGCT_FILTER_TRANSFER = 0, 1, 2, 3


class mgct_filter(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("taps", ctypes.c_float * 27),
        ("radial_table", ctypes.POINTER(ctypes.c_float)),
        ("n_table", ctypes.c_int),
        ("rho_max", ctypes.c_float),
        ("transfer", ctypes.c_void_p * 8),
    ]


class mgct_mg_params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("n_outer", ctypes.c_int),
        ("filter", mgct_filter),
        ("alpha", ctypes.c_double * 8),
        ("power_iters", ctypes.c_int),
        ("power_seed", ctypes.c_uint64),
        ("lambda_", ctypes.c_double),
        ("bilateral_on", ctypes.c_int),
        ("sigma_s", ctypes.c_double),
        ("sigma_r", ctypes.c_double),
        ("coarse_subsets", ctypes.c_int),
        ("coarse_passes", ctypes.c_int),
        ("learned", ctypes.c_int),
        ("capture_update", ctypes.c_void_p),
        ("capture_iterate", ctypes.c_void_p),
    ]


# name -> (restype, argtypes); mirrors include/mgct.h
_vp, _ci, _cd, _u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(mgct_filter)
SIGNATURES = {
    "mgct_status_string": (ctypes.c_char_p, [_ci]),
    "mgct_filter_eq5": (_ci, [_fp]),
    "mgct_create": (_ci, [_ci, ctypes.POINTER(_vp)]),
    "mgct_destroy": (_ci, [_vp]),
    "mgct_set_geometry": (_ci, [_vp, _ci, _ci, _ci, _cd, _dp, _ci, _ci, _ci, _dp]),
    "mgct_project": (_ci, [_vp, _ci, _vp, _ci, _vp, _ci, _vp]),
    "mgct_backproject": (_ci, [_vp, _ci, _vp, _ci, _vp, _ci, _vp]),
    "mgct_project_noalloc": (_ci, [_vp, _ci, _vp, _ci, _vp, _ci, _vp]),
    "mgct_precondition": (_ci, [_vp, _ci, _vp, _vp, _fp, _vp]),
    "mgct_estimate_step": (_ci, [_vp, _ci, _fp, _ci, _u64, _dp, _vp]),
    "mgct_landweber_step": (_ci, [_vp, _ci, _vp, _vp, _ci, _cd, _fp, _dp, _vp]),
    "mgct_set_divergence": (_ci, [_vp, _cd]),
    "mgct_set_projector": (_ci, [_vp, _ci]),
    "mgct_residual_diverged": (_ci, [_cd, _cd, _cd]),
    "mgct_psf_spectrum": (_ci, [_vp, _ci, _vp, _vp]),
    "mgct_transfer_from_spectrum": (_ci, [_vp, _ci, _vp, _cd, _vp, _vp]),
    "mgct_radial_profile": (_ci, [_vp, _ci, _vp, _ci, _cd, _dp, ctypes.POINTER(_ci), _vp]),
    "mgct_restrict_volume": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "mgct_restrict_stack": (_ci, [_vp, _ci, _vp, _vp, _vp]),
    "mgct_prolong_add": (_ci, [_vp, _ci, _vp, _vp, _vp, _vp]),
    "mgct_soft_threshold": (_ci, [_vp, _ci, _vp, _cd, _vp]),
    "mgct_bilateral": (_ci, [_vp, _ci, _vp, _vp, _cd, _cd, _vp]),
    "mgct_osemtr": (_ci, [_vp, _ci, _vp, _vp, _ci, _ci, _vp]),
    "mgct_multigrid_solve": (_ci, [_vp, _vp, _vp, _ci, ctypes.POINTER(mgct_mg_params), _dp, _vp]),
    "mgct_set_precision": (_ci, [_vp, _ci, _ci]),
    "mgct_project_geom_grad": (_ci, [_vp, _ci, _vp, _vp, _dp, _vp]),
    "mgct_geometry_param_grad": (_ci, [_ci, _dp, _dp, _cd, _cd, _cd, _cd, _dp]),
    "mgct_cnn_set_weights": (_ci, [_vp, ctypes.POINTER(ctypes.c_float), _ci]),
    "mgct_cnn_get_weights": (_ci, [_vp, ctypes.POINTER(ctypes.c_float), _ci]),
    "mgct_learned_judge": (_ci, [_vp, _dp, _dp, ctypes.POINTER(ctypes.c_int)]),
    "mgct_cnn_forward": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, _vp]),
    "mgct_cnn_gradients": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, ctypes.POINTER(ctypes.c_float), _dp, _vp]),
    "mgct_cnn_train_step": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, _cd, _dp, _vp]),
    "mgct_cnn_backward": (_ci, [_vp, _ci, _ci, _ci, _vp, _vp, ctypes.POINTER(ctypes.c_float), _vp]),
    "mgct_adam_step": (_ci, [_vp, ctypes.POINTER(ctypes.c_float), _ci, _cd, _vp]),
    "mgct_learned_stats": (_ci, [_vp, ctypes.POINTER(_ci), ctypes.POINTER(_ci)]),
    "mgct_synth_line_integrals": (_ci, [_vp, _dp, _ci, _dp, _ci, _vp, _vp]),
    "mgct_synth_voxelize": (_ci, [_vp, _dp, _ci, _dp, _ci, _ci, _vp, _vp]),
    "mgct_kernel_timing": (_ci, [_vp, _ci]),
    "mgct_kernel_time": (_ci, [_vp, _ci, _ci, _dp, ctypes.POINTER(_ci)]),
    "mgct_kernel_timing_select": (_ci, [_vp, ctypes.c_uint, ctypes.c_uint]),
}

MGCT_OP_PROJECT, MGCT_OP_BACKPROJECT, MGCT_OP_PRECONDITION = 0, 1, 2
MGCT_OP_VOLUME_TRANSPOSE, MGCT_OP_DATA_PRESCALE = 3, 4

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmgct.so (built by ``python -m paper_2103_10329_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmgct.so is not built (%s); run python -m paper_2103_10329_amd.build" % path)
    # torch carries its own HIP runtime (same soname as the system one); load
    # it first so that the library binds to that copy and the process holds a
    # single runtime shared by torch's allocator/streams and our kernels.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
        globals()[name] = fn
    _lib = lib
    return lib


class MgctError(RuntimeError):
    def __init__(self, code: int, where: str):
        load_library()
        msg = mgct_status_string(code).decode()  # noqa: F821
        super().__init__("%s failed: %s (%d)" % (where, msg, code))
        self.code = code


def check(code: int, where: str = "mgct"):
    if code != MGCT_OK:
        raise MgctError(code, where)


# --------------------------------------------------------------- filters ---

def filter_identity() -> mgct_filter:
    f = mgct_filter()
    f.kind = MGCT_FILTER_IDENTITY
    return f


def filter_eq5() -> mgct_filter:
    load_library()
    f = mgct_filter()
    check(mgct_filter_eq5(ctypes.byref(f)), "mgct_filter_eq5")  # noqa: F821
    return f


def filter_stencil27(taps) -> mgct_filter:
    f = mgct_filter()
    f.kind = MGCT_FILTER_STENCIL27
    t = np.asarray(taps, dtype=np.float32).reshape(27)
    for i in range(27):
        f.taps[i] = float(t[i])
    return f


def filter_radial(table, rho_max: float) -> mgct_filter:
    """Radial Fourier filter from a sampled profile (the array is kept alive
    on the returned structure)."""
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float32))
    f = mgct_filter()
    f.kind = MGCT_FILTER_RADIAL
    f.radial_table = t.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    f.n_table = t.size
    f.rho_max = float(rho_max)
    f._keep = t
    return f


def filter_transfer(arrays) -> mgct_filter:
    """Fourier filter with a full transfer function per grid: arrays[g] is a
    device F32 tensor of grid g's shape (DFT order) or None (the tensors are
    kept alive on the returned structure)."""
    f = mgct_filter()
    f.kind = MGCT_FILTER_TRANSFER
    for g, a in enumerate(arrays):
        if a is not None:
            f.transfer[g] = a.data_ptr()
    f._keep = list(arrays)
    return f


def ramp_table(n: int, n_table: int = 4097, rho_max: float = math.sqrt(3.0)):
    """Samples of the isotropic ramp H(rho) = max(rho, 2/n) on [0, rho_max]."""
    rho = np.linspace(0.0, rho_max, n_table)
    return np.maximum(rho, 2.0 / n).astype(np.float32), rho_max


# --------------------------------------------------------------- context ---

_DT = {"float32": MGCT_F32, "float16": MGCT_F16, "bfloat16": MGCT_BF16}


def _dtype_code(t) -> int:
    name = str(t.dtype).replace("torch.", "")
    if name not in _DT:
        raise TypeError("unsupported dtype %s" % t.dtype)
    return _DT[name]


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libmgct context bound to one device and one scan geometry."""

    def __init__(self, device: int = 0):
        load_library()
        h = ctypes.c_void_p()
        check(mgct_create(device, ctypes.byref(h)), "mgct_create")  # noqa: F821
        self.handle = h
        self.device = device
        self.geom = None

    def close(self):
        if getattr(self, "handle", None):
            mgct_destroy(self.handle)  # noqa: F821
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_geometry(self, nx, ny, nz, voxel, origin, nu, nv, views):
        views = np.ascontiguousarray(np.asarray(views, dtype=np.float64).reshape(-1, 12))
        org = np.ascontiguousarray(np.asarray(origin, dtype=np.float64).reshape(3))
        dp = ctypes.POINTER(ctypes.c_double)
        check(mgct_set_geometry(self.handle, nx, ny, nz, float(voxel), org.ctypes.data_as(dp), nu, nv,  # noqa: F821
                                views.shape[0], views.ctypes.data_as(dp)), "mgct_set_geometry")
        self.geom = dict(nx=nx, ny=ny, nz=nz, nu=nu, nv=nv, n_views=views.shape[0], voxel=voxel,
                         origin=tuple(float(o) for o in org))
        self._views_np = views.copy()

    def shapes(self, level: int = 0):
        g = self.geom
        f = 2 ** level
        return (g["nz"] // f, g["ny"] // f, g["nx"] // f), (g["n_views"], g["nv"] // f, g["nu"] // f)

    def set_precision(self, volume_copy: str = "float32", stack: str = "float32"):
        """Storage of the Landweber steps' internal copies: volume copy
        float32|bfloat16, data stacks float32|float16."""
        check(mgct_set_precision(self.handle, _DT[volume_copy], _DT[stack]), "mgct_set_precision")  # noqa: F821

    # ---- operators
    def project(self, vol, out=None, level: int = 0, out_dtype=None):
        import torch
        vs, ss = self.shapes(level)
        if out is None:
            out = torch.empty(ss, dtype=out_dtype or torch.float32, device=vol.device)
        check(mgct_project(self.handle, level, _ptr(vol), _dtype_code(vol), _ptr(out), _dtype_code(out),  # noqa: F821
                           _stream()), "mgct_project")
        return out

    def backproject(self, proj, out=None, level: int = 0, out_dtype=None):
        import torch
        vs, ss = self.shapes(level)
        if out is None:
            out = torch.empty(vs, dtype=out_dtype or torch.float32, device=proj.device)
        check(mgct_backproject(self.handle, level, _ptr(proj), _dtype_code(proj), _ptr(out), _dtype_code(out),  # noqa: F821
                               _stream()), "mgct_backproject")
        return out

    def precondition(self, x, filt, out=None, level: int = 0):
        import torch
        if out is None:
            out = torch.empty_like(x)
        check(mgct_precondition(self.handle, level, _ptr(x), _ptr(out), ctypes.byref(filt), _stream()),  # noqa: F821
              "mgct_precondition")
        return out

    def estimate_step(self, filt=None, level: int = 0, iters: int = 30, seed: int = 0) -> float:
        a = ctypes.c_double()
        fp = ctypes.byref(filt) if filt is not None else None
        check(mgct_estimate_step(self.handle, level, fp, iters, seed, ctypes.byref(a), _stream()),  # noqa: F821
              "mgct_estimate_step")
        return a.value

    def project_noalloc(self, vol, out, level: int = 0):
        """A vol into ``out`` with no device allocation (fixed per-GPU scratch;
        concurrent calls on one GPU race)."""
        check(mgct_project_noalloc(self.handle, level, _ptr(vol), _dtype_code(vol), _ptr(out),  # noqa: F821
                                   _dtype_code(out), _stream()), "mgct_project_noalloc")
        return out

    def landweber_step(self, vol, b, alpha, filt=None, level: int = 0, want_norm: bool = True):
        r = ctypes.c_double()
        fp = ctypes.byref(filt) if filt is not None else None
        check(mgct_landweber_step(self.handle, level, _ptr(vol), _ptr(b), _dtype_code(b), float(alpha), fp,  # noqa: F821
                                  ctypes.byref(r) if want_norm else None, _stream()), "mgct_landweber_step")
        return r.value if want_norm else None

    def set_projector(self, variant: str = "auto"):
        """Forward projector of the separable geometry: auto | gather | staged
        (bit-identical results)."""
        code = {"auto": 0, "gather": 1, "staged": 2}[variant]
        check(mgct_set_projector(self.handle, code), "mgct_set_projector")  # noqa: F821

    def set_divergence(self, ratio: float):
        """Ratio of the divergence test (>= 1, or 0: non-finite residuals only)."""
        check(mgct_set_divergence(self.handle, float(ratio)), "mgct_set_divergence")  # noqa: F821

    def restrict_volume(self, fine, coarse, level: int = 0):
        check(mgct_restrict_volume(self.handle, level, _ptr(fine), _ptr(coarse), _stream()),  # noqa: F821
              "mgct_restrict_volume")

    def restrict_stack(self, fine, coarse, level: int = 0):
        check(mgct_restrict_stack(self.handle, level, _ptr(fine), _ptr(coarse), _stream()),  # noqa: F821
              "mgct_restrict_stack")

    def prolong_add(self, cnew, cold, fine, level: int = 0):
        check(mgct_prolong_add(self.handle, level, _ptr(cnew), _ptr(cold), _ptr(fine), _stream()),  # noqa: F821
              "mgct_prolong_add")

    def soft_threshold(self, vol, lam, level: int = 0):
        check(mgct_soft_threshold(self.handle, level, _ptr(vol), float(lam), _stream()),  # noqa: F821
              "mgct_soft_threshold")

    def bilateral(self, x, out, sigma_s, sigma_r, level: int = 0):
        check(mgct_bilateral(self.handle, level, _ptr(x), _ptr(out), float(sigma_s), float(sigma_r),  # noqa: F821
                             _stream()), "mgct_bilateral")

    def osemtr(self, vol, b, subsets=8, passes=2, level: int = 0):
        check(mgct_osemtr(self.handle, level, _ptr(vol), _ptr(b), subsets, passes, _stream()),  # noqa: F821
              "mgct_osemtr")

    # ---- preconditioners derived from the scan
    def psf_spectrum(self, level: int = 0, out=None):
        """Transfer function of A^T A on grid `level` (device F32, DFT order)."""
        import torch
        if out is None:
            out = torch.empty(self.shapes(level)[0], dtype=torch.float32, device="cuda")
        check(mgct_psf_spectrum(self.handle, level, _ptr(out), _stream()), "mgct_psf_spectrum")  # noqa: F821
        return out

    def transfer_from_spectrum(self, T, floor_rel: float, level: int = 0, out=None):
        """H = 1 / max(T, floor_rel * T[0]) (device F32; out must not be T)."""
        import torch
        if out is None:
            out = torch.empty_like(T)
        check(mgct_transfer_from_spectrum(self.handle, level, _ptr(T), float(floor_rel), _ptr(out),  # noqa: F821
                                          _stream()), "mgct_transfer_from_spectrum")
        return out

    def derived_filter(self, levels: int, floor_rel: float = 0.03):
        """TRANSFER filter 1/max(T, floor_rel T[0]) from the measured transfer
        function T of A^T A on each of grids 0 .. levels-1 (one A and one A^T
        of an impulse and a forward DFT per grid, computed once per geometry)."""
        hs = []
        for g in range(levels):
            T = self.psf_spectrum(level=g)
            hs.append(self.transfer_from_spectrum(T, floor_rel, level=g))
            del T
        return filter_transfer(hs)

    def radial_profile(self, T, level: int = 0, n_table: int = 1025, rho_max: float = math.sqrt(3.0)):
        """Shell means of a spectrum (host float64, NaN for empty shells) and counts."""
        prof = np.zeros(n_table)
        cnt = np.zeros(n_table, dtype=np.int32)
        check(mgct_radial_profile(self.handle, level, _ptr(T), n_table, float(rho_max),  # noqa: F821
                                  prof.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream()),
              "mgct_radial_profile")
        return prof, cnt

    def project_geom_grad(self, vol, cot, level: int = 0) -> np.ndarray:
        """d/d(views) of sum(cot * A vol): (n_views, 12) float64 (s, d, u, v)."""
        out = np.zeros((self.geom["n_views"], 12))
        check(mgct_project_geom_grad(self.handle, level, _ptr(vol), _ptr(cot),  # noqa: F821
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
              "mgct_project_geom_grad")
        return out

    # ---- learned preconditioner
    CNN_PARAMS = 42849

    def cnn_set_weights(self, flat):
        w = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        check(mgct_cnn_set_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),  # noqa: F821
              "mgct_cnn_set_weights")

    def cnn_get_weights(self) -> np.ndarray:
        w = np.zeros(self.CNN_PARAMS, dtype=np.float32)
        check(mgct_cnn_get_weights(self.handle, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),  # noqa: F821
              "mgct_cnn_get_weights")
        return w

    def cnn_forward(self, u, out=None):
        import torch
        nz, ny, nx = u.shape
        if out is None:
            out = torch.empty_like(u)
        check(mgct_cnn_forward(self.handle, nx, ny, nz, _ptr(u), _ptr(out), _stream()), "mgct_cnn_forward")  # noqa: F821
        return out

    def cnn_gradients(self, u, target):
        nz, ny, nx = u.shape
        g = np.zeros(self.CNN_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        check(mgct_cnn_gradients(self.handle, nx, ny, nz, _ptr(u), _ptr(target),  # noqa: F821
                                 g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss), _stream()),
              "mgct_cnn_gradients")
        return g, loss.value

    def cnn_backward(self, u, dout):
        """Parameter gradients of sum(dout * f-network output) at input u (device tensors)."""
        nz, ny, nx = u.shape
        g = np.zeros(self.CNN_PARAMS, dtype=np.float32)
        check(mgct_cnn_backward(self.handle, nx, ny, nz, _ptr(u), _ptr(dout),  # noqa: F821
                                g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream()), "mgct_cnn_backward")
        return g

    def adam_step(self, grads, lr):
        """One Adam step of the context's weights with the given gradients (host array)."""
        g = np.ascontiguousarray(np.asarray(grads, dtype=np.float32).reshape(-1))
        check(mgct_adam_step(self.handle, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), g.size,  # noqa: F821
                             float(lr), _stream()), "mgct_adam_step")

    def cnn_train_step(self, u, target, lr, want_loss=True):
        nz, ny, nx = u.shape
        loss = ctypes.c_double()
        check(mgct_cnn_train_step(self.handle, nx, ny, nz, _ptr(u), _ptr(target), float(lr),  # noqa: F821
                                  ctypes.byref(loss) if want_loss else None, _stream()), "mgct_cnn_train_step")
        return loss.value if want_loss else None

    def kernel_timing(self, enable: bool, ops=None, levels=None):
        """Enable (clearing the records) or disable kernel timing.  `ops` and
        `levels` (iterables of operation codes and grid indices, default all)
        choose which launches are recorded from now on."""
        om = 0xFFFFFFFF if ops is None else sum(1 << int(o) for o in ops)
        lm = 0xFFFFFFFF if levels is None else sum(1 << int(g) for g in levels)
        check(mgct_kernel_timing_select(self.handle, om, lm), "mgct_kernel_timing_select")  # noqa: F821
        check(mgct_kernel_timing(self.handle, 1 if enable else 0), "mgct_kernel_timing")  # noqa: F821

    def kernel_time(self, op: int, level: int = -1):
        """(total milliseconds, number of launches) of kernel `op` since timing was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        check(mgct_kernel_time(self.handle, op, level, ctypes.byref(ms), ctypes.byref(n)), "mgct_kernel_time")  # noqa: F821
        return ms.value, n.value

    def learned_judge(self):
        """(r0, r1, view_step) of the last learned step's judge: squared
        residual norms before and after the network's refinement, over every
        view_step-th view."""
        r0, r1, k = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        check(mgct_learned_judge(self.handle, ctypes.byref(r0), ctypes.byref(r1), ctypes.byref(k)),  # noqa: F821
              "mgct_learned_judge")
        return r0.value, r1.value, k.value

    def learned_stats(self):
        a, r = ctypes.c_int(), ctypes.c_int()
        check(mgct_learned_stats(self.handle, ctypes.byref(a), ctypes.byref(r)), "mgct_learned_stats")  # noqa: F821
        return a.value, r.value

    def synth_line_integrals(self, phantom, out=None):
        import torch
        e = np.ascontiguousarray(phantom.ellipsoids, dtype=np.float64).reshape(-1, 16)
        b = np.ascontiguousarray(phantom.boxes, dtype=np.float64).reshape(-1, 7)
        if out is None:
            out = torch.empty(self.shapes(0)[1], dtype=torch.float32, device="cuda")
        dp = ctypes.POINTER(ctypes.c_double)
        check(mgct_synth_line_integrals(self.handle, e.ctypes.data_as(dp), e.shape[0], b.ctypes.data_as(dp),  # noqa: F821
                                        b.shape[0], _ptr(out), _stream()), "mgct_synth_line_integrals")
        return out

    def synth_voxelize(self, phantom, ss=4, out=None):
        import torch
        e = np.ascontiguousarray(phantom.ellipsoids, dtype=np.float64).reshape(-1, 16)
        b = np.ascontiguousarray(phantom.boxes, dtype=np.float64).reshape(-1, 7)
        if out is None:
            out = torch.empty(self.shapes(0)[0], dtype=torch.float32, device="cuda")
        dp = ctypes.POINTER(ctypes.c_double)
        check(mgct_synth_voxelize(self.handle, e.ctypes.data_as(dp), e.shape[0], b.ctypes.data_as(dp),  # noqa: F821
                                  b.shape[0], ss, _ptr(out), _stream()), "mgct_synth_voxelize")
        return out

    def multigrid_solve(self, vol, b, levels, n_outer, filt, alphas=None, power_iters=30, power_seed=0,
                        lam=0.0, bilateral=None, coarse_subsets=8, coarse_passes=2, want_hist=True,
                        learned=False, capture_update=None, capture_iterate=None):
        p = mgct_mg_params()
        p.levels = levels
        p.n_outer = n_outer
        p.filter = filt
        for i in range(8):
            p.alpha[i] = 0.0
        if alphas is not None:
            for i, a in enumerate(alphas):
                p.alpha[i] = float(a)
        p.power_iters = power_iters
        p.power_seed = power_seed
        p.lambda_ = lam
        p.bilateral_on = 1 if bilateral else 0
        p.sigma_s, p.sigma_r = bilateral if bilateral else (1.0, 1.0)
        p.coarse_subsets = coarse_subsets
        p.coarse_passes = coarse_passes
        p.learned = 1 if learned else 0
        p.capture_update = capture_update.data_ptr() if capture_update is not None else None
        p.capture_iterate = capture_iterate.data_ptr() if capture_iterate is not None else None
        hist = np.zeros(max(n_outer * levels, 1))
        hp = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_hist else None
        check(mgct_multigrid_solve(self.handle, _ptr(vol), _ptr(b), _dtype_code(b), ctypes.byref(p), hp,  # noqa: F821
                                   _stream()), "mgct_multigrid_solve")
        return hist[: n_outer * levels].reshape(n_outer, levels) if want_hist else None


def residual_diverged(prev: float, cur: float, ratio: float) -> bool:
    """The library's divergence rule (host only): cur not finite, or
    ratio > 0, prev > 0 and cur > ratio * prev."""
    load_library()
    return bool(mgct_residual_diverged(float(prev), float(cur), float(ratio)))  # noqa: F821


def geometry_param_grad(views0, dviews, voxel, dx, dz, tilt_deg) -> np.ndarray:
    """d/d(dx, dz, tilt_deg) from per-view gradients (see mgct.h)."""
    load_library()
    v0 = np.ascontiguousarray(np.asarray(views0, dtype=np.float64).reshape(-1, 12))
    dv = np.ascontiguousarray(np.asarray(dviews, dtype=np.float64).reshape(-1, 12))
    out = np.zeros(3)
    dp = ctypes.POINTER(ctypes.c_double)
    check(mgct_geometry_param_grad(v0.shape[0], v0.ctypes.data_as(dp), dv.ctypes.data_as(dp), float(voxel),  # noqa: F821
                                   float(dx), float(dz), float(tilt_deg), out.ctypes.data_as(dp)),
          "mgct_geometry_param_grad")
    return out


def cnn_flatten(params) -> np.ndarray:
    """[[W1, b1], ..., [W4, b4]] (W as [co][ci][3][3][3]) -> flat FP32 vector in
    the library's order W1 b1 W2 b2 W3 b3 W4 b4."""
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for layer in params for a in layer]).astype(
        np.float32)


def cnn_unflatten(flat):
    shapes = [((16, 1, 3, 3, 3), (16,)), ((32, 16, 3, 3, 3), (32,)), ((32, 32, 3, 3, 3), (32,)), ((1, 32, 3, 3, 3), (1,))]
    out, k = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for ws, bs in shapes:
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append([flat[k:k + nw].reshape(ws), flat[k + nw:k + nw + nb].reshape(bs)])
        k += nw + nb
    return out

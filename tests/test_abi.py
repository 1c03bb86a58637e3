"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/mgct.h, the binding mirrors them, and host-only
calls behave."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2103_10329_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgct.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgct_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mg.LIB_PATH):
        from paper_2103_10329_amd import build
        build.build()
    return mg.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
        assert n in mg.SIGNATURES, n


def test_binding_has_no_undeclared_entry_points(lib):
    assert set(mg.SIGNATURES) == set(_declared())


def test_status_strings(lib):
    for code in range(0, -10, -1):
        s = mg.mgct_status_string(code).decode()
        assert s and s != "unknown status"
    assert mg.mgct_status_string(-99).decode() == "unknown status"


def test_eq5_filter_matches_oracle_taps(lib):
    f = mg.filter_eq5()
    assert f.kind == mg.MGCT_FILTER_STENCIL27
    taps = np.array(f.taps[:]).reshape(3, 3, 3)
    assert np.allclose(taps, oracle.STENCIL27_TAPS, atol=0)


def test_null_arguments_are_rejected(lib):
    assert mg.mgct_create(0, None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_destroy(None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_project(None, 0, None, 0, None, 0, None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_filter_eq5(None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_cnn_backward(None, 32, 1, 1, None, None, None, None) == mg.MGCT_ERR_INVALID_ARG
    assert mg.mgct_adam_step(None, None, 0, 1e-3, None) == mg.MGCT_ERR_INVALID_ARG


def test_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    assert mg.mgct_create(0, ctypes.byref(h)) != mg.MGCT_OK

"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/rmsynth.h declares, and rejects invalid arguments before
touching the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1810_06250_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmsynth.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmsynth_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rs.LIB_PATH):
        pytest.skip("librmsynth.so not built")
    return rs.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rmsynth_plan", "rmsynth_rmsf", "rmsynth_execute", "rmsynth_peaks"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(rs.SIGNATURES) == _declared()


def test_version_and_empty_error(lib):
    assert rs.rmsynth_version().startswith("rmsynth")
    assert isinstance(rs.rmsynth_last_error(), str)


def _plan_rc(lam, w, phi, l0=float("nan")):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = rs.load_library().rmsynth_plan(lam.ctypes.data, w.ctypes.data, lam.size, phi.ctypes.data,
                                        phi.size, l0, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["zero_weights", "negative_weight", "nan_weight", "inf_lambda2",
                                  "nan_phi", "inf_lambda0"])
def test_plan_rejects_invalid_values(lib, case):
    lam = np.linspace(0.1, 0.2, 8)
    w = np.ones(8)
    phi = np.linspace(-10, 10, 5)
    l0 = float("nan")
    if case == "zero_weights":
        w[:] = 0
    elif case == "negative_weight":
        w[2] = -1
    elif case == "nan_weight":
        w[3] = math.nan
    elif case == "inf_lambda2":
        lam[1] = math.inf
    elif case == "nan_phi":
        phi[0] = math.nan
    elif case == "inf_lambda0":
        l0 = math.inf
    rc, h = _plan_rc(lam, w, phi, l0)
    assert rc == rs.rmsynth.RMSYNTH_EINVAL and not h.value
    assert rs.rmsynth_last_error()


def test_plan_rejects_bad_sizes_and_null(lib):
    h = ctypes.c_void_p()
    lam = np.ones(4)
    assert lib.rmsynth_plan(lam.ctypes.data, lam.ctypes.data, 0, lam.ctypes.data, 4,
                            math.nan, ctypes.byref(h)) == rs.rmsynth.RMSYNTH_EINVAL
    assert lib.rmsynth_plan(lam.ctypes.data, lam.ctypes.data, 4, lam.ctypes.data, 0,
                            math.nan, ctypes.byref(h)) == rs.rmsynth.RMSYNTH_EINVAL
    assert lib.rmsynth_plan(None, lam.ctypes.data, 4, lam.ctypes.data, 4,
                            math.nan, ctypes.byref(h)) == rs.rmsynth.RMSYNTH_EINVAL
    assert lib.rmsynth_plan(lam.ctypes.data, lam.ctypes.data, 4, lam.ctypes.data, 4,
                            math.nan, None) == rs.rmsynth.RMSYNTH_EINVAL


def test_calls_reject_null_plan(lib):
    E = rs.rmsynth.RMSYNTH_EINVAL
    assert lib.rmsynth_execute(None, None, None, 1, 0, 0, None, None, None, None, 0, None) == E
    assert lib.rmsynth_peaks(None, None, None, 1, None, None, None, None, None, None) == E
    assert lib.rmsynth_rmsf(None, None, None, None) == E
    b = ctypes.c_size_t()
    assert lib.rmsynth_workspace_size(None, 1, 0, 0, ctypes.byref(b)) == E
    assert lib.rmsynth_plan_info(None, None, None, None, None, None, None) == E
    lib.rmsynth_destroy(None)  # no-op


def test_error_raises_in_binding(lib):
    with pytest.raises(rs.RmsynthError) as ei:
        rs.rmsynth_plan(np.ones(3), np.zeros(3), np.zeros(2))
    assert ei.value.code == rs.rmsynth.RMSYNTH_EINVAL

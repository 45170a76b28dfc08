"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the headers under include/ declare, and rejects invalid arguments before
touching the device."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

import paper_1810_06250_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(rmsynth_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


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


def _mlp_rc(nchan, h1, h2, weights=None, phi_scale=300.0):
    h = ctypes.c_void_p()
    w = None
    if weights is not None:
        w = np.ascontiguousarray(weights, dtype=np.float32)
    rc = rs.load_library().rmsynth_mlp_create(nchan, h1, h2,
                                              None if w is None else w.ctypes.data, phi_scale, 0,
                                              ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("args", [
    (0, 64, 64), (10, 0, 64), (10, 65, 64), (10, 64, 100), (10, 64, 8192),
])
def test_mlp_create_rejects_bad_shapes(lib, args):
    rc, h = _mlp_rc(*args)
    assert rc == rs.RMSYNTH_EINVAL and not h.value
    assert "rmsynth_mlp_create" in rs.rmsynth_last_error()


def test_mlp_create_rejects_bad_weights_and_scale(lib):
    assert _mlp_rc(4, 64, 64, weights=[1, -1, 1, 1])[0] == rs.RMSYNTH_EINVAL
    assert _mlp_rc(4, 64, 64, weights=[1, np.nan, 1, 1])[0] == rs.RMSYNTH_EINVAL
    assert _mlp_rc(4, 64, 64, phi_scale=0.0)[0] == rs.RMSYNTH_EINVAL
    assert _mlp_rc(4, 64, 64, phi_scale=float("inf"))[0] == rs.RMSYNTH_EINVAL


def test_mlp_calls_reject_null_handles(lib):
    n = ctypes.c_int64()
    assert lib.rmsynth_mlp_num_params(None, ctypes.byref(n)) == rs.RMSYNTH_EINVAL
    assert lib.rmsynth_mlp_train_step(None, None, None, 1, None, None, 1e-3, None, None) == rs.RMSYNTH_EINVAL
    assert lib.rmsynth_mlp_infer(None, None, None, 1, None, None, None) == rs.RMSYNTH_EINVAL
    assert lib.rmsynth_gate_execute(None, None, None, None, 1, 0.5, None, None, None, None, None, 0,
                                    None) == rs.RMSYNTH_EINVAL
    b = ctypes.c_size_t()
    assert lib.rmsynth_gate_workspace_size(None, None, 1, ctypes.byref(b)) == rs.RMSYNTH_EINVAL
    lib.rmsynth_mlp_destroy(None)


def test_mlp_load_rejects_missing_and_foreign_files(lib, tmp_path):
    h = ctypes.c_void_p()
    assert lib.rmsynth_mlp_load(str(tmp_path / "none.bin").encode(), ctypes.byref(h)) == rs.RMSYNTH_EINVAL
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTANMLP" + bytes(64))
    assert lib.rmsynth_mlp_load(str(bad).encode(), ctypes.byref(h)) == rs.RMSYNTH_EINVAL
    assert not h.value

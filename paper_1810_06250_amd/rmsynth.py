"""Python binding of librmsynth (argument marshalling only).

The functions named like the C ABI (`rmsynth_plan`, `rmsynth_execute`, ...)
take torch tensors for device buffers and numpy arrays for host arrays, pass
their pointers and torch's current HIP stream, and raise `RmsynthError` on a
non-zero status.  `Plan` is a small convenience wrapper over the same calls.

Every step of the transform runs in the HIP library; if librmsynth.so is
missing this module raises on import of the library, it never falls back.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librmsynth.so")

RMSYNTH_OK = 0
RMSYNTH_EINVAL = -1
RMSYNTH_ENOMEM = -2
RMSYNTH_EHIP = -3
RMSYNTH_EUNSUPPORTED = -4
RMSYNTH_EWORKSPACE = -5

RMSYNTH_LOS_MAJOR = 0
RMSYNTH_FREQ_MAJOR = 1

RMSYNTH_FP32 = 0
RMSYNTH_SPLIT_BF16 = 1
RMSYNTH_SPLIT_FP16 = 2

PRECISIONS = {"fp32": RMSYNTH_FP32, "bf16x3": RMSYNTH_SPLIT_BF16, "fp16x3": RMSYNTH_SPLIT_FP16}
LAYOUTS = {"los": RMSYNTH_LOS_MAJOR, "freq": RMSYNTH_FREQ_MAJOR}

# (name, restype, argtypes) of every exported symbol.
_P, _I32, _I64, _D, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "rmsynth_plan": (ctypes.c_int, [_P, _P, _I32, _P, _I32, _D, ctypes.POINTER(_P)]),
    "rmsynth_plan_info": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "rmsynth_workspace_size": (ctypes.c_int, [_P, _I64, _I32, _I32, ctypes.POINTER(_SZ)]),
    "rmsynth_rmsf": (ctypes.c_int, [_P, _P, _P, _P]),
    "rmsynth_execute": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _P, _P, _SZ, _P]),
    "rmsynth_peaks": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P, _P, _P]),
    "rmsynth_execute_peaks": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P,
                                             _P, _P, _P, _SZ, _P]),
    "rmsynth_execute_peaks_workspace_size": (ctypes.c_int, [_P, _I64, _I32, _I32,
                                                            ctypes.POINTER(_SZ)]),
    "rmsynth_peak_angle": (ctypes.c_int, [_P, _P, _P, _P, _I64, _P, _P]),
    "rmsynth_search": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P,
                                      _SZ, _P]),
    "rmsynth_search_workspace_size": (ctypes.c_int, [_P, _I64, _I32, _I32, ctypes.POINTER(_SZ)]),
    "rmsynth_search_noalloc": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _P, _P, _P, _P, _P, _P,
                                              _P, _P]),
    "rmsynth_search_noalloc_scratch_bytes": (_SZ, []),
    "rmsynth_peak_fit": (ctypes.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "rmsynth_adjoint": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _P, _P, _P, _SZ, _P]),
    "rmsynth_adjoint_workspace_size": (ctypes.c_int, [_P, _I64, _I32, ctypes.POINTER(_SZ)]),
    "rmsynth_execute_nufft": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P]),
    "rmsynth_rmclean": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.c_float, ctypes.c_float, _I32, _D,
                                       _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "rmsynth_rmclean_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(_SZ)]),
    "rmsynth_destroy": (None, [_P]),
    "rmsynth_last_error": (ctypes.c_char_p, []),
    "rmsynth_version": (ctypes.c_char_p, []),
    # learned gate (include/rmsynth_mlp.h)
    "rmsynth_mlp_create": (ctypes.c_int, [_I32, _I32, _I32, _P, ctypes.c_float, ctypes.c_uint64,
                                          ctypes.POINTER(_P)]),
    "rmsynth_mlp_num_params": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "rmsynth_mlp_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                        ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_float)]),
    "rmsynth_mlp_get_params": (ctypes.c_int, [_P, _P]),
    "rmsynth_mlp_set_params": (ctypes.c_int, [_P, _P]),
    "rmsynth_mlp_grad": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P, _P, _P]),
    "rmsynth_mlp_train_step": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, ctypes.c_float, _P, _P]),
    "rmsynth_mlp_infer": (ctypes.c_int, [_P, _P, _P, _I64, _P, _P, _P]),
    "rmsynth_gate_workspace_size": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(_SZ)]),
    "rmsynth_gate_execute": (ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.c_float, _P, _P, _P, _P,
                                            _P, _SZ, _P]),
    "rmsynth_gate_search": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I32, ctypes.c_float, _P, _P, _P, _P,
                                           _P, _SZ, _P]),
    "rmsynth_gate_search_workspace_size": (ctypes.c_int, [_P, _P, _I64, _I32, ctypes.POINTER(_SZ)]),
    "rmsynth_train_workspace_size": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_SZ)]),
    "rmsynth_synth_training": (ctypes.c_int, [_P, _P, ctypes.c_uint64, _I64, _I64, _P, _P, _P, _P,
                                              _P, _P, _P, _SZ, _P]),
    "rmsynth_mlp_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "rmsynth_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_P)]),
    "rmsynth_mlp_destroy": (None, [_P]),
}

_lib = None


class RmsynthError(RuntimeError):
    def __init__(self, call: str, code: int, msg: str):
        super().__init__(f"{call} failed with status {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH):
    """Load librmsynth.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_1810_06250_amd.build` (HIP, gfx950)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(call: str, rc: int):
    if rc != RMSYNTH_OK:
        raise RmsynthError(call, rc, load_library().rmsynth_last_error().decode())


def _stream(stream=None):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, name, dtype=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _host64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# Size checks.  The C ABI takes bare pointers and cannot see how large a
# buffer is, so every wrapper below checks the tensors it is given against
# the sizes it passes (LOS, channels, phi) before anything is launched, and
# raises ValueError on a mismatch.
def _need(t, name, n):
    """t (may be None) holds at least n elements."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, {n} needed")


def _need_rows(t, name, nrows, ncols):
    """t holds nrows x ncols elements; a 2-D t has rows of exactly ncols."""
    if t is None:
        return
    if t.dim() == 2 and t.shape[1] != ncols:
        raise ValueError(f"{name} has rows of {t.shape[1]}, expected {ncols}")
    _need(t, name, nrows * ncols)


def _need_cube(Q, U, nlos, nchan, layout):
    """Q, U hold a cube of nlos LOS x nchan channels in the given layout."""
    if Q is not None and U is not None and tuple(Q.shape) != tuple(U.shape):
        raise ValueError(f"Q {tuple(Q.shape)} and U {tuple(U.shape)} differ in shape")
    for t, name in ((Q, "Q"), (U, "U")):
        if t is None:
            continue
        if layout == RMSYNTH_FREQ_MAJOR:
            # channel planes of exactly nlos values (the plane stride is nlos)
            if t.dim() == 2 and tuple(t.shape) != (nchan, nlos):
                raise ValueError(f"{name} is {tuple(t.shape)}, frequency-major needs ({nchan}, {nlos})")
            _need(t, name, nlos * nchan)
        elif layout == RMSYNTH_LOS_MAJOR:
            _need_rows(t, name, nlos, nchan)


def _need_bytes(ws, nbytes):
    if ws is not None and ws.numel() * ws.element_size() < nbytes:
        raise ValueError(f"workspace has {ws.numel() * ws.element_size()} bytes, "
                         f"workspace_bytes says {nbytes}")


def _plan_dims(plan):
    info = rmsynth_plan_info(plan)
    return info["nchan"], info["nphi"]


# ------------------------------------------------------------------ C-ABI names
def rmsynth_plan(lambda2, weights, phi, lambda0_sq: float = float("nan")) -> ctypes.c_void_p:
    lam, w, ph = _host64(lambda2), _host64(weights), _host64(phi)
    if lam.shape != w.shape:
        raise ValueError("lambda2 and weights must have the same length")
    h = ctypes.c_void_p()
    _check("rmsynth_plan", load_library().rmsynth_plan(
        lam.ctypes.data_as(_P), w.ctypes.data_as(_P), lam.size, ph.ctypes.data_as(_P), ph.size,
        float(lambda0_sq), ctypes.byref(h)))
    return h


def rmsynth_plan_info(plan) -> dict:
    K, l0, fw, pm = (ctypes.c_double() for _ in range(4))
    nc, nphi = ctypes.c_int32(), ctypes.c_int32()
    _check("rmsynth_plan_info", load_library().rmsynth_plan_info(
        plan, ctypes.byref(K), ctypes.byref(l0), ctypes.byref(fw), ctypes.byref(pm),
        ctypes.byref(nc), ctypes.byref(nphi)))
    return dict(K=K.value, lambda0_sq=l0.value, fwhm_est=fw.value, phimax_est=pm.value,
                nchan=nc.value, nphi=nphi.value)


def rmsynth_workspace_size(plan, nlos: int, layout: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_workspace_size", load_library().rmsynth_workspace_size(
        plan, int(nlos), int(layout), int(precision), ctypes.byref(b)))
    return b.value


def rmsynth_rmsf(plan, R_re, R_im, stream=None):
    import torch
    _, nphi = _plan_dims(plan)
    _need(R_re, "R_re", nphi)
    _need(R_im, "R_im", nphi)
    _check("rmsynth_rmsf", load_library().rmsynth_rmsf(
        plan, _dev(R_re, "R_re", torch.float32), _dev(R_im, "R_im", torch.float32), _stream(stream)))


def rmsynth_execute(plan, Q, U, nlos: int, layout: int, precision: int, Fq, Fu, Fabs=None,
                    workspace=None, workspace_bytes: int = 0, stream=None):
    import torch
    nchan, nphi = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, layout)
    for t, name in ((Fq, "Fq"), (Fu, "Fu"), (Fabs, "Fabs")):
        _need_rows(t, name, int(nlos), nphi)
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_execute", load_library().rmsynth_execute(
        plan, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), int(layout), int(precision),
        _dev(Fq, "Fq", f32), _dev(Fu, "Fu", f32), _dev(Fabs, "Fabs", f32),
        _dev(workspace, "workspace"), int(workspace_bytes), _stream(stream)))


def rmsynth_peaks(plan, Fq, Fu, nlos: int, idx, phi_pk=None, amp=None, q_pk=None, u_pk=None,
                  stream=None):
    import torch
    _, nphi = _plan_dims(plan)
    _need_rows(Fq, "Fq", int(nlos), nphi)
    _need_rows(Fu, "Fu", int(nlos), nphi)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (q_pk, "q_pk"), (u_pk, "u_pk")):
        _need(t, name, int(nlos))
    f32 = torch.float32
    _check("rmsynth_peaks", load_library().rmsynth_peaks(
        plan, _dev(Fq, "Fq", f32), _dev(Fu, "Fu", f32), int(nlos), _dev(idx, "idx", torch.int32),
        _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32), _dev(q_pk, "q_pk", f32),
        _dev(u_pk, "u_pk", f32), _stream(stream)))


def rmsynth_peak_angle(plan, phi_pk, q_pk, u_pk, nlos: int, chi0, stream=None):
    import torch
    for t, name in ((phi_pk, "phi_pk"), (q_pk, "q_pk"), (u_pk, "u_pk"), (chi0, "chi0")):
        _need(t, name, int(nlos))
    f32 = torch.float32
    _check("rmsynth_peak_angle", load_library().rmsynth_peak_angle(
        plan, _dev(phi_pk, "phi_pk", f32), _dev(q_pk, "q_pk", f32), _dev(u_pk, "u_pk", f32),
        int(nlos), _dev(chi0, "chi0", f32), _stream(stream)))


def rmsynth_execute_peaks_workspace_size(plan, nlos: int, layout: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_execute_peaks_workspace_size", load_library().rmsynth_execute_peaks_workspace_size(
        plan, int(nlos), int(layout), int(precision), ctypes.byref(b)))
    return b.value


def rmsynth_execute_peaks(plan, Q, U, nlos: int, layout: int, precision: int, Fq, Fu, Fabs, idx,
                          phi_pk=None, amp=None, q_pk=None, u_pk=None, workspace=None,
                          workspace_bytes: int = 0, stream=None):
    import torch
    nchan, nphi = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, layout)
    for t, name in ((Fq, "Fq"), (Fu, "Fu"), (Fabs, "Fabs")):
        _need_rows(t, name, int(nlos), nphi)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (q_pk, "q_pk"), (u_pk, "u_pk")):
        _need(t, name, int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_execute_peaks", load_library().rmsynth_execute_peaks(
        plan, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), int(layout), int(precision),
        _dev(Fq, "Fq", f32), _dev(Fu, "Fu", f32), _dev(Fabs, "Fabs", f32),
        _dev(idx, "idx", torch.int32), _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32),
        _dev(q_pk, "q_pk", f32), _dev(u_pk, "u_pk", f32), _dev(workspace, "workspace"),
        int(workspace_bytes), _stream(stream)))


def rmsynth_search_workspace_size(plan, nlos: int, layout: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_search_workspace_size", load_library().rmsynth_search_workspace_size(
        plan, int(nlos), int(layout), int(precision), ctypes.byref(b)))
    return b.value


def rmsynth_search(plan, Q, U, nlos: int, layout: int, precision: int, idx, phi_pk=None, amp=None,
                   q_pk=None, u_pk=None, phi_fit=None, amp_fit=None, workspace=None,
                   workspace_bytes: int = 0, stream=None):
    import torch
    nchan, _ = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, layout)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (q_pk, "q_pk"), (u_pk, "u_pk"),
                    (phi_fit, "phi_fit"), (amp_fit, "amp_fit")):
        _need(t, name, int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_search", load_library().rmsynth_search(
        plan, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), int(layout), int(precision),
        _dev(idx, "idx", torch.int32), _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32),
        _dev(q_pk, "q_pk", f32), _dev(u_pk, "u_pk", f32), _dev(phi_fit, "phi_fit", f32),
        _dev(amp_fit, "amp_fit", f32), _dev(workspace, "workspace"), int(workspace_bytes),
        _stream(stream)))


def rmsynth_search_noalloc(plan, Q, U, nlos: int, layout: int, precision: int, idx, phi_pk=None,
                           amp=None, q_pk=None, u_pk=None, phi_fit=None, amp_fit=None,
                           stream=None):
    import torch
    nchan, _ = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, layout)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (q_pk, "q_pk"), (u_pk, "u_pk"),
                    (phi_fit, "phi_fit"), (amp_fit, "amp_fit")):
        _need(t, name, int(nlos))
    f32 = torch.float32
    _check("rmsynth_search_noalloc", load_library().rmsynth_search_noalloc(
        plan, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), int(layout), int(precision),
        _dev(idx, "idx", torch.int32), _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32),
        _dev(q_pk, "q_pk", f32), _dev(u_pk, "u_pk", f32), _dev(phi_fit, "phi_fit", f32),
        _dev(amp_fit, "amp_fit", f32), _stream(stream)))


def rmsynth_search_noalloc_scratch_bytes() -> int:
    return int(load_library().rmsynth_search_noalloc_scratch_bytes())


def rmsynth_peak_fit(plan, Fq, Fu, idx, nlos: int, phi_fit=None, amp_fit=None, stream=None):
    import torch
    _, nphi = _plan_dims(plan)
    _need_rows(Fq, "Fq", int(nlos), nphi)
    _need_rows(Fu, "Fu", int(nlos), nphi)
    for t, name in ((idx, "idx"), (phi_fit, "phi_fit"), (amp_fit, "amp_fit")):
        _need(t, name, int(nlos))
    f32 = torch.float32
    _check("rmsynth_peak_fit", load_library().rmsynth_peak_fit(
        plan, _dev(Fq, "Fq", f32), _dev(Fu, "Fu", f32), _dev(idx, "idx", torch.int32), int(nlos),
        _dev(phi_fit, "phi_fit", f32), _dev(amp_fit, "amp_fit", f32), _stream(stream)))


def rmsynth_adjoint_workspace_size(plan, nlos: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_adjoint_workspace_size", load_library().rmsynth_adjoint_workspace_size(
        plan, int(nlos), int(precision), ctypes.byref(b)))
    return b.value


def rmsynth_adjoint(plan, Cq, Cu, nlos: int, precision: int, Pq, Pu, workspace=None,
                    workspace_bytes: int = 0, stream=None):
    import torch
    nchan, nphi = _plan_dims(plan)
    if Cq is not None and Cu is not None and tuple(Cq.shape) != tuple(Cu.shape):
        raise ValueError(f"Cq {tuple(Cq.shape)} and Cu {tuple(Cu.shape)} differ in shape")
    for t, name in ((Cq, "Cq"), (Cu, "Cu")):
        _need_rows(t, name, int(nlos), nphi)
    for t, name in ((Pq, "Pq"), (Pu, "Pu")):
        _need_rows(t, name, int(nlos), nchan)
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_adjoint", load_library().rmsynth_adjoint(
        plan, _dev(Cq, "Cq", f32), _dev(Cu, "Cu", f32), int(nlos), int(precision),
        _dev(Pq, "Pq", f32), _dev(Pu, "Pu", f32), _dev(workspace, "workspace"),
        int(workspace_bytes), _stream(stream)))


def rmsynth_execute_nufft(plan, Q, U, nlos: int, Fq, Fu, Fabs=None, stream=None):
    import torch
    nchan, nphi = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, RMSYNTH_LOS_MAJOR)
    for t, name in ((Fq, "Fq"), (Fu, "Fu"), (Fabs, "Fabs")):
        _need_rows(t, name, int(nlos), nphi)
    f32 = torch.float32
    _check("rmsynth_execute_nufft", load_library().rmsynth_execute_nufft(
        plan, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), _dev(Fq, "Fq", f32),
        _dev(Fu, "Fu", f32), _dev(Fabs, "Fabs", f32), _stream(stream)))


def rmsynth_rmclean_workspace_size(plan) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_rmclean_workspace_size", load_library().rmsynth_rmclean_workspace_size(
        plan, ctypes.byref(b)))
    return b.value


def rmsynth_rmclean(plan, Fq, Fu, nlos: int, gain: float, cutoff: float, max_iter: int,
                    fwhm: float, rq, ru, cq, cu, Rq=None, Ru=None, niter=None, workspace=None,
                    workspace_bytes: int = 0, stream=None):
    import torch
    _, nphi = _plan_dims(plan)
    for t, name in ((Fq, "Fq"), (Fu, "Fu"), (rq, "rq"), (ru, "ru"), (cq, "cq"), (cu, "cu"),
                    (Rq, "Rq"), (Ru, "Ru")):
        _need_rows(t, name, int(nlos), nphi)
    _need(niter, "niter", int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_rmclean", load_library().rmsynth_rmclean(
        plan, _dev(Fq, "Fq", f32), _dev(Fu, "Fu", f32), int(nlos), float(gain), float(cutoff),
        int(max_iter), float(fwhm), _dev(rq, "rq", f32), _dev(ru, "ru", f32), _dev(cq, "cq", f32),
        _dev(cu, "cu", f32), _dev(Rq, "Rq", f32), _dev(Ru, "Ru", f32),
        _dev(niter, "niter", torch.int32), _dev(workspace, "workspace"), int(workspace_bytes),
        _stream(stream)))


def rmsynth_destroy(plan):
    if plan:
        load_library().rmsynth_destroy(plan)


def rmsynth_last_error() -> str:
    return load_library().rmsynth_last_error().decode()


def rmsynth_version() -> str:
    return load_library().rmsynth_version().decode()


# ------------------------------------------------------------------ learned gate
def rmsynth_mlp_create(nchan: int, h1: int, h2: int, weights=None, phi_scale: float = 300.0,
                       seed: int = 0) -> ctypes.c_void_p:
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
    if w is not None and w.size != nchan:
        raise ValueError("weights must have nchan entries")
    h = ctypes.c_void_p()
    _check("rmsynth_mlp_create", load_library().rmsynth_mlp_create(
        int(nchan), int(h1), int(h2), None if w is None else w.ctypes.data_as(_P),
        float(phi_scale), int(seed) & (2**64 - 1), ctypes.byref(h)))
    return h


def rmsynth_mlp_info(mlp) -> dict:
    nc, h1, h2 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ps = ctypes.c_float()
    _check("rmsynth_mlp_info", load_library().rmsynth_mlp_info(
        mlp, ctypes.byref(nc), ctypes.byref(h1), ctypes.byref(h2), ctypes.byref(ps)))
    return dict(nchan=nc.value, h1=h1.value, h2=h2.value, phi_scale=ps.value)


def _need_batch(mlp, Q, U, batch, phi_label, det_label):
    nchan = rmsynth_mlp_info(mlp)["nchan"]
    _need_cube(Q, U, batch, nchan, RMSYNTH_LOS_MAJOR)
    _need(phi_label, "phi_label", batch)
    _need(det_label, "det_label", batch)


def rmsynth_mlp_num_params(mlp) -> int:
    n = ctypes.c_int64()
    _check("rmsynth_mlp_num_params", load_library().rmsynth_mlp_num_params(mlp, ctypes.byref(n)))
    return n.value


def rmsynth_mlp_get_params(mlp) -> np.ndarray:
    out = np.empty(rmsynth_mlp_num_params(mlp), dtype=np.float32)
    _check("rmsynth_mlp_get_params", load_library().rmsynth_mlp_get_params(
        mlp, out.ctypes.data_as(_P)))
    return out


def rmsynth_mlp_set_params(mlp, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if p.size != rmsynth_mlp_num_params(mlp):
        raise ValueError("parameter vector has the wrong length")
    _check("rmsynth_mlp_set_params", load_library().rmsynth_mlp_set_params(
        mlp, p.ctypes.data_as(_P)))


def rmsynth_mlp_grad(mlp, Q, U, batch: int, phi_label, det_label, grad, loss=None, stream=None):
    import torch
    _need_batch(mlp, Q, U, int(batch), phi_label, det_label)
    _need(grad, "grad", rmsynth_mlp_num_params(mlp))
    _need(loss, "loss", 1)
    f32 = torch.float32
    _check("rmsynth_mlp_grad", load_library().rmsynth_mlp_grad(
        mlp, _dev(Q, "Q", f32), _dev(U, "U", f32), int(batch), _dev(phi_label, "phi_label", f32),
        _dev(det_label, "det_label", f32), _dev(grad, "grad", f32), _dev(loss, "loss", f32),
        _stream(stream)))


def rmsynth_mlp_train_step(mlp, Q, U, batch: int, phi_label, det_label, lr: float, loss=None,
                           stream=None):
    import torch
    _need_batch(mlp, Q, U, int(batch), phi_label, det_label)
    _need(loss, "loss", 1)
    f32 = torch.float32
    _check("rmsynth_mlp_train_step", load_library().rmsynth_mlp_train_step(
        mlp, _dev(Q, "Q", f32), _dev(U, "U", f32), int(batch), _dev(phi_label, "phi_label", f32),
        _dev(det_label, "det_label", f32), float(lr), _dev(loss, "loss", f32), _stream(stream)))


def rmsynth_mlp_infer(mlp, Q, U, nlos: int, phi_hat, score, stream=None):
    import torch
    nchan = rmsynth_mlp_info(mlp)["nchan"]
    _need_cube(Q, U, int(nlos), nchan, RMSYNTH_LOS_MAJOR)
    _need(phi_hat, "phi_hat", int(nlos))
    _need(score, "score", int(nlos))
    f32 = torch.float32
    _check("rmsynth_mlp_infer", load_library().rmsynth_mlp_infer(
        mlp, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), _dev(phi_hat, "phi_hat", f32),
        _dev(score, "score", f32), _stream(stream)))


def rmsynth_gate_workspace_size(plan, mlp, nlos: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_gate_workspace_size", load_library().rmsynth_gate_workspace_size(
        plan, mlp, int(nlos), ctypes.byref(b)))
    return b.value


def rmsynth_gate_execute(plan, mlp, Q, U, nlos: int, tau: float, idx, phi_pk, amp, gated,
                         workspace, workspace_bytes: int, stream=None):
    import torch
    nchan, _ = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, RMSYNTH_LOS_MAJOR)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (gated, "gated")):
        _need(t, name, int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32, i32 = torch.float32, torch.int32
    _check("rmsynth_gate_execute", load_library().rmsynth_gate_execute(
        plan, mlp, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), float(tau),
        _dev(idx, "idx", i32), _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32),
        _dev(gated, "gated", i32), _dev(workspace, "workspace"), int(workspace_bytes),
        _stream(stream)))


def rmsynth_gate_search_workspace_size(plan, mlp, nlos: int, precision: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_gate_search_workspace_size", load_library().rmsynth_gate_search_workspace_size(
        plan, mlp, int(nlos), int(precision), ctypes.byref(b)))
    return b.value


def rmsynth_gate_search(plan, mlp, Q, U, nlos: int, precision: int, tau: float, idx, phi_pk, amp,
                        gated, workspace, workspace_bytes: int, stream=None):
    import torch
    nchan, _ = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, RMSYNTH_LOS_MAJOR)
    for t, name in ((idx, "idx"), (phi_pk, "phi_pk"), (amp, "amp"), (gated, "gated")):
        _need(t, name, int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32, i32 = torch.float32, torch.int32
    _check("rmsynth_gate_search", load_library().rmsynth_gate_search(
        plan, mlp, _dev(Q, "Q", f32), _dev(U, "U", f32), int(nlos), int(precision), float(tau),
        _dev(idx, "idx", i32), _dev(phi_pk, "phi_pk", f32), _dev(amp, "amp", f32),
        _dev(gated, "gated", i32), _dev(workspace, "workspace"), int(workspace_bytes),
        _stream(stream)))


class TrainSpec(ctypes.Structure):
    """rmsynth_train_spec: class mix, parameter ranges, noise and detection threshold."""
    _fields_ = [(n, ctypes.c_double) for n in (
        "frac_noise", "frac_thin1", "frac_thin2", "p0_lo", "p0_hi", "phi_lo", "phi_hi",
        "w_lo", "w_hi", "sigma", "det_threshold")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


def rmsynth_train_workspace_size(plan, nlos: int) -> int:
    b = ctypes.c_size_t()
    _check("rmsynth_train_workspace_size", load_library().rmsynth_train_workspace_size(
        plan, int(nlos), ctypes.byref(b)))
    return b.value


def rmsynth_synth_training(plan, spec: TrainSpec, seed: int, first_los: int, nlos: int, Q, U,
                           phi_label=None, det_label=None, cls=None, truth=None, workspace=None,
                           workspace_bytes: int = 0, stream=None):
    import torch
    nchan, _ = _plan_dims(plan)
    _need_cube(Q, U, int(nlos), nchan, RMSYNTH_LOS_MAJOR)
    for t, name in ((phi_label, "phi_label"), (det_label, "det_label"), (cls, "cls")):
        _need(t, name, int(nlos))
    _need(truth, "truth", 4 * int(nlos))
    _need_bytes(workspace, int(workspace_bytes))
    f32 = torch.float32
    _check("rmsynth_synth_training", load_library().rmsynth_synth_training(
        plan, ctypes.byref(spec), int(seed) & (2**64 - 1), int(first_los), int(nlos),
        _dev(Q, "Q", f32), _dev(U, "U", f32), _dev(phi_label, "phi_label", f32),
        _dev(det_label, "det_label", f32), _dev(cls, "cls", torch.int32), _dev(truth, "truth", f32),
        _dev(workspace, "workspace"), int(workspace_bytes), _stream(stream)))


def rmsynth_mlp_save(mlp, path: str):
    _check("rmsynth_mlp_save", load_library().rmsynth_mlp_save(mlp, os.fsencode(path)))


def rmsynth_mlp_load(path: str) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check("rmsynth_mlp_load", load_library().rmsynth_mlp_load(os.fsencode(path), ctypes.byref(h)))
    return h


def rmsynth_mlp_destroy(mlp):
    if mlp:
        load_library().rmsynth_mlp_destroy(mlp)


# ------------------------------------------------------------------ convenience
class Plan:
    """Owns an rmsynth plan; allocates outputs with torch on the current device."""

    def __init__(self, lambda2, weights, phi, lambda0_sq: float = float("nan")):
        self.handle = rmsynth_plan(lambda2, weights, phi, lambda0_sq)
        self.info = rmsynth_plan_info(self.handle)
        self.nchan, self.nphi = self.info["nchan"], self.info["nphi"]

    def close(self):
        if self.handle:
            rmsynth_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rmsf(self):
        import torch
        re = torch.empty(self.nphi, dtype=torch.float32, device="cuda")
        im = torch.empty_like(re)
        rmsynth_rmsf(self.handle, re, im)
        return re, im

    def execute(self, Q, U, layout: int = RMSYNTH_LOS_MAJOR, precision: int = RMSYNTH_FP32,
                want_abs: bool = False, out: Optional[tuple] = None):
        import torch
        nlos = Q.shape[0] if layout == RMSYNTH_LOS_MAJOR else Q.shape[1]
        if out is None:
            Fq = torch.empty((nlos, self.nphi), dtype=torch.float32, device=Q.device)
            Fu = torch.empty_like(Fq)
            Fa = torch.empty_like(Fq) if want_abs else None
        else:
            Fq, Fu, Fa = out
        ws_bytes = rmsynth_workspace_size(self.handle, nlos, layout, precision)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=Q.device) if ws_bytes else None
        rmsynth_execute(self.handle, Q, U, nlos, layout, precision, Fq, Fu, Fa, ws, ws_bytes)
        return Fq, Fu, Fa

    def execute_peaks(self, Q, U, layout: int = RMSYNTH_LOS_MAJOR, precision: int = RMSYNTH_FP32,
                      want_abs: bool = False):
        """Transform and peaks in one call (rmsynth_execute_peaks)."""
        import torch
        nlos = Q.shape[0] if layout == RMSYNTH_LOS_MAJOR else Q.shape[1]
        dev = Q.device
        Fq = torch.empty((nlos, self.nphi), dtype=torch.float32, device=dev)
        Fu = torch.empty_like(Fq)
        Fa = torch.empty_like(Fq) if want_abs else None
        out = dict(idx=torch.empty(nlos, dtype=torch.int32, device=dev),
                   phi_pk=torch.empty(nlos, dtype=torch.float32, device=dev),
                   amp=torch.empty(nlos, dtype=torch.float32, device=dev),
                   q_pk=torch.empty(nlos, dtype=torch.float32, device=dev),
                   u_pk=torch.empty(nlos, dtype=torch.float32, device=dev))
        nb = rmsynth_execute_peaks_workspace_size(self.handle, nlos, layout, precision)
        ws = torch.empty(nb, dtype=torch.uint8, device=dev) if nb else None
        rmsynth_execute_peaks(self.handle, Q, U, nlos, layout, precision, Fq, Fu, Fa, out["idx"],
                              out["phi_pk"], out["amp"], out["q_pk"], out["u_pk"], ws, nb)
        return Fq, Fu, Fa, out

    def search(self, Q, U, layout: int = RMSYNTH_LOS_MAJOR, precision: int = RMSYNTH_FP32,
               workspace_bytes: Optional[int] = None):
        """Peaks and sub-grid peaks without storing F (rmsynth_search).  A
        workspace_bytes below the whole call's need runs it in LOS batches."""
        import torch
        nlos = Q.shape[0] if layout == RMSYNTH_LOS_MAJOR else Q.shape[1]
        dev = Q.device
        out = dict(idx=torch.empty(nlos, dtype=torch.int32, device=dev))
        for k in ("phi_pk", "amp", "q_pk", "u_pk", "phi_fit", "amp_fit"):
            out[k] = torch.empty(nlos, dtype=torch.float32, device=dev)
        nb = rmsynth_search_workspace_size(self.handle, nlos, layout, precision)
        if workspace_bytes is not None:
            nb = int(workspace_bytes)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        rmsynth_search(self.handle, Q, U, nlos, layout, precision, out["idx"], out["phi_pk"],
                       out["amp"], out["q_pk"], out["u_pk"], out["phi_fit"], out["amp_fit"], ws, nb)
        return out

    def adjoint(self, Cq, Cu, precision: int = RMSYNTH_FP32):
        """Spectra [nlos][nchan] of Faraday-depth components [nlos][nphi]
        (rmsynth_adjoint)."""
        import torch
        nlos = Cq.shape[0]
        Pq = torch.empty((nlos, self.nchan), dtype=torch.float32, device=Cq.device)
        Pu = torch.empty_like(Pq)
        nb = rmsynth_adjoint_workspace_size(self.handle, nlos, precision)
        ws = torch.empty(nb, dtype=torch.uint8, device=Cq.device) if nb else None
        rmsynth_adjoint(self.handle, Cq, Cu, nlos, precision, Pq, Pu, ws, nb)
        return Pq, Pu

    def execute_nufft(self, Q, U, want_abs: bool = False):
        """F by the non-uniform FFT (rmsynth_execute_nufft), LOS-major input."""
        import torch
        nlos = Q.shape[0]
        Fq = torch.empty((nlos, self.nphi), dtype=torch.float32, device=Q.device)
        Fu = torch.empty_like(Fq)
        Fa = torch.empty_like(Fq) if want_abs else None
        rmsynth_execute_nufft(self.handle, Q, U, nlos, Fq, Fu, Fa)
        return Fq, Fu, Fa

    def rmclean(self, Fq, Fu, gain: float, cutoff: float, max_iter: int,
                fwhm: float = float("nan"), restore: bool = True):
        """RM-CLEAN of the spectra (rmsynth_rmclean): dict of resid (rq, ru),
        components (cq, cu), restored (Rq, Ru) and niter."""
        import torch
        nlos = Fq.shape[0]
        o = {k: torch.empty_like(Fq) for k in ("rq", "ru", "cq", "cu")}
        if restore:
            o["Rq"], o["Ru"] = torch.empty_like(Fq), torch.empty_like(Fq)
        o["niter"] = torch.empty(nlos, dtype=torch.int32, device=Fq.device)
        nb = rmsynth_rmclean_workspace_size(self.handle)
        ws = torch.empty(nb, dtype=torch.uint8, device=Fq.device)
        rmsynth_rmclean(self.handle, Fq, Fu, nlos, gain, cutoff, max_iter, fwhm, o["rq"], o["ru"],
                        o["cq"], o["cu"], o.get("Rq"), o.get("Ru"), o["niter"], ws, nb)
        return o

    def peak_fit(self, Fq, Fu, idx):
        """Sub-grid peak (rmsynth_peak_fit) around the indices idx."""
        import torch
        nlos = Fq.shape[0]
        pf = torch.empty(nlos, dtype=torch.float32, device=Fq.device)
        af = torch.empty_like(pf)
        rmsynth_peak_fit(self.handle, Fq, Fu, idx, nlos, pf, af)
        return pf, af

    def peak_angle(self, pk):
        """Polarization angle at each LOS's peak referred to lambda^2 = 0
        (rmsynth_peak_angle) from a peaks dict (phi_pk, q_pk, u_pk)."""
        import torch
        chi = torch.empty_like(pk["phi_pk"])
        rmsynth_peak_angle(self.handle, pk["phi_pk"], pk["q_pk"], pk["u_pk"], chi.shape[0], chi)
        return chi

    def peaks(self, Fq, Fu):
        import torch
        nlos = Fq.shape[0]
        dev = Fq.device
        out = dict(idx=torch.empty(nlos, dtype=torch.int32, device=dev),
                   phi_pk=torch.empty(nlos, dtype=torch.float32, device=dev),
                   amp=torch.empty(nlos, dtype=torch.float32, device=dev),
                   q_pk=torch.empty(nlos, dtype=torch.float32, device=dev),
                   u_pk=torch.empty(nlos, dtype=torch.float32, device=dev))
        rmsynth_peaks(self.handle, Fq, Fu, nlos, out["idx"], out["phi_pk"], out["amp"],
                      out["q_pk"], out["u_pk"])
        return out


def make_training_data(plan: "Plan", spec: TrainSpec, seed: int, first_los: int, nlos: int,
                       labels: bool = True, extras: bool = False, device="cuda"):
    """Allocate and fill one batch of training data with rmsynth_synth_training."""
    import torch
    out = dict(Q=torch.empty((nlos, plan.nchan), dtype=torch.float32, device=device),
               U=torch.empty((nlos, plan.nchan), dtype=torch.float32, device=device))
    ws, nb = None, 0
    if labels:
        out["phi_label"] = torch.empty(nlos, dtype=torch.float32, device=device)
        out["det_label"] = torch.empty(nlos, dtype=torch.float32, device=device)
        nb = rmsynth_train_workspace_size(plan.handle, nlos)
        ws = torch.empty(nb, dtype=torch.uint8, device=device)
    if extras:
        out["cls"] = torch.empty(nlos, dtype=torch.int32, device=device)
        out["truth"] = torch.empty((nlos, 4), dtype=torch.float32, device=device)
    rmsynth_synth_training(plan.handle, spec, seed, first_los, nlos, out["Q"], out["U"],
                           out.get("phi_label"), out.get("det_label"), out.get("cls"),
                           out.get("truth"), ws, nb)
    return out


class Mlp:
    """Owns a gate network (rmsynth_mlp_*); outputs are torch tensors."""

    def __init__(self, nchan: int = 0, h1: int = 256, h2: int = 256, weights=None,
                 phi_scale: float = 300.0, seed: int = 0, handle=None):
        self.handle = handle if handle is not None else rmsynth_mlp_create(
            nchan, h1, h2, weights, phi_scale, seed)
        self.nparams = rmsynth_mlp_num_params(self.handle)

    @classmethod
    def load(cls, path: str) -> "Mlp":
        return cls(handle=rmsynth_mlp_load(path))

    def save(self, path: str):
        rmsynth_mlp_save(self.handle, path)

    def close(self):
        if self.handle:
            rmsynth_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        return rmsynth_mlp_get_params(self.handle)

    def set_params(self, params):
        rmsynth_mlp_set_params(self.handle, params)

    def grad(self, Q, U, phi_label, det_label):
        import torch
        g = torch.empty(self.nparams, dtype=torch.float32, device=Q.device)
        loss = torch.empty(1, dtype=torch.float32, device=Q.device)
        rmsynth_mlp_grad(self.handle, Q, U, Q.shape[0], phi_label, det_label, g, loss)
        return g, loss

    def train_step(self, Q, U, phi_label, det_label, lr: float, loss=None):
        rmsynth_mlp_train_step(self.handle, Q, U, Q.shape[0], phi_label, det_label, lr, loss)

    def infer(self, Q, U):
        import torch
        n = Q.shape[0]
        phi_hat = torch.empty(n, dtype=torch.float32, device=Q.device)
        score = torch.empty_like(phi_hat)
        rmsynth_mlp_infer(self.handle, Q, U, n, phi_hat, score)
        return phi_hat, score

    def gate(self, plan: "Plan", Q, U, tau: float, precision: Optional[int] = None):
        """Gated peak search: rmsynth_gate_execute (FP32 transform + peaks on
        the gated LOS), or with a precision rmsynth_gate_search (the
        peaks-only search in that precision)."""
        import torch
        n = Q.shape[0]
        dev = Q.device
        out = dict(idx=torch.empty(n, dtype=torch.int32, device=dev),
                   phi_pk=torch.empty(n, dtype=torch.float32, device=dev),
                   amp=torch.empty(n, dtype=torch.float32, device=dev),
                   gated=torch.empty(n, dtype=torch.int32, device=dev))
        if precision is None:
            nb = rmsynth_gate_workspace_size(plan.handle, self.handle, n)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            rmsynth_gate_execute(plan.handle, self.handle, Q, U, n, tau, out["idx"], out["phi_pk"],
                                 out["amp"], out["gated"], ws, nb)
        else:
            nb = rmsynth_gate_search_workspace_size(plan.handle, self.handle, n, precision)
            ws = torch.empty(nb, dtype=torch.uint8, device=dev)
            rmsynth_gate_search(plan.handle, self.handle, Q, U, n, precision, tau, out["idx"],
                                out["phi_pk"], out["amp"], out["gated"], ws, nb)
        return out

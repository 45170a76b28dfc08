"""Python face of the FP64 oracle (test infrastructure only).

* `fdf`, `rmsf`, `peaks`, `plan`, `plan_info`, `cost_flop` call the plain C
  triple loop in rmsynth_oracle.c (built by `build()` with gcc, no fast-math).
* `peak_angle` is the polarization angle at the peak (eq. (14)), numpy FP64.
* `fdf_bruteforce` is a second, independent evaluation of eq. (11) as a
  numpy complex128 matrix product, for tiny cubes.
* `per_los_error` and `peak_agreement` are the comparison rules used by the
  parity tests and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmsynth_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the C oracle into oracle/liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        P = ctypes.c_void_p
        lib.oracle_plan.argtypes = [P, P, i32, d, P, P]
        lib.oracle_plan.restype = ctypes.c_int
        lib.oracle_plan_info.argtypes = [P, P, i32, P, P]
        lib.oracle_plan_info.restype = ctypes.c_int
        lib.oracle_cost_flop.argtypes = [i64, i64, i64]
        lib.oracle_cost_flop.restype = d
        lib.oracle_fdf.argtypes = [P, P, i64, i32, P, P, i32, P, i32, d, d, i32, P, P]
        lib.oracle_fdf.restype = ctypes.c_int
        lib.oracle_rmsf.argtypes = [P, P, i32, P, i32, d, d, P, P]
        lib.oracle_rmsf.restype = ctypes.c_int
        lib.oracle_peaks.argtypes = [P, P, i64, i32, P, P, P, P, P, P, P]
        lib.oracle_peaks.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = [P, P, i64, P, i32, P, i32, d, P, P]
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def plan(lambda2, w, lambda0_sq=float("nan")):
    """K (eq. 13) and lambda0^2 (weighted mean of lambda^2 unless given)."""
    lam, w = _f64(lambda2), _f64(w)
    K, l0 = ctypes.c_double(), ctypes.c_double()
    rc = _load().oracle_plan(_ptr(lam), _ptr(w), lam.size, float(lambda0_sq),
                             ctypes.byref(K), ctypes.byref(l0))
    if rc != 0:
        raise ValueError("oracle_plan: invalid channel set")
    return K.value, l0.value


def plan_info(lambda2, w):
    """(2 sqrt3 / Delta lambda^2, sqrt3 / delta lambda^2), eqs. (20)-(21)."""
    lam, w = _f64(lambda2), _f64(w)
    a, b = ctypes.c_double(), ctypes.c_double()
    if _load().oracle_plan_info(_ptr(lam), _ptr(w), lam.size, ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("oracle_plan_info failed")
    return a.value, b.value


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().oracle_threads())


def cost_flop(nlos, nchan, nphi) -> float:
    return _load().oracle_cost_flop(int(nlos), int(nchan), int(nphi))


def fdf(Q, U, lambda2, w, phi, layout=0, lambda0_sq=float("nan"), table_mode=True):
    """F = Fq + i Fu, each float64 [nlos][nphi], of a Q/U cube (float64 copy of
    whatever precision the caller holds).  layout 0: Q[l][j]; 1: Q[j][l]."""
    Q, U = _f64(Q), _f64(U)
    lam, w, phi = _f64(lambda2), _f64(w), _f64(phi)
    nchan, nphi = lam.size, phi.size
    if Q.ndim != 2:
        raise ValueError("Q must be 2-D")
    nlos = Q.shape[0] if layout == 0 else Q.shape[1]
    K, l0 = plan(lam, w, lambda0_sq)
    Fq = np.empty((nlos, nphi), dtype=np.float64)
    Fu = np.empty((nlos, nphi), dtype=np.float64)
    rc = _load().oracle_fdf(_ptr(Q), _ptr(U), nlos, int(layout), _ptr(lam), _ptr(w), nchan,
                            _ptr(phi), nphi, K, l0, 1 if table_mode else 0, _ptr(Fq), _ptr(Fu))
    if rc != 0:
        raise ValueError("oracle_fdf failed")
    return Fq, Fu


def adjoint(Cre, Cim, lambda2, w, phi, lambda0_sq=float("nan")):
    """Spectrum of grid components C [nlos][nphi] (eq. (4) as a sum over the
    grid, referred to lambda0^2): P = Pq + i Pu, each float64 [nlos][nchan].
    w only fixes lambda0^2 (the weighted mean, unless lambda0_sq is given)."""
    Cre, Cim = _f64(Cre), _f64(Cim)
    lam, w, phi = _f64(lambda2), _f64(w), _f64(phi)
    if Cre.ndim != 2 or Cre.shape[1] != phi.size or Cim.shape != Cre.shape:
        raise ValueError("C must be [nlos][nphi]")
    _, l0 = plan(lam, w, lambda0_sq)
    nlos = Cre.shape[0]
    Pq = np.empty((nlos, lam.size))
    Pu = np.empty((nlos, lam.size))
    if _load().oracle_adjoint(_ptr(Cre), _ptr(Cim), nlos, _ptr(phi), phi.size, _ptr(lam), lam.size,
                              l0, _ptr(Pq), _ptr(Pu)):
        raise ValueError("oracle_adjoint failed")
    return Pq, Pu


def rmsf(lambda2, w, phi, lambda0_sq=float("nan")):
    """R(phi) of eq. (12) as (re, im) float64 [nphi]."""
    lam, w, phi = _f64(lambda2), _f64(w), _f64(phi)
    K, l0 = plan(lam, w, lambda0_sq)
    re = np.empty(phi.size)
    im = np.empty(phi.size)
    if _load().oracle_rmsf(_ptr(lam), _ptr(w), lam.size, _ptr(phi), phi.size, K, l0,
                           _ptr(re), _ptr(im)):
        raise ValueError("oracle_rmsf failed")
    return re, im


def peaks(Fq, Fu, phi):
    """Per-LOS peak of |F|: dict(idx, phi_pk, amp, q_pk, u_pk, margin)."""
    Fq, Fu, phi = _f64(Fq), _f64(Fu), _f64(phi)
    nlos, nphi = Fq.shape
    out = dict(idx=np.empty(nlos, np.int32), phi_pk=np.empty(nlos), amp=np.empty(nlos),
               q_pk=np.empty(nlos), u_pk=np.empty(nlos), margin=np.empty(nlos))
    if _load().oracle_peaks(_ptr(Fq), _ptr(Fu), nlos, nphi, _ptr(phi), _ptr(out["idx"]),
                            _ptr(out["phi_pk"]), _ptr(out["amp"]), _ptr(out["q_pk"]),
                            _ptr(out["u_pk"]), _ptr(out["margin"])):
        raise ValueError("oracle_peaks failed")
    return out


def peak_angle(q_pk, u_pk, phi_pk, lambda0_sq):
    """Polarization angle of the peak referred to lambda^2 = 0 (eq. (14)):
    half the phase of F(phi_pk) after undoing the exp(2i phi_pk lambda0^2)
    that the lambda0^2 term of eq. (11) puts on it, in [0, pi) radians; NaN
    where an input is not finite.  FP64, numpy."""
    q, u, ph = _f64(q_pk), _f64(u_pk), _f64(phi_pk)
    z = (q + 1j * u) * np.exp(-2j * ph * float(lambda0_sq))
    chi = np.mod(0.5 * np.angle(z), np.pi)
    bad = ~(np.isfinite(q) & np.isfinite(u) & np.isfinite(ph))
    return np.where(bad, np.nan, chi)


def peak_fit(amp_prev, amp_pk, amp_next, phi_prev, phi_pk, phi_next):
    """Sub-grid peak of |F| (the paper gives phi_peak on the grid only; this
    refinement is an extension): the vertex of the parabola through the three
    points (phi_prev, amp_prev), (phi_pk, amp_pk), (phi_next, amp_next),
    elementwise in FP64.  Returns (phi_fit, amp_fit).  Where a neighbour is
    missing (NaN: the peak sits at an end of the grid) or the parabola does not
    open downwards, the grid values are returned unchanged; where amp_pk or
    phi_pk is NaN (no peak), both results are NaN."""
    y0, y1, y2 = (np.asarray(a, np.float64) for a in (amp_prev, amp_pk, amp_next))
    x0, x1, x2 = (np.asarray(a, np.float64) for a in (phi_prev, phi_pk, phi_next))
    with np.errstate(divide="ignore", invalid="ignore"):
        d0, d2 = x0 - x1, x2 - x1          # d0 < 0 < d2
        # y(t) = y1 + B t + A t^2 through (d0, y0), (0, y1), (d2, y2), t = phi - phi_pk
        s0, s2 = (y0 - y1) / d0, (y2 - y1) / d2
        A = (s0 - s2) / (d0 - d2)
        B = s0 - A * d0
        t = -B / (2.0 * A)
        top = y1 - B * B / (4.0 * A)
    ok = np.isfinite(y0) & np.isfinite(y2) & np.isfinite(t) & (A < 0)
    phi_fit = np.where(ok, x1 + t, x1)
    amp_fit = np.where(ok, top, y1)
    nopk = ~(np.isfinite(y1) & np.isfinite(x1))
    return np.where(nopk, np.nan, phi_fit), np.where(nopk, np.nan, amp_fit)


def peak_fit_from_spectra(Fq, Fu, phi, idx):
    """peak_fit around the index idx[l] of each LOS of F (any precision):
    |F| at idx - 1, idx, idx + 1 as FP64 hypot, neighbours past the grid ends
    missing; idx = -1 gives NaN."""
    Fq, Fu, phi = _f64(Fq), _f64(Fu), _f64(phi)
    idx = np.asarray(idx, np.int64)
    nlos, nphi = Fq.shape
    rows = np.arange(nlos)
    have = idx >= 0
    k = np.where(have, idx, 0)

    def amp_at(kk):
        inside = have & (kk >= 0) & (kk < nphi)
        kc = np.clip(kk, 0, nphi - 1)
        return np.where(inside, np.hypot(Fq[rows, kc], Fu[rows, kc]), np.nan), \
            np.where(inside, phi[kc], np.nan)

    (y0, x0), (y1, x1), (y2, x2) = amp_at(k - 1), amp_at(k), amp_at(k + 1)
    return peak_fit(y0, y1, y2, x0, x1, x2)


def fdf_bruteforce(Q, U, lambda2, w, phi, lambda0_sq=None):
    """eq. (11) as one complex128 matrix product (LOS-major input, tiny cubes)."""
    lam, w, phi = _f64(lambda2), _f64(w), _f64(phi)
    keep = w > 0
    K = 1.0 / w.sum()
    l0 = K * np.sum(w * lam) if lambda0_sq is None else lambda0_sq
    P = (_f64(Q) + 1j * _f64(U))[:, keep] * w[keep]
    E = np.exp(-2j * np.outer(lam[keep] - l0, phi))
    F = K * (P @ E)
    return F.real.copy(), F.imag.copy()


def incoherent_scale(Q, U, w, layout=0):
    """K sqrt(sum_j w_j^2 |P_j|^2) per LOS: the typical |F| of a spectrum whose
    channels add with random phases (finite channels of non-zero weight)."""
    Q, U, w = _f64(Q), _f64(U), _f64(w)
    if layout == 1:
        Q, U = Q.T, U.T
    keep = w > 0
    P2 = Q[:, keep] ** 2 + U[:, keep] ** 2
    P2 = np.where(np.isfinite(P2), P2, 0.0)
    return np.sqrt(P2 @ (w[keep] ** 2)) / w.sum()


def per_los_error(Fq_gpu, Fu_gpu, Fq_ref, Fu_ref, floor=None):
    """e_l = max_k |F_gpu - F_ref| / max(max_k |F_ref|, floor_l) per LOS.
    `floor` (e.g. `incoherent_scale`) only matters on grids so short that
    max_k |F_ref| can fall below the LOS's typical |F|."""
    dq = np.asarray(Fq_gpu, np.float64) - Fq_ref
    du = np.asarray(Fu_gpu, np.float64) - Fu_ref
    num = np.sqrt(dq * dq + du * du).max(axis=1)
    den = np.hypot(Fq_ref, Fu_ref).max(axis=1)
    if floor is not None:
        den = np.maximum(den, floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, num / den, num)


def peak_agreement(idx_gpu, Fq_ref, Fu_ref, ref_peaks, margin_thr=2e-5):
    """Peak-index rule.  Where the oracle's margin exceeds `margin_thr` the
    index must match exactly; elsewhere any index whose oracle |F| is within
    (1 - margin_thr) of the maximum is accepted.  A LOS the oracle flags
    (non-finite |F|, idx -1) must be flagged (-1) by the GPU too, and a LOS the
    oracle does not flag must not be.  Returns
    (n_unambiguous, n_mismatch_unambiguous, n_invalid_other), the last counting
    ambiguous LOS with an unacceptable index and flag disagreements."""
    idx_gpu = np.asarray(idx_gpu).astype(np.int64)
    flagged = np.asarray(ref_peaks["idx"]) < 0
    unamb = (ref_peaks["margin"] > margin_thr) & ~flagged
    mism = int(np.sum(unamb & (idx_gpu != ref_peaks["idx"])))
    bad = int(np.sum(flagged & (idx_gpu != -1)))
    amb = np.flatnonzero(~unamb & ~flagged)
    for l in amb:
        k = idx_gpu[l]
        if k < 0 or k >= Fq_ref.shape[1]:
            bad += 1
            continue
        a = np.hypot(Fq_ref[l, k], Fu_ref[l, k])
        if a < (1.0 - margin_thr) * ref_peaks["amp"][l]:
            bad += 1
    return int(unamb.sum()), mism, bad
